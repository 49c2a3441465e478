"""Mixed precision against the FP64 device path (needs an MI355X).

Workload: D=6, chi=72, d=4, W=8, V=1, dt=0.05, Neel start, 100 Trotter steps
(t = 5); every 10 steps 10 CTMRG iterations (cold the first time, warm after)
and a readout, the same schedule in both precisions.  The FP32 path runs the
CTMRG contractions in FP32 on MFMA and keeps the simple update, the projector
SVDs and the normalisations in FP64; its imbalance must stay within 1e-3 of
the FP64 path at every observation.  The errors are printed (pytest -s).
"""
import numpy as np
import pytest

P = pytest.importorskip("paper_1910_11359_amd")

pytestmark = pytest.mark.gpu


def _series(dtype, n_steps=100, every=10, iters=10):
    st = P.State(P.make_config(6, 72, J=1.0, V=1.0, W=8.0, dt=0.05, dtype=dtype))
    out, first = [], True
    for _ in range(n_steps // every):
        st.trotter_step(every)
        st.ctmrg(0.0, iters, first)
        first = False
        out.append(st.observe())
    st.close()
    return out


def test_fp32_imbalance_within_1e3_of_fp64():
    s64, s32 = _series("fp64"), _series("fp32")
    err = np.array([abs(a["imbalance"] - b["imbalance"]) for a, b in zip(s64, s32)])
    nerr = np.array([np.max(np.abs(a["n"] - b["n"])) for a, b in zip(s64, s32)])
    for a, e, ne in zip(s64, err, nerr):
        print(f"t={a['t']:.2f} I64={a['imbalance']:.8f} |dI|={e:.2e} max|dn|={ne:.2e}")
    assert np.all(np.isfinite(err))
    assert err.max() <= 1e-3, err
