"""Mixed precision against the FP64 device path (needs an MI355X).

Workload: D=6, chi=72, d=4, W=8, V=1, dt=0.05, Neel start, 100 Trotter steps
(t = 5); every 10 steps 10 CTMRG iterations (cold the first time, warm after)
and a readout, the same schedule in every precision.  The FP32 path runs the
CTMRG contractions in FP32 on MFMA; the BF16 paths round their operands to
BF16 and accumulate in FP32 (tensors stored in FP32, the readout
contraction in FP32), split BF16 with two BF16 terms per operand; all keep
the simple update, the projector SVDs and the normalisations in FP64.  The
imbalance must stay within 1e-3 of the FP64 path at every observation for
FP32 and split BF16; plain BF16 is held to its measured level.  The errors
are printed (pytest -s).
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


_S64 = {}


# plain BF16 operands (8-bit mantissa) miss the 1e-3 bar at this size
# (measured ~1e-2 early in the evolution); split BF16 (two BF16 terms per
# operand) and FP32 must meet it
@pytest.mark.parametrize("dtype,bar", [("fp32", 1e-3), ("bf16x3", 1e-3), ("bf16", 3e-2)])
def test_low_precision_imbalance_within_1e3_of_fp64(dtype, bar):
    if "s" not in _S64:
        _S64["s"] = _series("fp64")
    s64, s32 = _S64["s"], _series(dtype)
    err = np.array([abs(a["imbalance"] - b["imbalance"]) for a, b in zip(s64, s32)])
    nerr = np.array([np.max(np.abs(a["n"] - b["n"])) for a, b in zip(s64, s32)])
    for a, e, ne in zip(s64, err, nerr):
        print(f"{dtype} t={a['t']:.2f} I64={a['imbalance']:.8f} |dI|={e:.2e} max|dn|={ne:.2e}")
    assert np.all(np.isfinite(err))
    assert err.max() <= bar, err
