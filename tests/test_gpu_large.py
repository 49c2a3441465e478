"""The largest shapes of the serving workload on the device (needs an
MI355X): D = 8, chi = 128 (n = chi D^2 = 8192, the 8192 x 8192 enlarged
corner; subspace blocks of 170 columns in FP64 and 136 in FP32, the wide
Cholesky and Jacobi variants) and D = 7, chi = 98.  No oracle reaches these
sizes in seconds (a cut there is an 8192^2 complex SVD), so the checks are
the properties that hold at any size: particle-number conservation (the
four occupations sum to 2, the physical one-site matrices are diagonal),
occupations in [0, 1], entropies in [0, ln 2], finite corner spectra of
unit norm, and the FP32 / split-BF16 paths within 1e-3 of FP64 (the same
schedule).  Parity of the wide (k > 128) kernels with the oracle is in
tests/test_gpu_path_goldens.py (D = 3, chi = 108)."""
import numpy as np
import pytest

P = pytest.importorskip("paper_1910_11359_amd")

pytestmark = pytest.mark.gpu


def _run(D, chi, dtype, steps=3, iters=3):
    print(f"large: D={D} chi={chi} {dtype}", flush=True)
    st = P.State(P.make_config(D, chi, J=1.0, V=1.0, W=8.0, dt=0.05, dtype=dtype))
    st.trotter_step(steps)
    st.ctmrg(0.0, iters, True)
    o = st.observe()
    cs = st.corner_spectra()
    st.close()
    return o, cs


@pytest.mark.parametrize("D,chi", [(7, 98), (8, 128)])
def test_largest_serving_shapes(D, chi):
    o64, cs = _run(D, chi, "fp64")
    assert abs(o64["sum_n"] - 2.0) < 1e-9 and o64["max_offdiag"] < 1e-9
    assert np.all(o64["n"] >= -1e-12) and np.all(o64["n"] <= 1 + 1e-12)
    assert np.all(o64["renyi1"] >= -1e-12) and np.all(o64["renyi1"] <= np.log(2) + 1e-12)
    assert np.all(np.isfinite(cs)) and np.allclose(np.linalg.norm(cs, axis=1), 1.0, atol=1e-12)
    for dtype in ("fp32", "bf16x3"):
        o, _ = _run(D, chi, dtype)
        print(f"  {dtype}: |dI| = {abs(o['imbalance'] - o64['imbalance']):.2e}", flush=True)
        assert abs(o["imbalance"] - o64["imbalance"]) < 1e-3
        assert abs(o["sum_n"] - 2.0) < 1e-5
