"""Asynchronous readout (ipeps_observe_async / ipeps_observe_result) against
the synchronous one (needs an MI355X).

The asynchronous readout works on a snapshot of the environment taken when it
is started, so it must return exactly what ipeps_observe returns for that
environment (same kernels on the same inputs), even when the next Trotter
step and CTMRG iterations overwrite the live tensors before the result is
collected.  One readout may be pending per state.
"""
import numpy as np
import pytest

P = pytest.importorskip("paper_1910_11359_amd")

pytestmark = pytest.mark.gpu

FIELDS = ("t", "imbalance", "sum_n", "max_offdiag", "ctm_iters", "ctm_delta")
ARRAYS = ("n", "eps", "renyi1", "renyi_half")


def _same(a, b):
    for k in FIELDS:
        assert a[k] == b[k], (k, a[k], b[k])
    for k in ARRAYS:
        np.testing.assert_array_equal(np.asarray(a[k]), np.asarray(b[k]), err_msg=k)


@pytest.mark.parametrize("D,chi,dtype,prelude", [(3, 18, "fp64", 5), (6, 72, "fp32", 20)])
def test_async_readout_equals_sync(D, chi, dtype, prelude):
    st = P.State(P.make_config(D, chi, J=1.0, V=1.0, W=3.0, dt=0.05, dtype=dtype))
    st.trotter_step(prelude)
    st.ctmrg(0.0, 6, True)
    with pytest.raises(P.IpepsError):
        st.observe_result()  # nothing pending
    for _ in range(3):
        ref = st.observe()
        st.observe_async()
        with pytest.raises(P.IpepsError):
            st.observe_async()  # one pending readout per state
        # the next step overwrites C, T, A and eps while the readout may run
        st.trotter_step(1)
        st.ctmrg(0.0, 2, False)
        _same(st.observe_result(), ref)
    # pipelined as in bench.py: start step t's readout, collect it after step t+1
    st.observe_async()
    ref = None
    for _ in range(2):
        st.trotter_step(1)
        st.ctmrg(0.0, 1, False)
        got = st.observe_result()
        if ref is not None:
            _same(got, ref)
        ref = st.observe()
        st.observe_async()
    _same(st.observe_result(), ref)
    st.close()
