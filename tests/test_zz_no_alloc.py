"""ff_neel_dynamics_noalloc (fixed device scratch, no allocation) against
ff_neel_dynamics (stream-ordered workspace) through the C ABI: the same
kernels on the same fields, so the outputs must be identical.  Two calls in
a row, the second smaller than the first (the scratch keeps the first call's
contents), and a request larger than the scratch, refused on the host."""
import ctypes as C

import numpy as np
import pytest

import synthetic

P = pytest.importorskip("paper_1910_11359_amd")
from paper_1910_11359_amd import native as N  # noqa: E402

pytestmark = pytest.mark.gpu


def _run(fn, L, eps, n_times, dt):
    n_real = eps.shape[0]
    d_eps = N._DeviceArray(eps.size)
    d_eps.put(eps)
    ne, no = N._DeviceArray(n_real * n_times), N._DeviceArray(n_real * n_times)
    print(f"{fn.__name__}: L={L} n_real={n_real} n_times={n_times}", flush=True)
    fn(L, d_eps.p.value, n_real, ne.p.value, no.p.value, n_times, dt)
    assert N._hip_runtime().hipDeviceSynchronize() == 0
    return ne.get(), no.get()


@pytest.mark.parametrize("seq", [((12, 8, 10, 7), (7, 3, 4, 8))])
def test_noalloc_matches_allocating_entry_point(seq):
    for L, n_real, n_times, seed in seq:
        eps = synthetic.ff_fields(L, n_real, 10.0, "continuous", seed)
        a = _run(N.ff_neel_dynamics_device, L, eps, n_times, 0.2)
        b = _run(N.ff_neel_dynamics_noalloc_device, L, eps, n_times, 0.2)
        assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1]), (L, n_real, n_times)
        assert np.all(np.isfinite(a[0])) and np.all(a[0] > 0)


def test_noalloc_rejects_requests_beyond_the_scratch():
    lib = N.load()
    buf = N._DeviceArray(16)
    # 2 * 65535 * 100 * ceil(45^2 / 2) doubles >> 8 Mi: refused on the host
    # by the size check, before any device work is enqueued
    p = C.c_void_p(buf.p.value)
    rc = lib.ff_neel_dynamics_noalloc(45, 0, 0.5, 0.1, 100, 65535, p, p, p, None)
    assert rc == N.IPEPS_ETOOBIG
