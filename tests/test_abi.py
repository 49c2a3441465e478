"""Host-side checks of the C ABI (no GPU needed, no device compute).

* the gfx950 library loads and exports every function include/ipeps.h
  declares;
* the footprint query (pure host arithmetic) is consistent and rejects
  invalid configurations;
* error strings, defaults, and argument validation without a device.
"""
import ctypes
import os
import re

import numpy as np
import pytest

import paper_1910_11359_amd as P
from paper_1910_11359_amd import native

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_functions():
    names = set()
    for fn in os.listdir(os.path.join(ROOT, "include")):
        if not fn.endswith(".h"):
            continue
        text = open(os.path.join(ROOT, "include", fn)).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        text = re.sub(r"typedef[^;]*;", "", text)
        for m in re.finditer(r"\b([A-Za-z_]\w*)\s*\(", text):
            name = m.group(1)
            if name.startswith(("ipeps_", "solve_", "ctmrg_", "ff_")) and name not in ("ipeps_alloc_fn", "ipeps_free_fn"):
                names.add(name)
    return names


def test_library_exports_every_declared_symbol():
    lib = native.load()
    declared = _declared_functions()
    assert len(declared) >= 15
    for name in sorted(declared):
        assert hasattr(lib, name), name
    assert set(native.EXPORTS) <= declared


def test_config_defaults_and_layout():
    c = P.make_config(4, 32)
    assert (c.D, c.chi, c.d_A, c.trotter_order, c.dtype) == (4, 32, 2, 2, 0)
    assert list(c.layer_w) == [0.25] * 4 and list(c.layer_J) == [1.0] * 4
    assert ctypes.sizeof(native.Obs) == 8 * 21 + 8  # 21 doubles + an int padded to 8


def test_footprint_monotone_and_validation():
    fp = lambda **kw: P.footprint_bytes(P.make_config(**kw))
    a = fp(D=4, chi=32)
    b = fp(D=4, chi=48)
    c = fp(D=6, chi=72)
    assert 0 < a < b < c
    assert fp(D=6, chi=72, dtype="fp32") < c
    assert fp(D=4, chi=8) == 0          # chi < D^2
    assert fp(D=9, chi=81) == 0         # D > 8
    assert fp(D=2, chi=8, dt=-0.1) == 0
    assert fp(D=2, chi=8, d_A=3) > 0    # d_A = 1..5 are accepted
    assert fp(D=2, chi=8, d_A=6) == 0   # d = 2 d_A <= 10
    assert fp(D=5, chi=25, d_A=5) > 0   # simple update d min(D^3, dD) = 500 <= 512
    assert fp(D=6, chi=36, d_A=5) == 0  # 600 > 512
    # cut matrices: formed (n = chi D^2 <= 1024 by default) or factored; the
    # formed path holds F, G and N, the factored one only k-column blocks
    assert fp(D=4, chi=32, flags=P.FLAG_FACTORED_CUTS) < a
    assert fp(D=6, chi=72, flags=P.FLAG_FORMED_CUTS) > c
    assert fp(D=4, chi=32, flags=P.FLAG_FORMED_CUTS) == a
    assert fp(D=6, chi=72, flags=P.FLAG_FACTORED_CUTS) == c
    assert fp(D=4, chi=32, flags=P.FLAG_FACTORED_CUTS | P.FLAG_FORMED_CUTS) == 0
    assert fp(D=4, chi=32, flags=8) == 0  # unknown flag


def test_strerror():
    lib = native.load()
    assert lib.ipeps_strerror(0) == b"ok"
    assert b"converge" in lib.ipeps_strerror(-5)
    assert lib.ipeps_strerror(-99) == b"unknown error"


def test_init_rejects_bad_config_before_touching_the_device():
    with pytest.raises(P.IpepsError) as e:
        P.State(P.make_config(D=3, chi=4))
    assert e.value.code == native.IPEPS_EINVAL


def test_ff_bessel_coefficients_match_scipy():
    # host copy of the routine behind the free-fermion propagator
    from scipy.special import jv
    k = np.arange(161)
    for x in (0.0, 1e-3, 0.3, 0.499, 0.5, 1.0, 7.5, 30.0, 60.0):
        got = P.ff_bessel_j(x, 160)
        ref = jv(k, x)
        assert np.max(np.abs(got - ref)) < 2e-15, x


def test_ff_rejects_bad_arguments_without_device():
    lib = native.load()
    bad = [(0, 0, 0.5, 0.1, 1, 1), (46, 0, 0.5, 0.1, 1, 1), (2, 1, 0.5, 0.1, 1, 1), (4, 2, 0.5, 0.1, 1, 1),
           (4, 0, 0.5, 0.0, 1, 1), (4, 0, float("nan"), 0.1, 1, 1), (4, 0, 0.5, 0.1, -1, 1),
           (4, 0, 0.5, 0.1, 1, 70000), (4, 0, 0.5, 0.1, 1, 1)]
    for i, (L, pbc, tau, dt, nt, nr) in enumerate(bad):
        # the last case has valid sizes but NULL buffers
        assert lib.ff_neel_dynamics(L, pbc, tau, dt, nt, nr, None, None, None, None) == native.IPEPS_EINVAL, i
    # nothing to do: OK without touching the device
    assert lib.ff_neel_dynamics(4, 0, 0.5, 0.1, 0, 3, None, None, None, None) == native.IPEPS_OK
    assert lib.ff_neel_dynamics(4, 0, 0.5, 0.1, 5, 0, None, None, None, None) == native.IPEPS_OK


def test_ff_spectrum_rejects_bad_arguments_without_device():
    """Argument checks of ff_spectrum_ipr run before any device work."""
    lib = native.load()
    bad = [(0, 0, 0.5, 2), (41, 0, 0.5, 2), (2, 1, 0.5, 2), (4, 2, 0.5, 2), (4, 0, float("nan"), 2),
           (4, 0, 0.5, -1), (4, 0, 0.5, 70000), (4, 0, 0.5, 3)]  # last: NULL buffers with work
    for i, (L, pbc, tau, nr) in enumerate(bad):
        assert lib.ff_spectrum_ipr(L, pbc, tau, nr, None, None, None, None, None, None) == native.IPEPS_EINVAL, i
    assert lib.ff_spectrum_ipr(4, 0, 0.5, 0, None, None, None, None, None, None) == native.IPEPS_OK
