"""Free-fermion Néel dynamics on the device vs the dense exact oracle, through
the C ABI (needs an MI355X).

Tolerance: 1e-12 absolute on the sublattice occupations (FP64 throughout;
the Chebyshev series is cut at |J_k| < 1e-18, so the error per interval is
rounding, ~1e-15 times the number of terms).  Inputs: seeded fields from
synthetic.ff_fields.
"""
import numpy as np
import pytest
from scipy.special import j0

import synthetic
from oracle import freefermion as off

P = pytest.importorskip("paper_1910_11359_amd")

pytestmark = pytest.mark.gpu


def _times(dt, n_times):
    return dt * np.arange(1, n_times + 1)


@pytest.mark.parametrize("L,pbc,kind,h,n_real,dt,n_times,seed", [
    (1, False, "continuous", 3.0, 2, 0.3, 4, 1),      # single site
    (2, False, "continuous", 0.0, 1, 0.25, 12, 2),    # clean plaquette
    (3, True, "continuous", 4.0, 3, 0.2, 10, 3),      # odd, periodic
    (5, False, "discrete3", 10.0, 3, 0.1, 20, 4),     # odd, open, spin-1 levels
    (8, True, "continuous", 10.0, 2, 0.1, 30, 5),
    (10, False, "discrete3", 100.0, 2, 0.1, 50, 6),   # strong field: ~40 terms per interval
    (7, False, "continuous", 100.0, 2, 1.5, 4, 7),    # a*dt > 60: split intervals
    (17, True, "continuous", 4.0, 1, 0.2, 8, 8),      # 289 sites: two per thread (ragged)
])
def test_neel_dynamics_vs_oracle(L, pbc, kind, h, n_real, dt, n_times, seed):
    eps = synthetic.ff_fields(L, n_real, h, kind, seed)
    ne, no = P.ff_neel_dynamics(L, eps, n_times, dt, tau=0.5, pbc=pbc)
    t = _times(dt, n_times)
    for r in range(n_real):
        oe, oo = off.neel_dynamics(L, pbc, 0.5, eps[r], t)
        assert np.max(np.abs(ne[r] - oe)) < 1e-12, (r, np.max(np.abs(ne[r] - oe)))
        assert np.max(np.abs(no[r] - oo)) < 1e-12, r


def test_clean_torus_closed_form_on_device():
    L, tau = 28, 0.5
    dt, nt = 0.25, 12
    ne, no = P.ff_neel_dynamics(L, np.zeros((1, L * L)), nt, dt, tau=tau, pbc=True)
    t = _times(dt, nt)
    assert np.max(np.abs((ne[0] - no[0]) - j0(4 * tau * t) ** 2)) < 1e-12


def test_full_size_sampled_and_invariants():
    """The benchmark workload's shape (L = 40, open, continuous h = 10, dt = 0.1,
    50 intervals) on 3 realizations: every output conserves the particle
    number, two realizations match the oracle at 5 sampled times, and a
    repeat run is bitwise identical."""
    cfg = synthetic.ff_headline()
    L, nt, dt = cfg["L"], cfg["n_times"], cfg["dt"]
    eps = synthetic.ff_fields(L, 3, cfg["h"], cfg["kind"], 20191025)
    ne, no = P.ff_neel_dynamics(L, eps, nt, dt, tau=cfg["tau"], pbc=cfg["pbc"])
    M = (L * L + 1) // 2
    Mo = L * L - M
    assert np.max(np.abs(ne * M + no * Mo - M)) < 1e-9
    ne2, no2 = P.ff_neel_dynamics(L, eps, nt, dt, tau=cfg["tau"], pbc=cfg["pbc"])
    assert np.array_equal(ne, ne2) and np.array_equal(no, no2)
    idx = [9, 19, 29, 39, 49]
    for r in range(2):
        oe, oo = off.neel_dynamics(L, cfg["pbc"], cfg["tau"], eps[r], _times(dt, nt)[idx])
        assert np.max(np.abs(ne[r, idx] - oe)) < 1e-12
        assert np.max(np.abs(no[r, idx] - oo)) < 1e-12


def test_invalid_arguments_raise():
    with pytest.raises(P.IpepsError) as e:
        P.ff_neel_dynamics(2, np.zeros((1, 4)), 3, 0.1, pbc=True)
    assert e.value.code == -1
    with pytest.raises(P.IpepsError):
        P.ff_neel_dynamics(4, np.zeros((1, 16)), 3, -0.1)
