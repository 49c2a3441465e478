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


# ------------------------------------------------------------ spectrum, IPR
def _check_spectrum(L, pbc, eps, tau=0.5):
    """Device energies, IPRs and bins against the oracle for every realization.
    Energies to 1e-10 of the Gershgorin scale G.  IPRs where the level
    spacing d exceeds 1e-6 G (degenerate levels have no unique eigenvectors),
    to 1e-10 + 4 m / d, m the mixing the solver's stopping rule allows between
    two levels: L <= 16 (Jacobi SVD of h + 2G I, every pair of columns with
    norms up to 3G orthogonal to 4 n eps relative) m = (4 n eps)(3G); L > 16
    (block Jacobi, off-diagonal part below 1e-13 of the Frobenius norm, which
    is at most sqrt(n) 3G) m = 1e-13 sqrt(n) 3G; the IPR moves by at most 4
    times the mixing.  The bins exactly as the oracle bins the device's own
    energies."""
    E, I, B, K = P.ff_spectrum_ipr(L, eps, tau, pbc)
    n = L * L
    for r in range(eps.shape[0]):
        G = np.max(np.abs(eps[r])) + 4 * abs(tau)
        Eo, Io = off.spectrum_ipr(L, pbc, tau, eps[r])
        assert np.all(np.diff(E[r]) >= 0)
        np.testing.assert_allclose(E[r], Eo, atol=1e-10 * max(G, 1.0), rtol=0)
        gap = np.full(n, np.inf)
        if n > 1:
            d = np.diff(Eo)
            gap[:-1] = np.minimum(gap[:-1], d)
            gap[1:] = np.minimum(gap[1:], d)
        ok = gap > 1e-6 * max(G, 1.0)
        mix = (4 * n * 1.11e-16 if L <= 16 else 1e-13 * np.sqrt(n)) * 3 * max(G, 1.0)
        tol = 1e-10 + 4 * mix / gap[ok]
        assert np.all(np.abs(I[r][ok] - Io[ok]) <= tol), np.max(np.abs(I[r][ok] - Io[ok]) / tol)
        assert np.all(I[r] <= 1 + 1e-12) and np.all(I[r] >= 1.0 / n - 1e-12)
        sums, counts = off.cumulative_ipr(E[r], I[r])
        np.testing.assert_array_equal(K[r], counts)
        np.testing.assert_allclose(B[r], sums, atol=1e-13, rtol=0)
        assert K[r].sum() == n


@pytest.mark.parametrize("L,pbc,kind,h,n_real,seed", [
    (1, False, "continuous", 3.0, 2, 11),
    (2, False, "continuous", 1.0, 2, 12),
    (3, True, "continuous", 4.0, 3, 13),
    (5, False, "discrete3", 10.0, 3, 14),
    (8, True, "continuous", 4.0, 2, 15),
    (10, False, "discrete3", 100.0, 3, 16),
    (10, False, "continuous", 100.0, 3, 17),
    (12, False, "discrete2", 10.0, 2, 18),
    # block Jacobi (L > 16): n = 289 padded to 320, 400, 1600
    (17, False, "continuous", 4.0, 2, 22),
    (20, True, "discrete3", 100.0, 2, 23),
    (20, False, "continuous", 10.0, 2, 24),
    (40, False, "continuous", 10.0, 2, 25),
    (40, True, "discrete2", 4.0, 1, 26),
])
def test_spectrum_ipr_vs_oracle(L, pbc, kind, h, n_real, seed):
    print(f"spectrum L={L} pbc={pbc} {kind} h={h} n_real={n_real}", flush=True)
    _check_spectrum(L, pbc, synthetic.ff_fields(L, n_real, h, kind, seed))


def test_spectrum_ipr_limits():
    """No hopping: the energies are the sorted fields and every IPR is 1; the
    clean plaquette's outer states have IPR 1/4 (one per site each)."""
    eps = synthetic.ff_fields(6, 2, 5.0, "continuous", 21)
    E, I, B, K = P.ff_spectrum_ipr(6, eps, 0.0)
    np.testing.assert_allclose(E, np.sort(eps, axis=1), atol=1e-13, rtol=0)
    np.testing.assert_allclose(I, 1.0, atol=1e-13)
    E, I, B, K = P.ff_spectrum_ipr(2, np.zeros((1, 4)), 0.7)
    np.testing.assert_allclose(E[0], [-1.4, 0.0, 0.0, 1.4], atol=1e-13)
    np.testing.assert_allclose(I[0, [0, 3]], 0.25, atol=1e-13)


def test_spectrum_ipr_full_size():
    """The one-workgroup solver's largest lattice, L = 16 (256 x 256), 100
    realizations of continuous disorder h = 10, every realization against
    the oracle; and L = 20 (400 x 400), 100 realizations on the block Jacobi."""
    _check_spectrum(16, False, synthetic.ff_fields(16, 100, 10.0, "continuous", 20191025))
    _check_spectrum(20, False, synthetic.ff_fields(20, 100, 10.0, "continuous", 20191026))
