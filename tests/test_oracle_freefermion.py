"""Pins of the free-fermion oracle against values fixed independently of it
(closed forms, analytic spectra, invariants).  CPU only."""
import numpy as np
import pytest
from scipy.special import j0

from oracle import freefermion as ff


def test_clean_torus_imbalance_is_j0_squared():
    # infinite clean lattice: orbital amplitudes factorise into J_n(2 tau t)
    # per direction, and sum_n (-1)^n J_n(z)^2 = J_0(2z) gives the imbalance
    # J_0(4 tau t)^2; a 28 x 28 torus matches until the front wraps around
    tau, L = 0.5, 28
    t = np.linspace(0.0, 3.0, 13)
    ne, no = ff.neel_dynamics(L, True, tau, np.zeros(L * L), t)
    assert np.max(np.abs((ne - no) - j0(4 * tau * t) ** 2)) < 1e-12


@pytest.mark.parametrize("tau", [0.5, 1.3])
def test_plaquette_closed_form(tau):
    # open 2 x 2 lattice = ring of four sites with levels -2tau, 0, 0, 2tau;
    # the two filled corners give n_even = (1 + cos^2(2 tau t)) / 2
    t = np.linspace(0.0, 5.0, 21)
    ne, no = ff.neel_dynamics(2, False, tau, np.zeros(4), t)
    c = np.cos(2 * tau * t)
    assert np.max(np.abs(ne - (1 + c * c) / 2)) < 1e-14
    assert np.max(np.abs(no - (1 - c * c) / 2)) < 1e-14


@pytest.mark.parametrize("L,pbc", [(3, True), (4, False), (5, False), (6, True)])
def test_clean_spectrum(L, pbc):
    tau = 0.7
    E = np.linalg.eigvalsh(ff.hamiltonian(L, pbc, tau, np.zeros(L * L)))
    k = np.arange(L)
    if pbc:
        c = np.cos(2 * np.pi * k / L)
    else:
        c = np.cos(np.pi * (k + 1) / (L + 1))
    ref = np.sort((-2 * tau * (c[:, None] + c[None, :])).ravel())
    assert np.max(np.abs(E - ref)) < 1e-13


def test_conservation_shift_and_frozen():
    rng = np.random.default_rng(5)
    L, tau = 5, 0.5
    eps = rng.uniform(-4, 4, L * L)
    t = np.linspace(0, 3, 7)
    n = ff.occupations(L, False, tau, eps, t)
    assert np.max(np.abs(n.sum(axis=1) - ff.sublattice(L).sum())) < 1e-12
    assert n.min() > -1e-13 and n.max() < 1 + 1e-13
    n2 = ff.occupations(L, False, tau, eps + 3.7, t)
    assert np.max(np.abs(n - n2)) < 1e-12
    n0 = ff.occupations(L, False, 0.0, eps, t)
    assert np.max(np.abs(n0 - ff.sublattice(L).astype(float))) < 1e-14


def test_strong_disorder_freezes_imbalance():
    # |eps| >> tau: second-order perturbation theory bounds the lost
    # imbalance by 8 tau^2 / min gap^2-like terms; with gaps >= 50 and
    # tau = 0.5 the imbalance stays above 0.99
    rng = np.random.default_rng(3)
    L = 6
    eps = np.where(ff.sublattice(L), 100.0, -100.0) + rng.uniform(-1, 1, L * L)
    ne, no = ff.neel_dynamics(L, True, 0.5, eps, np.linspace(0, 5, 11))
    assert np.min(ne - no) > 0.99


# ---------------------------------------------------------------- spectrum, IPR
def test_ipr_without_hopping_is_one():
    """tau = 0: every eigenvector sits on one site (IPR exactly 1) and the
    energies are the sorted fields."""
    rng = np.random.default_rng(5)
    eps = rng.uniform(-4, 4, 25)
    E, ipr = ff.spectrum_ipr(5, False, 0.0, eps)
    np.testing.assert_array_equal(E, np.sort(eps))
    np.testing.assert_allclose(ipr, 1.0, atol=1e-15)


def test_ipr_plaquette_extremes():
    """Clean 2 x 2 lattice (a ring of four sites): E = -2 tau, 0, 0, 2 tau; the
    two non-degenerate states are uniform and staggered, IPR = 4 (1/2)^4."""
    E, ipr = ff.spectrum_ipr(2, False, 0.7, np.zeros(4))
    np.testing.assert_allclose(E, [-1.4, 0.0, 0.0, 1.4], atol=1e-14)
    np.testing.assert_allclose(ipr[[0, 3]], 0.25, atol=1e-14)


def test_ipr_weak_hopping_second_order():
    """Fields 3 apart at least, tau = 1e-3: second-order perturbation theory
    gives E_i = eps_i + sum_j tau^2 / (eps_i - eps_j) and
    IPR_i = 1 - 2 sum_j tau^2 / (eps_i - eps_j)^2 over the neighbours j of i,
    up to O(tau^4 / 3^4)."""
    L, tau = 4, 1e-3
    rng = np.random.default_rng(9)
    eps = 3.0 * rng.permutation(L * L)
    E, ipr = ff.spectrum_ipr(L, False, tau, eps)
    h = ff.hamiltonian(L, False, tau, eps)
    e2, s2 = np.zeros(L * L), np.zeros(L * L)
    for i in range(L * L):
        for j in np.flatnonzero(h[i] != 0):
            if j != i:
                d = eps[i] - eps[j]
                e2[i] += tau ** 2 / d
                s2[i] += tau ** 2 / d ** 2
    order = np.argsort(eps)
    np.testing.assert_allclose(E, (eps + e2)[order], atol=1e-11)
    np.testing.assert_allclose(ipr, (1.0 - 2.0 * s2)[order], atol=1e-11)


def test_cumulative_ipr_bins():
    """Rescaled energies: E_min in bin 0, E_max in the last bin, every state
    counted once, the bin sums adding up to the total IPR."""
    rng = np.random.default_rng(2)
    eps = rng.uniform(-10, 10, 36)
    E, ipr = ff.spectrum_ipr(6, False, 0.5, eps)
    sums, counts = ff.cumulative_ipr(E, ipr)
    b = ff.ipr_bin(E)
    assert b[0] == 0 and b[-1] == ff.N_IPR_BINS - 1
    assert counts.sum() == 36 and np.all(np.diff(b) >= 0)
    np.testing.assert_allclose(sums.sum(), ipr.sum(), rtol=1e-14)
    eps_r = (E - E[0]) / (E[-1] - E[0])
    np.testing.assert_array_equal(b, np.minimum(np.floor(eps_r / 0.05), 19).astype(int))
