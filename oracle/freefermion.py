"""Free-fermion Néel dynamics (TEST INFRASTRUCTURE ONLY: imported by tests/,
__graft_entry__.smoke() and bench.py's cpu_baseline leg, never by the product).

Follows the paper's set-up for non-interacting fermions (section "Set up for
non-interacting fermions" and the free-fermion figure of the results): an
L x L square lattice, one orbital per site, hopping between nearest
neighbours and a disorder field on every site; the Néel state (every other
site filled) evolves under the single-particle Hamiltonian, and the mean
occupation of the two sublattices is recorded in time.

Conventions (readings stated in the design notes):
    site i = x * L + y, x, y in [0, L); sublattice "even" = (x + y) even,
    which is the filled one at t = 0;
    h = -tau * sum over nearest-neighbour pairs (|i><j| + |j><i|)
        + sum_i eps_i |i><i|,
    open boundaries, or periodic ones (pbc, L >= 3) in both directions.

Because the fermions do not interact, the many-body state stays a Slater
determinant of the orbitals that start on the filled sites; orbital j
evolves as U(t) e_j with U(t) = exp(-i h t), so the occupation of site i is
n_i(t) = sum over filled j of |U_ij(t)|^2.  This module forms h densely,
diagonalises it (numpy.linalg.eigh) and builds U(t) = V diag(exp(-i E t)) V^T
exactly for every requested time: no time stepping.

Parity status: pinned (tests/test_oracle_freefermion.py) by the clean-torus
closed form J_0(4 tau t)^2 for the imbalance, the 2 x 2 plaquette closed
form cos^2(2 tau t), the analytic single-particle spectra of the clean open
and periodic lattices, particle-number conservation, invariance under a
uniform field shift, and frozen occupations without hopping.
"""
import numpy as np


def sublattice(L):
    """Boolean mask over sites, True on the filled (even) sublattice."""
    x, y = np.divmod(np.arange(L * L), L)
    return (x + y) % 2 == 0


def hamiltonian(L, pbc, tau, eps):
    """Dense single-particle Hamiltonian (real symmetric, L^2 x L^2)."""
    n = L * L
    h = np.diag(np.asarray(eps, dtype=np.float64).reshape(n).copy())
    for x in range(L):
        for y in range(L):
            i = x * L + y
            for dx, dy in ((1, 0), (0, 1)):
                xn, yn = x + dx, y + dy
                if pbc:
                    xn %= L
                    yn %= L
                elif xn >= L or yn >= L:
                    continue
                j = xn * L + yn
                h[i, j] -= tau
                h[j, i] -= tau
    return h


def occupations(L, pbc, tau, eps, times):
    """n_i(t) for every site and time, shape (len(times), L^2)."""
    h = hamiltonian(L, pbc, tau, eps)
    E, V = np.linalg.eigh(h)
    filled = np.flatnonzero(sublattice(L))
    out = np.empty((len(times), L * L))
    for m, t in enumerate(times):
        U = (V * np.exp(-1j * E * t)) @ V.T  # exp(-i h t)
        out[m] = np.sum(np.abs(U[:, filled]) ** 2, axis=1)
    return out


def neel_dynamics(L, pbc, tau, eps, times):
    """Mean occupation of the even (initially filled) and odd sublattices at
    each time: arrays n_even, n_odd of shape (len(times),)."""
    n = occupations(L, pbc, tau, eps, times)
    ev = sublattice(L)
    odd = n[:, ~ev].mean(axis=1) if (~ev).any() else np.zeros(len(times))  # L = 1: no odd site
    return n[:, ev].mean(axis=1), odd
