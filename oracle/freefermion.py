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

The single-particle spectrum and the inverse participation ratios (the
IPR equation and the rescaled energy epsilon(E) of the same section):
spectrum_ipr diagonalises h (numpy.linalg.eigh) and returns the energies in
ascending order with I_k = sum_i |<i|E_k>|^4; cumulative_ipr rescales each
realization's spectrum to [0, 1] with its own E_min, E_max and sums the IPR
of the states in bins of width 0.05 (epsilon = 1 counted in the last bin).

Parity status: pinned (tests/test_oracle_freefermion.py) by the clean-torus
closed form J_0(4 tau t)^2 for the imbalance, the 2 x 2 plaquette closed
form cos^2(2 tau t), the analytic single-particle spectra of the clean open
and periodic lattices, particle-number conservation, invariance under a
uniform field shift, and frozen occupations without hopping; the IPR by
its exact value 1 without hopping, the clean plaquette's non-degenerate
states (1/4), and the second-order perturbative IPR at weak hopping.
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


def spectrum_ipr(L, pbc, tau, eps):
    """Energies E_k (ascending) of h and the IPR I_k = sum_i |<i|E_k>|^4 of
    each eigenvector, both of shape (L^2,)."""
    E, V = np.linalg.eigh(hamiltonian(L, pbc, tau, eps))
    return E, np.sum(V ** 4, axis=0)


N_IPR_BINS = 20  # rescaled-energy intervals of width 0.05


def ipr_bin(E):
    """Bin index of every energy after the rescaling epsilon = (E - E_min) /
    (E_max - E_min) of one realization (all 0 when the spectrum is flat)."""
    E = np.asarray(E, dtype=np.float64)
    lo, hi = E.min(), E.max()
    if not hi > lo:
        return np.zeros(E.shape, dtype=int)
    b = np.floor((E - lo) / (hi - lo) / 0.05).astype(int)
    return np.minimum(b, N_IPR_BINS - 1)


def cumulative_ipr(E, ipr):
    """Summed IPR and number of states per rescaled-energy bin of one
    realization: arrays of shape (20,)."""
    b = ipr_bin(E)
    sums = np.zeros(N_IPR_BINS)
    counts = np.zeros(N_IPR_BINS, dtype=int)
    np.add.at(sums, b, ipr)
    np.add.at(counts, b, 1)
    return sums, counts
