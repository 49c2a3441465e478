/* Free-fermion Néel dynamics and single-particle spectra on one gfx950 GPU: the non-interacting
 * comparison workload of arXiv:1910.11359 (section "Set up for
 * non-interacting fermions"; results for the non-interacting case, the
 * free-fermion figure: mean occupation of the two sublattices of a finite
 * lattice after a Néel start, averaged over disorder realizations).
 *
 * Model: L x L square lattice, site i = x*L + y (0 <= x, y < L), one orbital
 * per site, single-particle Hamiltonian
 *     h = -tau * sum over nearest-neighbour pairs (|i><j| + |j><i|) + sum_i eps_i |i><i|
 * with open boundaries (pbc = 0) or periodic ones in both directions
 * (pbc = 1, L >= 3).  Start: the Néel state, sites with x + y even filled.
 * Without interactions the state stays a Slater determinant of the orbitals
 * that start on the filled sites, each evolving as exp(-i h t) e_j; the
 * library integrates them exactly (Chebyshev expansion of the propagator over
 * each interval dt, split so that each piece needs at most a few tens of
 * terms) and never forms h densely.
 *
 * Error codes are those of ipeps.h. */
#ifndef FF_H
#define FF_H

#include "ipeps.h"

#ifdef __cplusplus
extern "C" {
#endif

/* Runs n_real independent realizations on hip_stream (NULL: the default
 * stream) and returns after enqueueing; results are valid once the stream
 * has completed.
 *   L        1..45 (L*L <= 2048)
 *   pbc      0 open, 1 periodic (needs L >= 3)
 *   tau      hopping amplitude (finite; tau = 1/2 is the hopping of the
 *            spin model's J (SxSx + SySy) at J = 1)
 *   dt       observation interval (> 0); observations at t = m*dt, m = 1..n_times
 *   eps      DEVICE, FP64, n_real * L*L on-site fields, realization-major
 *   n_even   DEVICE, FP64, n_real * n_times outputs: mean occupation of the
 *            initially filled sublattice (x + y even), [r*n_times + m - 1]
 *   n_odd    DEVICE, FP64, same layout, the other sublattice (0 when L = 1)
 * The caller owns all buffers; the library allocates a stream-ordered
 * workspace of 16 * n_real * n_times * ceil(L*L/2) bytes for the call.
 * The imbalance of the iPEPS readout corresponds to n_even - n_odd.
 * Returns IPEPS_OK, IPEPS_EINVAL (argument out of range, a NULL buffer with
 * work to do, n_real > 65535), IPEPS_ENOMEM, IPEPS_EDEVICE.  NaN fields give
 * NaN outputs. */
int ff_neel_dynamics(int L, int pbc, double tau, double dt, int n_times, int n_real,
                     const double* eps, double* n_even, double* n_odd, void* hip_stream);

/* ff_neel_dynamics for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): the same kernels and results, with the per-orbital partial
 * weights in a fixed scratch array of FF_NOALLOC_SCRATCH_DOUBLES doubles
 * (64 MiB) that the library holds on every device it runs on until the
 * process ends.  Allocates nothing (no hipMalloc / hipFree / stream-ordered
 * allocation).  Needs 2 * n_real * n_times * ceil(L*L/2) <=
 * FF_NOALLOC_SCRATCH_DOUBLES (the L = 40, 100-realization, 50-time workload
 * fits), else returns IPEPS_ETOOBIG with a message on stderr.  Every call on
 * one device shares that device's scratch: calls whose work overlaps on one
 * device (two streams, or two host threads) race and must be ordered by the
 * caller.  The scratch needs no clearing (each entry is written before it is
 * read).  Other arguments, results and errors as for ff_neel_dynamics. */
#define FF_NOALLOC_SCRATCH_DOUBLES (8L * 1024 * 1024)
int ff_neel_dynamics_noalloc(int L, int pbc, double tau, double dt, int n_times, int n_real,
                             const double* eps, double* n_even, double* n_odd, void* hip_stream);

/* Single-particle spectrum and inverse participation ratios (the spectrum
 * and cumulative-IPR figures of the non-interacting section: the IPR
 * equation I_k = sum_i |<i|E_k>|^4 and the rescaled energy
 * epsilon(E) = (E - E_min) / (E_max - E_min)) of n_real realizations of h
 * (model as above), on hip_stream.
 *   L          1..40.  L <= 16: the L^2 x L^2 eigenproblem is solved in one
 *              workgroup per realization (a one-sided Jacobi SVD of h + c I,
 *              with c twice a Gershgorin bound G, whose singular vectors are
 *              the eigenvectors of h); returns after enqueueing.  L > 16: a
 *              two-sided block Jacobi over blocks of 32 indices (each pair of
 *              blocks diagonalised exactly, its rotation applied to h and to
 *              the eigenvectors as 64 x 64 MFMA products), all realizations
 *              in every launch; the call waits for the stream once per sweep
 *              to test convergence (off-diagonal part of h below 1e-12 of its
 *              Frobenius norm, or at the level the 64 x 64 solves reach) and
 *              returns after enqueueing the readout
 *   pbc, tau   as above
 *   eps        DEVICE, FP64, n_real * L*L fields, realization-major
 *   energies   DEVICE, FP64, n_real * L*L: the energies of each realization
 *              in ascending order
 *   ipr        DEVICE, FP64, n_real * L*L: IPR of the eigenvector of the same
 *              energy (1 on one site, 1/L^2 spread evenly)
 *   bin_ipr    DEVICE, FP64, n_real * 20: per realization the summed IPR of
 *              the states with epsilon in [0.05 b, 0.05 (b + 1)), b = 0..19
 *              (epsilon = 1 in b = 19; all states in b = 0 for a flat
 *              spectrum)
 *   bin_count  DEVICE, int32, n_real * 20: the number of those states (0:
 *              the interval is not populated)
 * Eigenvectors of degenerate energies are any orthonormal basis of their
 * space (their IPRs are not unique).  The caller owns all buffers; the
 * library allocates a stream-ordered workspace of about
 * 16 * n_real * L^4 bytes for the call (L > 16: 16 * n_real * np^2 with np
 * = L^2 rounded up to a multiple of 64).  Returns IPEPS_OK, IPEPS_EINVAL
 * (argument out of range, a NULL buffer with work to do, n_real > 65535),
 * IPEPS_ENOMEM, IPEPS_ENOTCONV (L > 16: not converged in 60 sweeps; the
 * outputs hold the last iterate), IPEPS_EDEVICE.  NaN fields give NaN
 * outputs (L > 16: IPEPS_ENOTCONV). */
int ff_spectrum_ipr(int L, int pbc, double tau, int n_real, const double* eps, double* energies,
                    double* ipr, double* bin_ipr, int* bin_count, void* hip_stream);

/* Host copy of the Bessel-function routine behind the propagator's
 * coefficients: J_0(x) .. J_kmax(x) into out[0..kmax] (host), x >= 0,
 * 0 <= kmax <= 200.  Returns IPEPS_OK or IPEPS_EINVAL. */
int ff_bessel_j(double x, int kmax, double* out);

#ifdef __cplusplus
}
#endif

#endif
