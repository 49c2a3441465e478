"""Helpers shared by the GPU parity tests: run the oracle on the same inputs
as the device and derive per-case tolerances from the arithmetic.

The corner spectra of a CTMRG iterate are sensitive to rounding: singular
values of the cut matrix close to the 1e-12 relative cutoff are known only to
eps/cutoff relative accuracy, so two correct FP64 implementations differ by
that much.  ``oracle_spread`` measures it directly: the oracle is rerun on the
same state with every tensor element perturbed by a relative 1e-15, and the
largest change of a corner-spectrum entry is the case's rounding floor.  A
spectrum tolerance of max(1e-8, 10 * floor) is used (1e-8 being the target
for converged environments).

Near-degenerate pairs are worse: in an unconverged iterate the splitting of
two values whose exact fixed-point values coincide (relative gap ~1e-5)
depends on the rounding history; the oracle in the natural basis and the
same oracle in the Hermitian basis split such pairs differently by up to
~1e-7 while the pair's 2-norm agrees to <1e-9.  ``spectra_errors`` therefore
compares the 2-norms of clusters of entries closer than 1e-3 relative (to the
tolerance above) and every single entry only to 1e-6.
"""
import numpy as np

from oracle import peps as opeps
from oracle import run as orun
from oracle.model import Params


def oracle_params(D, chi, J=1.0, V=1.0, W=5.0, dt=0.05, **kw):
    return Params(D=D, chi=chi, J=J, V=V, W=W, dt=dt, **kw)


def oracle_state_from(gamma, lam, par):
    st = opeps.new_state(par)
    for i, s in enumerate(opeps.SITES):
        st["gam"][s] = np.array(gamma[i], dtype=complex)
        st["lam_h"][s] = np.array(lam[i], dtype=float)
        st["lam_v"][s] = np.array(lam[4 + i], dtype=float)
    return st


def oracle_spread(st, par, ctm_iters, ref_spectra, seed=0):
    rng = np.random.default_rng(seed)
    s2 = opeps.copy_state(st)
    for s in opeps.SITES:
        g = s2["gam"][s]
        s2["gam"][s] = g * (1 + 1e-15 * rng.normal(size=g.shape))
    o2, _ = orun.observe_state(s2, par, ctm_iters=ctm_iters)
    return float(np.max(np.abs(o2["corner_spectra"] - ref_spectra)))


def spectra_tol(spread):
    return max(1e-8, 10.0 * spread)


def _clusters(ref, rel=1e-3):
    """Index ranges of consecutive entries closer than rel (relative)."""
    out, start = [], 0
    for i in range(1, len(ref)):
        if not (ref[i - 1] > 0 and ref[i - 1] - ref[i] <= rel * ref[i - 1]):
            out.append((start, i))
            start = i
    out.append((start, len(ref)))
    return out


def spectra_errors(got, ref):
    """(largest cluster 2-norm error, largest single-entry error)."""
    cl = 0.0
    for g, r in zip(got, ref):
        for a, b in _clusters(r):
            cl = max(cl, abs(np.linalg.norm(g[a:b]) - np.linalg.norm(r[a:b])))
    return cl, float(np.max(np.abs(np.asarray(got) - np.asarray(ref))))


ENTRY_TOL = 1e-6


def assert_spectra(got, ref, spread, what=""):
    cl, en = spectra_errors(got, ref)
    assert cl < spectra_tol(spread), (what, cl, spread)
    assert en < ENTRY_TOL, (what, en)


# Converged environments (Delta below the convergence tolerance on both
# sides): the spectra are those of a fixed point, entry by entry to
# 1e-8 sigma_1.  Entries of a cluster whose relative gaps are below
# CLUSTER_GAP (exactly degenerate values of the fixed point, split at
# rounding level differently by two implementations) are compared through
# the cluster's 2-norm, to the same 1e-8 sigma_1.
CONVERGED_TOL = 1e-8
CLUSTER_GAP = 1e-6


def converged_spectra_errors(got, ref):
    """(largest single-entry error over entries outside clusters, largest
    cluster 2-norm error), each relative to the corner's sigma_1."""
    en = cl = 0.0
    for g, r in zip(np.asarray(got), np.asarray(ref)):
        s1 = r[0] if r[0] > 0 else 1.0
        for a, b in _clusters(r, rel=CLUSTER_GAP):
            if b - a == 1:
                en = max(en, abs(g[a] - r[a]) / s1)
            else:
                cl = max(cl, abs(np.linalg.norm(g[a:b]) - np.linalg.norm(r[a:b])) / s1)
    return en, cl
