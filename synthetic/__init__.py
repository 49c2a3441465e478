"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle.

This module holds no arithmetic of the method: only parameter sets of the
workloads, seeded random numbers and seeded random tensors in plain host
layouts.  Both the device path (through its Python binding) and the oracle
read their inputs from here, so a parity test feeds both sides the same
bytes.

Workloads (d_A = 2 throughout, Néel ⊗ |+> initial state; the paper uses no
dataset, its workloads are parameter points):
    small       D=2, chi=8,  J=1, V=1, W=5, dt=0.05, 20 steps, 10 CTMRG
                iterations per observation, observe every step
    plain       D=4, chi=32, W in {2, 10} x V in {0, 1}, dt=0.05, 100 steps,
                observe every 10, CTMRG to delta < 1e-10
    headline    D=6, chi=72, J=1, V=1, W=8, dt=0.05, 100 steps
    sweep       64 jobs: D in {3,4,5,6} x V in {0,1} x 8 W values drawn from
                default_rng(1911359).uniform(1, 20, 8); chi = 2 D^2; 50 steps
    serving     256 requests from default_rng(20191025)

Free-fermion workload (the paper's non-interacting comparison: L x L
lattices, 100 disorder realizations, Néel start, t up to 5):
    ff          L in {10, 20, 40} x h in {4, 10, 100} x {continuous, 3-level}
    ff headline L = 40, h = 10, continuous, 100 realizations, 50 observations
                every 0.1 (tau = 1/2, the hopping of J (SxSx + SySy) at J = 1)
Fields: continuous eps ~ h U[-1, 1]; s-level eps = h z with z uniform over s
equally spaced values in [-1, 1] (s = 3: spin-1 levels -h, 0, h).
"""
import numpy as np

SITES = [(0, 0), (1, 0), (0, 1), (1, 1)]


def small_config():
    return dict(D=2, chi=8, J=1.0, V=1.0, W=5.0, dt=0.05, n_steps=20, observe_every=1,
                ctm_iters=10)


def plain_configs():
    return [dict(D=4, chi=32, J=1.0, V=V, W=W, dt=0.05, n_steps=100, observe_every=10,
                 ctm_tol=1e-10, ctm_max_iter=2000)
            for W in (2.0, 10.0) for V in (0.0, 1.0)]


def headline_config():
    return dict(D=6, chi=72, J=1.0, V=1.0, W=8.0, dt=0.05, n_steps=100, observe_every=10)


def sweep_jobs():
    Ws = np.random.default_rng(1911359).uniform(1.0, 20.0, 8)
    jobs = []
    for D in (3, 4, 5, 6):
        for V in (0.0, 1.0):
            for W in Ws:
                jobs.append(dict(D=D, chi=2 * D * D, J=1.0, V=V, W=float(W), dt=0.05,
                                 n_steps=50, observe_every=10, ctm_iters=10))
    return jobs


def serving_stream(n=256, rate=1.0, seed=20191025):
    """Poisson arrivals (rate per second) with per-request parameters."""
    rng = np.random.default_rng(seed)
    out = []
    t = 0.0
    for _ in range(n):
        t += rng.exponential(1.0 / rate)
        D = int(rng.integers(3, 9))
        c = int(rng.integers(2, 4))
        out.append(dict(arrival=t, D=D, chi=min(128, c * D * D), J=1.0,
                        V=float(rng.uniform(0.0, 2.0)), W=float(rng.uniform(1.0, 20.0)),
                        dt=0.05, n_steps=int(rng.integers(20, 201)), observe_every=10,
                        ctm_iters=10))
    return out


def random_state(seed, D, d_A=2, lam_min=0.05):
    """Random site tensors and bond weights in the host layouts of both sides.

    gamma: complex (4, d, D, D, D, D) in site order SITES, legs (s,u,l,d,r);
    lam:   real (8, D): horizontal bonds of SITES then vertical bonds, each
           sorted descending, positive, unit 2-norm.
    """
    rng = np.random.default_rng(seed)
    d = 2 * d_A
    shape = (4, d, D, D, D, D)
    gamma = rng.normal(size=shape) + 1j * rng.normal(size=shape)
    lam = np.sort(rng.uniform(lam_min, 1.0, (8, D)), axis=1)[:, ::-1]
    lam = lam / np.linalg.norm(lam, axis=1, keepdims=True)
    return gamma, np.ascontiguousarray(lam)


def ff_configs():
    return [dict(L=L, h=h, kind=kind, n_real=100, tau=0.5, pbc=False, dt=0.1, n_times=50)
            for L in (10, 20, 40) for h in (4.0, 10.0, 100.0) for kind in ("continuous", "discrete3")]


def ff_headline():
    return dict(L=40, h=10.0, kind="continuous", n_real=100, tau=0.5, pbc=False, dt=0.1, n_times=50)


def ff_fields(L, n_real, h, kind, seed):
    """Seeded on-site fields, shape (n_real, L*L), FP64."""
    rng = np.random.default_rng(seed)
    if kind == "continuous":
        return h * rng.uniform(-1.0, 1.0, (n_real, L * L))
    s = int(kind.replace("discrete", ""))
    levels = np.linspace(-1.0, 1.0, s)
    return h * levels[rng.integers(0, s, (n_real, L * L))]
