"""Pins of the oracle's simple update (and, end to end, its CTMRG readout).

Every expected value here is fixed by the mathematics of the model, not by
the oracle itself:
    * truncation rule on hand-made spectra;
    * zero hopping: the gates are diagonal, the state stays a product and
      the imbalance is exactly 1 (Eq. Hanc with J = 0);
    * D = 1: the truncated two-site state keeps its dominant block, so the
      imbalance stays 1 while J dt is small;
    * dimer limit: only one layer of bonds carries the Hamiltonian (with the
      whole on-site field), the lattice splits into independent dimers, and
      the disorder-averaged Rabi formula gives the imbalance exactly;
    * 1D XX chain: decoupled chains, free fermions give I(t) = J0(2 J t);
      the error shrinks 4x when dt halves (second-order Trotter step);
    * symmetries J -> -J, W -> -W, V -> -V, dt -> -dt leave I unchanged;
    * particle-number conservation (U(1)) and the checkerboard symmetry;
    * short-time Taylor expansion I(t) = 1 - 2 J^2 t^2 + c4 t^4 with
      c4 = [5 J^4 + J^2 (9 V^2 + 2 W^2 Var z)] / 6 (nested commutators on the
      Néel state; checked by brute force in _taylor_reference below).
"""
import numpy as np
import pytest
from scipy.special import j0

from oracle import peps, run
from oracle.model import Params


def test_trunc_rule_cases():
    tr = peps.trunc_rule
    assert tr([1.0, 0.5, 0.25], 2) == 2
    assert tr([1.0, 0.5, 0.5, 0.1], 2) == 1          # never split the 0.5 pair
    assert tr([1.0, 0.5, 0.5, 0.1], 3) == 3
    assert tr([1.0, 0.5, 0.5], 5) == 3
    assert tr([1.0, 1e-13, 0.0], 3) == 1             # numerical zeros dropped
    assert tr([1.0, 0.3, 0.3 * (1 - 1e-11), 0.1], 2) == 1
    assert tr([1.0, 0.3, 0.3 * (1 - 1e-9), 0.1], 2) == 2
    assert tr([0.0, 0.0], 2) == 0
    assert tr([2.0, 2.0, 2.0, 1.0], 2) == 1          # stops at one value
    # the absolute part of the multiplet gap (1e-12 s_1) decides here: the
    # pair 1e-3, 1e-3 - 5e-13 is 5e-13 apart, above the relative gap
    # 1e-10 * 1e-3 = 1e-13 but below 1e-13 + 1e-12 * s_1, so it counts as one
    # multiplet and the cut moves below it; 2e-12 apart it is two values
    assert tr([1.0, 1e-3, 1e-3 - 5e-13, 1e-4], 2) == 1
    assert tr([1.0, 1e-3, 1e-3 - 2e-12, 1e-4], 2) == 2
    # the absolute part scales with s_1: the same relative pattern scaled by 1e6
    assert tr([1e6, 1e3, 1e3 - 5e-7, 1e2], 2) == 1
    assert tr([1e6, 1e3, 1e3 - 2e-6, 1e2], 2) == 2


def _imb(obs):
    return np.array([o["imbalance"] for o in obs])


def test_initial_state_and_zero_hopping():
    p = Params(D=2, chi=8, J=0.0, V=1.0, W=5.0, dt=0.1)
    obs, _ = run.run_job(p, 6, [0, 3, 6], ctm_iters=3)
    for o in obs:
        assert abs(o["imbalance"] - 1.0) < 1e-14
        assert np.max(np.abs(o["n"] - np.array([1.0, 0.0, 0.0, 1.0]))) < 1e-14


def test_D1_keeps_neel():
    p = Params(D=1, chi=1, J=1.0, V=1.0, W=5.0, dt=0.05)
    obs, _ = run.run_job(p, 10, [10], ctm_iters=2)
    assert abs(obs[0]["imbalance"] - 1.0) < 1e-14


def _dimer_exact(t, J, W):
    w = np.sqrt(J ** 2 + 4 * W ** 2)
    return 1 - np.sin(J * t / 2) ** 2 - J ** 2 / w ** 2 * np.sin(w * t / 2) ** 2


def _one_layer(layer):
    v = [0, 0, 0, 0]
    v[layer] = 1
    return tuple(v)


# layer 0 = H_A, 1 = H_B, 2 = V_A, 3 = V_B: horizontal dimers whose left site
# is on sublattice A (occupied) or B (empty), vertical dimers whose upper site
# is on A or B; V_B is applied once per step with dt, the others twice with dt/2
@pytest.mark.parametrize("W,steps,layer", [(5.0, [1, 2, 4], 0), (0.0, [2], 0),
                                           (5.0, [1, 2, 4], 1), (5.0, [1, 2, 4], 2),
                                           (0.0, [2], 2), (5.0, [1, 2, 4], 3)])
def test_dimer_limit(W, steps, layer):
    one = _one_layer(layer)
    p = Params(D=4, chi=16, J=1.0, V=1.0, W=W, dt=0.5, layer_J=one, layer_V=one, layer_w=one)
    obs, _ = run.run_job(p, max(steps), steps, ctm_iters=2)
    for o in obs:
        imb = _dimer_exact(o["t"], 1.0, W)
        assert abs(o["imbalance"] - imb) < 1e-12
        # sites (0,0), (1,1) are A, (1,0), (0,1) are B
        assert np.max(np.abs(o["n"] - 0.5 * (1.0 + imb * np.array([1, -1, -1, 1])))) < 1e-12
        # every site is one end of an isolated dimer: rho_p = diag(n, 1 - n)
        # with n = (1 + I)/2 on A sites, so both entropies are binary-entropy
        # closed forms of the exact imbalance
        nA = 0.5 * (1.0 + imb)
        h1 = -sum(x * np.log(x) for x in (nA, 1.0 - nA) if x > 0)
        hh = 2.0 * np.log(np.sqrt(nA) + np.sqrt(1.0 - nA))
        assert np.max(np.abs(o["renyi1"] - h1)) < 1e-10
        assert np.max(np.abs(o["renyi_half"] - hh)) < 1e-10
    if W == 0.0:
        assert abs(obs[0]["imbalance"] - np.cos(obs[0]["t"])) < 1e-12


def test_dimer_fixture_values():
    # closed-form values stored with their derivation in tests/golden
    import json, os
    fx = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "dimer_limit.json")))
    for t, v in fx["J1_W5"]:
        assert abs(_dimer_exact(t, 1.0, 5.0) - v) < 1e-11


def test_xx_chain_bessel_and_trotter_order():
    errs = []
    for dt in (0.05, 0.025):
        p = Params(D=4, chi=16, J=1.0, V=0.0, W=0.0, dt=dt,
                   layer_J=(1, 1, 0, 0), layer_V=(0, 0, 0, 0), layer_w=(0, 0, 0, 0))
        n = int(round(0.5 / dt))
        obs, _ = run.run_job(p, n, [n], ctm_iters=2)
        errs.append(obs[0]["imbalance"] - j0(2 * obs[0]["t"]))
    assert abs(errs[0]) < 2e-5
    assert 3.5 < errs[0] / errs[1] < 4.5


def test_symmetries():
    base = dict(D=2, chi=8, J=1.0, V=1.0, W=3.0, dt=0.05)
    ref = _imb(run.run_job(Params(**base), 5, [3, 5], ctm_iters=6)[0])
    for key in ("J", "V", "W", "dt"):
        kw = dict(base)
        kw[key] = -kw[key]
        got = _imb(run.run_job(Params(**kw), 5, [3, 5], ctm_iters=6)[0])
        assert np.max(np.abs(got - ref)) < 1e-10, key


def test_conservation_and_checkerboard():
    p = Params(D=2, chi=8, J=1.0, V=1.0, W=5.0, dt=0.05)
    obs, st = run.run_job(p, 10, [5, 10], ctm_iters=10)
    for o in obs:
        assert abs(o["sum_n"] - 2.0) < 1e-10
        assert o["max_offdiag"] < 1e-10
    assert np.array_equal(st["gam"][(0, 0)], st["gam"][(1, 1)])
    assert np.array_equal(st["gam"][(1, 0)], st["gam"][(0, 1)])
    for k in ("lam_h", "lam_v"):
        assert np.array_equal(st[k][(0, 0)], st[k][(1, 1)])
        assert np.array_equal(st[k][(1, 0)], st[k][(0, 1)])


def _taylor_c4(J, V, W, d_A=2):
    var_z = (d_A + 1) / (3.0 * (d_A - 1))
    return (5 * J ** 4 + J ** 2 * (9 * V ** 2 + 2 * W ** 2 * var_z)) / 6.0


def test_taylor_reference_by_brute_force():
    """The nested-commutator coefficient <[H,[H,[H,[H,n_0]]]]> on the Néel
    state of a 6x6 torus (no wrap-around loop of length <= 4) equals the
    closed form behind c4, for random fields:  (J^2/2) sum_j (3V + h_j -
    h_0)^2 + 10 J^4 over the four neighbours j of the occupied site 0."""
    rng = np.random.default_rng(5)
    Lx = Ly = 6
    N = Lx * Ly
    idx = lambda x, y: (y % Ly) * Lx + (x % Lx)
    bonds = sorted({tuple(sorted((idx(x, y), idx(x + dx, y + dy))))
                    for x in range(Lx) for y in range(Ly) for dx, dy in ((1, 0), (0, 1))})
    neel = tuple(1 if (x + y) % 2 == 0 else 0 for y in range(Ly) for x in range(Lx))
    J, V = 1.0, 1.0
    h = rng.uniform(-3, 3, N)

    def apply_H(vec):
        out = {}
        for cfg, amp in vec.items():
            sz = np.array(cfg) - 0.5
            e = sum(V * sz[a] * sz[b] for a, b in bonds) + float(h @ sz)
            out[cfg] = out.get(cfg, 0.0) + e * amp
            for a, b in bonds:
                if cfg[a] != cfg[b]:
                    c = list(cfg)
                    c[a], c[b] = c[b], c[a]
                    c = tuple(c)
                    out[c] = out.get(c, 0.0) + 0.5 * J * amp
        return out

    def dot(u, w, weight=lambda c: 1.0):
        return sum(a * w.get(c, 0.0) * weight(c) for c, a in u.items())

    n0 = lambda c: float(c[0])
    v0 = {neel: 1.0}
    v1 = apply_H(v0)
    v2 = apply_H(v1)
    w = apply_H({c: a * n0(c) for c, a in v1.items()})
    # <L^4 n0> = 2 n0(Neel) |v2|^2 - 8 <H n0 v1, v2> + 6 <v2|n0|v2>, H real symmetric
    L4 = 2 * n0(neel) * dot(v2, v2) - 8 * dot(w, v2) + 6 * dot(v2, v2, n0)
    nb = [idx(1, 0), idx(-1, 0), idx(0, 1), idx(0, -1)]
    closed = 0.5 * J ** 2 * sum((3 * V + h[j] - h[0]) ** 2 for j in nb) + 10 * J ** 4
    assert abs(L4 - closed) < 1e-9 * abs(closed)


def test_short_time_taylor():
    J, V, W = 1.0, 0.0, 2.0
    p = Params(D=4, chi=16, J=J, V=V, W=W, dt=0.01)
    obs, _ = run.run_job(p, 20, list(range(2, 21, 2)), ctm_iters=3)
    t = np.array([o["t"] for o in obs])
    y = _imb(obs) - 1.0
    c = np.linalg.lstsq(np.stack([t ** 2, t ** 4, t ** 6, t ** 8], 1), y, rcond=None)[0]
    assert abs(c[0] + 2 * J ** 2) < 1e-3
    assert abs(c[1] - _taylor_c4(J, V, W)) < 0.02
