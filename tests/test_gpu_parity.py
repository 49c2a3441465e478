"""Device path vs the oracle, through the C ABI (needs an MI355X).

Tolerances: imbalance and occupations 1e-6 absolute (the target stated for
the FP64 path), bond spectra and truncation errors 1e-10, corner spectra:
2-norms of near-degenerate clusters to max(1e-8, 10 x the oracle's own
rounding floor) and single entries to 1e-6 (tests/_parity.py explains why).
"""
import numpy as np
import pytest

import synthetic
from oracle import peps as opeps
from oracle import run as orun
from tests import _parity as par

P = pytest.importorskip("paper_1910_11359_amd")

pytestmark = pytest.mark.gpu


def _gpu_state(D, chi, **kw):
    return P.State(P.make_config(D, chi, **kw))


def test_small_workload_vs_oracle():
    """D=2, chi=8, W=5, V=1, dt=0.05: 20 steps, 10 cold CTMRG iterations
    after every step."""
    cfg = synthetic.small_config()
    kw = dict(J=cfg["J"], V=cfg["V"], W=cfg["W"], dt=cfg["dt"])
    st = _gpu_state(cfg["D"], cfg["chi"], **kw)
    p = par.oracle_params(cfg["D"], cfg["chi"], **kw)
    ost = opeps.new_state(p)
    for step in range(1, cfg["n_steps"] + 1):
        st.trotter_step(1)
        opeps.trotter_step(ost, p)
        st.ctmrg(0.0, cfg["ctm_iters"], True)
        g = st.observe()
        o, _ = orun.observe_state(ost, p, ctm_iters=cfg["ctm_iters"])
        assert abs(g["t"] - step * cfg["dt"]) < 1e-12
        assert abs(g["imbalance"] - o["imbalance"]) < 1e-6, step
        assert np.max(np.abs(g["n"] - o["n"])) < 1e-6, step
        assert np.max(np.abs(g["eps"] - o["eps"])) < 1e-10, step
        assert np.max(np.abs(st.bond_spectra() - o["bond_spectra"])) < 1e-10, step
        spread = par.oracle_spread(ost, p, cfg["ctm_iters"], o["corner_spectra"])
        par.assert_spectra(st.corner_spectra(), o["corner_spectra"], spread, step)
        assert abs(g["sum_n"] - 2.0) < 1e-10 and g["max_offdiag"] < 1e-10
        assert np.max(np.abs(g["renyi1"] - o["renyi1"])) < 1e-6, step
        assert np.max(np.abs(g["renyi_half"] - o["renyi_half"])) < 1e-6, step


@pytest.mark.parametrize("D,chi,seed,flags", [(2, 8, 3, 0), (3, 9, 4, 0), (3, 12, 5, 0), (4, 16, 6, 0),
                                              (4, 16, 7, 1), (3, 12, 5, 2), (4, 16, 6, 2),
                                              (4, 16, 7, 3)])
def test_random_state_vs_oracle(D, chi, seed, flags):
    """Seeded random site tensors and bond weights (full rank at every
    bond): CTMRG from the state, one Trotter step, CTMRG again.  Covers the
    direct projector SVD (n <= 96) and the subspace-iteration one with the
    cut matrices formed (the default at these n) and, with flag 2, applied
    through their enlarged-corner factors; flag 1 autotunes the GEMM tiles."""
    gam, lam = synthetic.random_state(seed, D)
    kw = dict(J=1.0, V=1.0, W=3.0, dt=0.05)
    st = _gpu_state(D, chi, flags=flags, **kw)
    st.set_state(gam, lam)
    p = par.oracle_params(D, chi, **kw)
    ost = par.oracle_state_from(gam, lam, p)
    for phase in range(2):
        st.ctmrg(0.0, 4, True)
        g = st.observe()
        o, _ = orun.observe_state(ost, p, ctm_iters=4)
        assert abs(g["imbalance"] - o["imbalance"]) < 1e-6
        assert np.max(np.abs(g["n"] - o["n"])) < 1e-6
        spread = par.oracle_spread(ost, p, 4, o["corner_spectra"])
        par.assert_spectra(st.corner_spectra(), o["corner_spectra"], spread, phase)
        if phase == 0:
            eps = st.trotter_step(1, want_eps=True)
            opeps.trotter_step(ost, p)
            assert np.max(np.abs(st.bond_spectra() - opeps.bond_spectra(ost))) < 1e-10
            assert np.max(np.abs(eps - np.array([ost["eps"][s] for s in opeps.SITES]))) < 1e-10


def test_product_start_low_rank_cuts():
    """Neel start, D=3, chi=18 (n=162: subspace-iteration SVD), large V.
    Right after the start the cut matrices have a few dominant singular
    values and a tail spanning ten decades above the cutoff: the tail
    directions sit below the rounding level of the dominant ones in a mixed
    block, so the device must recover them by restarting dropped columns.
    The same with the cut matrices applied through their factors (FP64,
    same bars), and the FP32 path with factored cuts (products in FP32)
    must stay finite with the imbalance within 1e-3."""
    kw = dict(J=1.0, V=1.6759187457576177, W=1.3506622087662332, dt=0.05)
    st = _gpu_state(3, 18, **kw)
    stf = _gpu_state(3, 18, flags=P.FLAG_FACTORED_CUTS, **kw)
    st32 = P.State(P.make_config(3, 18, dtype="fp32", flags=P.FLAG_FACTORED_CUTS, **kw))
    p = par.oracle_params(3, 18, **kw)
    ost = opeps.new_state(p)
    for step in range(1, 6):
        for s in (st, stf, st32):
            s.trotter_step(1)
        opeps.trotter_step(ost, p)
        if step not in (1, 2, 5):
            continue
        for s in (st, stf, st32):
            s.ctmrg(0.0, 10, True)
        g32 = st32.observe()
        o, _ = orun.observe_state(ost, p, ctm_iters=10)
        spread = par.oracle_spread(ost, p, 10, o["corner_spectra"])
        for s in (st, stf):
            g = s.observe()
            assert abs(g["imbalance"] - o["imbalance"]) < 1e-6, step
            assert np.max(np.abs(g["n"] - o["n"])) < 1e-6, step
            par.assert_spectra(s.corner_spectra(), o["corner_spectra"], spread, step)
        assert abs(g32["imbalance"] - o["imbalance"]) < 1e-3, step
    for s in (st, stf, st32):
        s.close()


@pytest.mark.parametrize("d_A,D,chi", [(1, 2, 8), (3, 2, 8), (4, 2, 8), (5, 2, 4), (3, 3, 9)])
def test_aux_levels_vs_oracle(d_A, D, chi):
    """More disorder levels (d = 2 d_A up to 10, fields on d_A equally spaced
    levels; d_A = 1 is the clean model): 6 steps, CTMRG from a cold start
    after steps 3 and 6."""
    kw = dict(J=1.0, V=1.0, W=3.0, dt=0.05, d_A=d_A)
    st = _gpu_state(D, chi, **kw)
    p = par.oracle_params(D, chi, **kw)
    ost = opeps.new_state(p)
    for step in range(1, 7):
        st.trotter_step(1)
        opeps.trotter_step(ost, p)
        if step % 3:
            continue
        st.ctmrg(0.0, 8, True)
        g = st.observe()
        o, _ = orun.observe_state(ost, p, ctm_iters=8)
        assert abs(g["imbalance"] - o["imbalance"]) < 1e-6, step
        assert np.max(np.abs(g["n"] - o["n"])) < 1e-6, step
        assert np.max(np.abs(g["eps"] - o["eps"])) < 1e-10, step
        assert np.max(np.abs(st.bond_spectra() - o["bond_spectra"])) < 1e-10, step
        assert np.max(np.abs(g["renyi1"] - o["renyi1"])) < 1e-6, step
        spread = par.oracle_spread(ost, p, 8, o["corner_spectra"])
        par.assert_spectra(st.corner_spectra(), o["corner_spectra"], spread, step)
    st.close()


def _dimer_exact(t, J, W):
    w = np.sqrt(J ** 2 + 4 * W ** 2)
    return 1 - np.sin(J * t / 2) ** 2 - J ** 2 / w ** 2 * np.sin(w * t / 2) ** 2


@pytest.mark.parametrize("layer", [0, 1, 2, 3])
def test_dimer_limit_closed_form(layer):
    """Only one layer of bonds carries the Hamiltonian, with the whole field:
    independent dimers, no Trotter error, exact readout.  Layers H_A, H_B
    (horizontal dimers with the occupied site left or right) and V_A, V_B
    (vertical dimers with the occupied site above or below), so both bond
    directions of the simple update and of the CTMRG are pinned."""
    one = [0, 0, 0, 0]
    one[layer] = 1
    st = _gpu_state(4, 16, J=1.0, V=1.0, W=5.0, dt=0.5, layer_J=one, layer_V=one, layer_w=one)
    for steps in (1, 1, 2):
        st.trotter_step(steps)
        st.ctmrg(0.0, 2, True)
        g = st.observe()
        imb = _dimer_exact(g["t"], 1.0, 5.0)
        assert abs(g["imbalance"] - imb) < 1e-12, (layer, g["t"])
        assert np.max(np.abs(g["n"] - 0.5 * (1.0 + imb * np.array([1, -1, -1, 1])))) < 1e-12
    st.close()


@pytest.mark.parametrize("dtype,tol", [("fp64", 1e-9), ("fp32", 1e-4)])
def test_autotuned_tiles_match_heuristic(dtype, tol):
    """D=4, chi=32: the autotuned tile kinds change only the summation order
    of the GEMMs, so observables agree with the default plan to rounding."""
    kw = dict(J=1.0, V=1.0, W=5.0, dt=0.05, dtype=dtype)
    out = []
    for flags in (0, P.FLAG_AUTOTUNE):
        st = _gpu_state(4, 32, flags=flags, **kw)
        st.trotter_step(4)
        st.ctmrg(0.0, 8, True)
        st.trotter_step(2)
        st.ctmrg(0.0, 3, False)
        out.append(st.observe())
        st.close()
    assert np.max(np.abs(out[0]["n"] - out[1]["n"])) < tol
    assert abs(out[0]["imbalance"] - out[1]["imbalance"]) < tol


def test_zero_hopping_keeps_neel():
    st = _gpu_state(3, 9, J=0.0, V=1.0, W=5.0, dt=0.1)
    st.trotter_step(4)
    st.ctmrg(0.0, 3, True)
    g = st.observe()
    assert abs(g["imbalance"] - 1.0) < 1e-13
    assert np.max(np.abs(g["n"] - np.array([1.0, 0.0, 0.0, 1.0]))) < 1e-13


def test_checkerboard_bitwise():
    st = _gpu_state(3, 9, J=1.0, V=1.0, W=2.0, dt=0.05)
    st.trotter_step(5)
    gam, lam = st.get_state()
    assert np.array_equal(gam[0], gam[3]) and np.array_equal(gam[1], gam[2])
    assert np.array_equal(lam[0], lam[3]) and np.array_equal(lam[1], lam[2])
    assert np.array_equal(lam[4], lam[7]) and np.array_equal(lam[5], lam[6])


def test_symmetries_on_device():
    base = dict(J=1.0, V=1.0, W=3.0, dt=0.05)

    def imb(**kw):
        st = _gpu_state(2, 8, **kw)
        st.trotter_step(5)
        st.ctmrg(0.0, 6, True)
        return st.observe()["imbalance"]

    ref = imb(**base)
    for key in ("J", "V", "W"):
        kw = dict(base)
        kw[key] = -kw[key]
        assert abs(imb(**kw) - ref) < 1e-10, key


def test_warm_start_continues():
    st = _gpu_state(2, 8, J=1.0, V=1.0, W=5.0, dt=0.05)
    st.trotter_step(6)
    st.ctmrg(0.0, 20, True)
    a = st.observe()
    it, dl = st.ctmrg(0.0, 2, False)
    b = st.observe()
    assert abs(a["imbalance"] - b["imbalance"]) < 1e-8
    assert dl < 1e-6


@pytest.mark.parametrize("D,chi,flags,dtype,tol", [(3, 12, 0, "fp64", 1e-11), (4, 32, 0, "fp64", 1e-11),
                                                     (4, 32, 2, "fp64", 1e-11), (4, 32, 2, "fp32", 1e-4)])
def test_corner_reuse_across_iterations(D, chi, flags, dtype, tol):
    """Within one CTMRG call the left move of the second and later
    iterations reuses the enlarged corners the down move left valid; a
    sequence of one-iteration calls recomputes them.  The two schedules are
    otherwise the same (warm projector subspaces persist across calls), so
    they agree to rounding."""
    kw = dict(J=1.0, V=1.0, W=4.0, dt=0.05, dtype=dtype, flags=flags)
    out = []
    for split in (False, True):
        st = _gpu_state(D, chi, **kw)
        st.trotter_step(5)
        if split:
            st.ctmrg(0.0, 1, True)
            for _ in range(4):
                st.ctmrg(0.0, 1, False)
        else:
            st.ctmrg(0.0, 5, True)
        out.append((st.observe(), st.corner_spectra()))
        st.close()
    (a, ca), (b, cb) = out
    assert np.max(np.abs(a["n"] - b["n"])) < tol
    assert abs(a["imbalance"] - b["imbalance"]) < tol
    assert np.max(np.abs(ca - cb)) < 100 * tol


def test_nan_state_is_reported_and_poisons():
    gam, lam = synthetic.random_state(9, 2)
    gam[0, 0, 0, 0, 0, 0] = np.nan
    st = _gpu_state(2, 8)
    st.set_state(gam, lam)
    with pytest.raises(P.IpepsError) as e:
        st.trotter_step(1, want_eps=True)
    assert e.value.code == -4
    with pytest.raises(P.IpepsError) as e:
        st.ctmrg(0.0, 1, True)
    assert e.value.code == -4


def test_not_converged_is_flagged():
    st = _gpu_state(2, 8, J=1.0, V=1.0, W=5.0, dt=0.05)
    st.trotter_step(3)
    with pytest.raises(P.IpepsError) as e:
        st.ctmrg(1e-30, 2, True)
    assert e.value.code == -5
    st.observe()  # environment still usable
