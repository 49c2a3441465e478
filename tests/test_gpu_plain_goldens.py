"""Plain FP64 workload (D=4, chi=32, W in {2, 10}, V in {0, 1}, dt=0.05 to
t=5) on the device against oracle values stored in tests/golden/ (written by
tests/golden/make_plain_golden.py, which calls only oracle/).

Every 10 steps CTMRG runs from a cold start until the corner spectra move by
less than 1e-10 in one iteration (capped at the golden's max_iter, the same
cap the oracle used).

The simple-update trajectory can be ill-conditioned: near-degenerate bond
weights make it amplify a rounding difference by ~3x per step (W=2, V=0
after t=3).  Each golden observation therefore carries "su_spread", the
oracle's own bond-spectrum change when its start is perturbed by 1e-15
relative.  Tolerances at an observation, with a = 1e3 * su_spread (device and
oracle differ by many roundings per step, not one):
* imbalance and occupations: max(1e-6, a); truncation errors and bond
  spectra: max(1e-10, a);
* corner spectra, where both the device and the oracle converged and
  a < 1e-10: 2-norms of near-degenerate clusters to 1e-8 and single entries
  to 1e-6 (an unconverged iterate's spectra are rounding-sensitive);
* observations with a > 1e-3 lie past the trajectory's predictability
  horizon and are not compared; at least the first half of the
  observations must be inside it.
"""
import json
import os

import numpy as np
import pytest

from tests import _parity as par

P = pytest.importorskip("paper_1910_11359_amd")

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
CASES = [(2, 0), (2, 1), (10, 0), (10, 1)]


def _golden(W, V):
    path = os.path.join(HERE, "golden", f"plain_W{W:g}_V{V:g}.json")
    if not os.path.exists(path):
        pytest.skip(f"{path} missing")
    g = json.load(open(path))
    cfg = g["config"]
    if len(g["obs"]) < cfg["n_steps"] // cfg["observe_every"] + 1 or "su_spread" not in g["obs"][-1]:
        pytest.skip(f"{path} incomplete ({len(g['obs'])} observations)")
    return g


@pytest.mark.parametrize("W,V", CASES)
def test_plain_fp64_against_oracle_goldens(W, V):
    g = _golden(W, V)
    cfg = g["config"]
    st = P.State(P.make_config(cfg["D"], cfg["chi"], J=cfg["J"], V=cfg["V"], W=cfg["W"],
                               dt=cfg["dt"]))
    obs = {o["step"]: o for o in g["obs"]}
    compared = 0
    for step in range(0, cfg["n_steps"] + 1):
        if step > 0:
            st.trotter_step(1)
        if step not in obs:
            continue
        o = obs[step]
        a = 1e3 * o["su_spread"]
        if a > 1e-3:
            continue
        compared += 1
        it, dl = st.ctmrg(g["tol"], g["max_iter"], True, allow_notconv=True)
        got = st.observe()
        tol_obs, tol_su = max(1e-6, a), max(1e-10, a)
        assert abs(got["imbalance"] - o["imbalance"]) < tol_obs, (step, got["imbalance"], o["imbalance"])
        assert np.max(np.abs(got["n"] - np.array(o["n"]))) < tol_obs, step
        assert np.max(np.abs(got["eps"] - np.array(o["eps"]))) < tol_su, step
        assert np.max(np.abs(st.bond_spectra() - np.array(o["bond_spectra"]))) < tol_su, step
        if o["ctm_delta"] < g["tol"] and dl < g["tol"] and a < 1e-10:
            cl, en = par.spectra_errors(st.corner_spectra(), np.array(o["corner_spectra"]))
            assert cl < 1e-8 and en < par.ENTRY_TOL, (step, cl, en)
    assert compared >= (len(obs) + 1) // 2, compared
    st.close()
