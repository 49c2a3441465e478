"""Oracle: one time-evolution job = Trotter steps + CTMRG readouts.

Test infrastructure only (see package docstring).

Follows the paper's three-step procedure (initialization, quench, readout)
and records at each observation the quantities the paper monitors:
occupation of each site with the auxiliary spin traced out, the imbalance,
and the accumulated local truncation error of each site.
"""
import numpy as np

from . import ctmrg as _ct
from . import peps as _pp


def observe_state(st, params, ctm_iters=10, tol=None, env=None, max_iter=None):
    """CTMRG (cold unless env given) + readout.  Returns (obs dict, env)."""
    a = _ct.double_layers(st)
    if tol is None:
        env, it, delta = _ct.ctmrg(a, params.chi, env=env, max_iter=ctm_iters)
    else:
        env, it, delta = _ct.ctmrg(a, params.chi, env=env,
                                   max_iter=max_iter or 2000, tol=tol)
    obs = _ct.observe(st, env, params.d_A)
    obs["ctm_iters"] = it
    obs["ctm_delta"] = delta
    obs["eps"] = np.array([st["eps"][s] for s in _pp.SITES])
    obs["corner_spectra"] = _ct.corner_spectra(env, params.chi)
    obs["bond_spectra"] = _pp.bond_spectra(st)
    return obs, env


def run_job(params, n_steps, observe_at, ctm_iters=10, tol=None, max_iter=None,
            state=None, callback=None):
    """Evolve from Néel ⊗ |+> (or ``state``) and observe at the listed steps.

    observe_at: iterable of step counts (0 = initial state).  Every
    observation starts CTMRG cold.  Returns a list of observation dicts with
    't' and 'step' added.
    """
    st = _pp.new_state(params) if state is None else _pp.copy_state(state)
    observe_at = sorted(set(int(s) for s in observe_at))
    out = []
    for step in range(0, n_steps + 1):
        if step > 0:
            _pp.trotter_step(st, params)
        if step in observe_at:
            obs, _ = observe_state(st, params, ctm_iters=ctm_iters, tol=tol,
                                   max_iter=max_iter)
            obs["step"] = step
            obs["t"] = step * params.dt
            out.append(obs)
            if callback is not None:
                callback(obs)
    return out, st
