"""The paper's validity monitors on top of the device path (section Results).

* the D-versus-(D+1) stopping rule: the same parameters are evolved at two
  bond dimensions and the evolution is trusted up to the first observation
  where their imbalances disagree by more than a tolerance;
* the local truncation error of each site and the Renyi entropies S_1,
  S_1/2 of the one-site physical matrix, which every observation carries
  (their distance from ln 2 indicates how far the state is from saturation).

Both jobs run concurrently through the request loop (solve_submit /
solve_poll); nothing here computes on the host beyond comparing the two
returned series.
"""
import time

from . import native


def compare_bond_dimensions(D, chi_of_D, n_steps, observe_every, ctm_iters, tol=1e-2,
                            timeout=3600.0, **params):
    """Evolve at D and D+1 (chi = chi_of_D(D)); return a dict with both
    observation series and `t_stop`, the time of the first observation where
    |I_D - I_{D+1}| > tol (None if they agree throughout)."""
    srv = native.Server(hbm_budget=0, max_slots=2)
    try:
        ids = [srv.submit(native.make_config(d, chi_of_D(d), **params), n_steps=n_steps,
                          observe_every=observe_every, ctm_iters=ctm_iters) for d in (D, D + 1)]
        series = {}
        t0 = time.time()
        while len(series) < 2:
            for d, j in zip((D, D + 1), ids):
                if d not in series:
                    res = srv.poll(j)[1]
                    if res is not None:
                        series[d] = res
            if time.time() - t0 > timeout:
                raise TimeoutError("bond-dimension comparison did not finish")
            time.sleep(0.01)
    finally:
        srv.close()
    t_stop = None
    for a, b in zip(series[D], series[D + 1]):
        if abs(a["imbalance"] - b["imbalance"]) > tol:
            t_stop = a["t"]
            break
    return {"series": series, "t_stop": t_stop, "tol": tol}
