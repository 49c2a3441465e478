"""Write oracle reference values for the plain FP64 workload (D=4, chi=32).

    python tests/golden/make_plain_golden.py W V [--max-iter N]

Calls only oracle/ (and synthetic/ for the parameters): evolves Néel ⊗ |+>
with dt=0.05 for 100 steps and, every 10 steps, runs CTMRG from a cold start
until the corner spectra change by less than 1e-10 in one iteration (capped at
--max-iter), then records the imbalance, occupations, truncation errors,
corner spectra and bond spectra to tests/golden/plain_W{W}_V{V}.json.

    python tests/golden/make_plain_golden.py W V --extend CAP

reruns, from the same trajectory, the observations of an existing file whose
CTMRG stopped at the cap above the tolerance, now with cap CAP, and records
each observation's cap as "max_iter" (converged observations are kept).

    python tests/golden/make_plain_golden.py W V --spread

adds to an existing file the oracle's own rounding sensitivity along the
trajectory: the simple update is run a second time from the same start with
every element of Gamma scaled by (1 + 1e-15 r), r standard normal (seeded),
and the largest bond-spectrum difference at each observation step is stored
as "su_spread" (the simple update's amplification of one rounding).
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import peps, run  # noqa: E402
from oracle.model import Params  # noqa: E402
import synthetic  # noqa: E402


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("W", type=float)
    ap.add_argument("V", type=float)
    ap.add_argument("--max-iter", type=int, default=200)
    ap.add_argument("--spread", action="store_true")
    ap.add_argument("--extend", type=int, default=0)
    args = ap.parse_args()
    cfg = [c for c in synthetic.plain_configs() if c["W"] == args.W and c["V"] == args.V][0]
    p = Params(D=cfg["D"], chi=cfg["chi"], J=cfg["J"], V=cfg["V"], W=cfg["W"], dt=cfg["dt"])
    out = {"config": cfg, "max_iter": args.max_iter, "tol": cfg["ctm_tol"], "obs": []}
    path = os.path.join(ROOT, "tests", "golden", f"plain_W{args.W:g}_V{args.V:g}.json")
    if args.spread:
        add_spread(path, p, cfg)
        return
    if args.extend:
        extend(path, p, cfg, args.extend)
        return
    st = peps.new_state(p)
    for step in range(0, cfg["n_steps"] + 1):
        if step > 0:
            peps.trotter_step(st, p)
        if step % cfg["observe_every"]:
            continue
        t0 = time.time()
        o, _ = run.observe_state(st, p, tol=cfg["ctm_tol"], max_iter=args.max_iter)
        out["obs"].append({"step": step, "imbalance": o["imbalance"], "n": o["n"].tolist(),
                           "eps": o["eps"].tolist(), "ctm_iters": o["ctm_iters"],
                           "ctm_delta": o["ctm_delta"],
                           "corner_spectra": o["corner_spectra"].tolist(),
                           "bond_spectra": o["bond_spectra"].tolist()})
        print(f"step {step} I={o['imbalance']:.12f} iters={o['ctm_iters']} "
              f"delta={o['ctm_delta']:.2e} ({time.time() - t0:.0f}s)", flush=True)
        with open(path, "w") as f:
            json.dump(out, f)


def extend(path, p, cfg, cap):
    with open(path) as f:
        out = json.load(f)
    obs = {o["step"]: o for o in out["obs"]}
    for o in out["obs"]:
        o.setdefault("max_iter", out["max_iter"])
    st = peps.new_state(p)
    for step in range(0, cfg["n_steps"] + 1):
        if step > 0:
            peps.trotter_step(st, p)
        o = obs.get(step)
        if o is None or o["ctm_delta"] < out["tol"]:
            continue
        t0 = time.time()
        n, _ = run.observe_state(st, p, tol=cfg["ctm_tol"], max_iter=cap)
        o.update({"imbalance": n["imbalance"], "n": n["n"].tolist(), "eps": n["eps"].tolist(),
                  "ctm_iters": n["ctm_iters"], "ctm_delta": n["ctm_delta"],
                  "corner_spectra": n["corner_spectra"].tolist(),
                  "bond_spectra": n["bond_spectra"].tolist(), "max_iter": cap})
        print(f"step {step} I={n['imbalance']:.12f} iters={n['ctm_iters']} "
              f"delta={n['ctm_delta']:.2e} ({time.time() - t0:.0f}s)", flush=True)
        with open(path, "w") as f:
            json.dump(out, f)


def add_spread(path, p, cfg):
    import numpy as np

    with open(path) as f:
        out = json.load(f)
    a, b = peps.new_state(p), peps.new_state(p)
    rng = np.random.default_rng(2019)
    for s in peps.SITES:
        g = b["gam"][s]
        b["gam"][s] = g * (1 + 1e-15 * rng.normal(size=g.shape))
    spread = {}
    for step in range(0, cfg["n_steps"] + 1):
        if step > 0:
            peps.trotter_step(a, p)
            peps.trotter_step(b, p)
        if step % cfg["observe_every"] == 0:
            spread[step] = float(np.max(np.abs(peps.bond_spectra(a) - peps.bond_spectra(b))))
            print(f"step {step} su_spread {spread[step]:.2e}", flush=True)
    for o in out["obs"]:
        o["su_spread"] = spread[o["step"]]
    with open(path, "w") as f:
        json.dump(out, f)


if __name__ == "__main__":
    main()
