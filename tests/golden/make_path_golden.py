"""Write oracle reference values for the device paths that run only at large n.

    python tests/golden/make_path_golden.py NAME [NAME ...]
    python tests/golden/make_path_golden.py --list

Calls only oracle/ (and synthetic/ for the inputs).  Each case runs on a
state of the sizes the headline and serving workloads use, where the device
takes paths that smaller tests never reach: 128 x 128 GEMM tiles for the
enlarged corners and the T update, cut matrices applied through their four
enlarged-corner factors (n > 1024), K split over workgroups, and subspace
blocks wider than 128 columns.  Paper passages: appendix (D = 4, 5 with
chi >= D^2, a converged environment); Results (the readout of n and the
imbalance).

Two kinds of case:
  random  seeded random site tensors and bond weights (full rank on every
          bond, synthetic.random_state), model W=8, V=1, dt=0.05.  CTMRG from
          a cold start until the corner spectra change by less than tol in
          one iteration (capped; tol = 0: exactly max_iter iterations),
          readout; one Trotter step; CTMRG from a cold start again, readout.
          Random states have short correlation lengths, so both environments
          converge and their corner spectra are compared entry by entry.
  neel    the headline model (D=6, chi=72, W=8, V=1, dt=0.05) from Néel ⊗ |+>
          for n_steps Trotter steps, then ctm_iters CTMRG iterations from a
          cold start and a readout (the throughput schedule's observation,
          the oracle's full SVDs against the device's subspace iteration).

Each observation stores the imbalance, occupations, Rényi entropies,
truncation errors, bond spectra, the CTMRG iteration count and last change,
and the normalised corner spectra; tests/golden/path_NAME.json.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

from oracle import peps, run  # noqa: E402
from oracle.model import Params  # noqa: E402
import synthetic  # noqa: E402

MODEL = dict(J=1.0, V=1.0, W=8.0, dt=0.05)

CASES = {
    # n = 625: formed cut matrices, subspace block k = 41
    "D5_chi25": dict(kind="random", D=5, chi=25, seed=51, tol=1e-10, max_iter=120),
    # n = 1296: factored cut matrices, 128 x 128 enlarged-corner tiles, split K
    "D6_chi36": dict(kind="random", D=6, chi=36, seed=61, tol=1e-10, max_iter=120),
    # n = 972: subspace block k = 144 in FP64 (> 128: the wide Cholesky and
    # Jacobi variants)
    "D3_chi108": dict(kind="random", D=3, chi=108, seed=31, tol=1e-10, max_iter=120),
    # the headline sizes, n = 2592: a fixed 8 cold iterations (the oracle
    # takes about 400 s per iteration here)
    "D6_chi72": dict(kind="random", D=6, chi=72, seed=62, tol=0.0, max_iter=8),
    "D6_chi72_neel10": dict(kind="neel", D=6, chi=72, n_steps=10, ctm_iters=10),
}


def _record(o, step):
    return {"step": step, "imbalance": o["imbalance"], "n": o["n"].tolist(),
            "renyi1": o["renyi1"].tolist(), "renyi_half": o["renyi_half"].tolist(),
            "eps": o["eps"].tolist(), "ctm_iters": int(o["ctm_iters"]),
            "ctm_delta": float(o["ctm_delta"]),
            "corner_spectra": o["corner_spectra"].tolist(),
            "bond_spectra": o["bond_spectra"].tolist()}


def make(name):
    c = CASES[name]
    p = Params(D=c["D"], chi=c["chi"], **MODEL)
    out = {"name": name, "case": c, "model": MODEL, "obs": []}
    path = os.path.join(ROOT, "tests", "golden", f"path_{name}.json")
    t0 = time.time()
    if c["kind"] == "random":
        gam, lam = synthetic.random_state(c["seed"], c["D"])
        st = peps.new_state(p)
        for i, s in enumerate(peps.SITES):
            st["gam"][s] = np.array(gam[i], dtype=complex)
            st["lam_h"][s] = np.array(lam[i], dtype=float)
            st["lam_v"][s] = np.array(lam[4 + i], dtype=float)
        for step in (0, 1):
            if step:
                peps.trotter_step(st, p)
            o, _ = run.observe_state(st, p, tol=c["tol"], max_iter=c["max_iter"])
            out["obs"].append(_record(o, step))
            print(f"{name} step {step}: I={o['imbalance']:.12f} iters={o['ctm_iters']} "
                  f"delta={o['ctm_delta']:.2e} ({time.time() - t0:.0f} s)", flush=True)
    else:
        st = peps.new_state(p)
        for _ in range(c["n_steps"]):
            peps.trotter_step(st, p)
        o, _ = run.observe_state(st, p, ctm_iters=c["ctm_iters"])
        out["obs"].append(_record(o, c["n_steps"]))
        print(f"{name} step {c['n_steps']}: I={o['imbalance']:.12f} delta={o['ctm_delta']:.2e} "
              f"({time.time() - t0:.0f} s)", flush=True)
    with open(path, "w") as f:
        json.dump(out, f)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("names", nargs="*")
    ap.add_argument("--list", action="store_true")
    args = ap.parse_args()
    if args.list or not args.names:
        print("\n".join(CASES))
        return
    for n in args.names:
        make(n)


if __name__ == "__main__":
    main()
