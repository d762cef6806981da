"""Stability of plain BGK against the Knudsen-number-based BGK on the
supersonic NACA0012 flow (Sec. 4).

The paper reports that plain BGK with the equilibrium of Eq.
(eq:discrete-equilibrium) stays stable up to Mach 1.2 and Reynolds 7500 on
this flow, and that the relaxation factor alpha(eps) of Eq. (eq:alpha) is what
takes it to Mach 1.5 at Reynolds 1e4.  This sweeps (Ma, Re) with alpha(eps)
off and on, on the airfoil set-up of ``precision_study.airfoil_case``, and
reports for each run whether it stayed finite and how many cell updates found
no equilibrium (in the first and second halves of the run).

    python -m paper_1910_13515_amd.stability_map [--steps 10000] [--scale 1] [--storage fp64]
        [--grid 1.5:7500,1.5:1e9] [--relax both|plain|eps]

Prints one JSON object.
"""
from __future__ import annotations

import argparse
import json
import sys

import numpy as np

from . import lbm, precision_study

GRID = [(1.2, 7500.0), (1.2, 1e4), (1.5, 7500.0), (1.5, 1e4)]


def run_case(mach, reynolds, kn_relax, steps, scale, storage, chunk=250, log=None):
    import torch
    shape, solid, kw = precision_study.airfoil_case(scale, mach)
    kw = dict(kw, reynolds=reynolds, kn_relax=kn_relax)
    s = lbm.Solver(shape, solid=solid, storage=storage, **kw)
    tau = s.info().tau
    failed = [0, 0]
    done = 0
    finite = True
    while done < steps:
        k = min(chunk, steps - done)
        st, code = lbm.lbm_step(s.ctx, k, with_stats=True)
        failed[0 if done < steps // 2 else 1] += int(st.failed)
        done += k
        _, tot = s.moments(fields=False)
        if not np.all(np.isfinite(tot)):
            finite = False
            break
        # more than 0.1% of the chunk's updates without equilibrium, past the
        # start-up: the flow keeps leaving the lattice's range (and each such
        # update runs the full cold-restart Newton); stop there
        if log:
            log(f"Ma {mach} Re {reynolds:g} alpha(eps) {'on' if kn_relax else 'off'}: {done} steps, "
                f"failed updates {failed[0] + failed[1]}")
        if done > steps // 4 and st.failed > 1e-3 * k * np.prod(shape):
            break
    s.close()
    del s
    torch.cuda.empty_cache()
    return {"mach": mach, "reynolds": reynolds, "kn_relax": kn_relax, "tau": tau, "steps_run": done,
            "finite": finite, "failed_first_half": failed[0], "failed_second_half": failed[1],
            "stable": finite and done == steps and failed[1] == 0}


def sweep(steps=10000, scale=1.0, storage="fp64", grid=GRID, log=None, relax=(False, True)):
    out = []
    for mach, re in grid:
        for kn in relax:
            r = run_case(mach, re, kn, steps, scale, storage, log=log)
            if log:
                log(json.dumps(r))
            out.append(r)
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--steps", type=int, default=10000)
    ap.add_argument("--scale", type=float, default=1.0)
    ap.add_argument("--storage", default="fp64", choices=["fp64", "fp32s", "fp16s"])
    ap.add_argument("--grid", default=None, help="Ma:Re pairs, comma-separated (default: the four of the sweep)")
    ap.add_argument("--relax", default="both", choices=["both", "plain", "eps"],
                    help="plain BGK, BGK with alpha(eps), or both for every (Ma, Re)")
    args = ap.parse_args()
    relax = {"both": (False, True), "plain": (False,), "eps": (True,)}[args.relax]
    grid = GRID if not args.grid else [tuple(float(v) for v in g.split(":")) for g in args.grid.split(",")]
    import torch
    if not torch.cuda.is_available():
        raise SystemExit("the stability map needs a GPU")
    torch.cuda.set_device(0)
    res = sweep(args.steps, args.scale, args.storage, grid, log=lambda m: print("#", m, file=sys.stderr, flush=True),
                relax=relax)
    print(json.dumps({"case": "airfoil", "scale": args.scale, "steps": args.steps, "storage": args.storage,
                      "T_ref": precision_study.T_OBSTACLE, "runs": res}), flush=True)


if __name__ == "__main__":
    main()
