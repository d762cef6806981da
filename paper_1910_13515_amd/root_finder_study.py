"""Newton-Raphson against the secant root finder (the choice of root-finding
algorithm that Sec. 6 leaves open), on the GPU in FP64.

For each case both solvers run the same steps from the same initial state;
reported per solver: throughput, root-finder updates per cell update, cells
without equilibrium, the alpha(eps) branch shares of the last step, and the
difference of the end states (relative L2 of rho, u, T over fluid cells).

    python -m paper_1910_13515_amd.root_finder_study [--cases tgv,airfoil] [--steps 200] [--scale 1]

Prints one JSON object.
"""
from __future__ import annotations

import argparse
import json
import sys
import time

import numpy as np

from . import lbm, precision_study


def run(case: str, solver: str, steps: int, scale: float, log=None):
    import torch
    make = {"tgv": precision_study.tgv_case, "airfoil": precision_study.airfoil_case,
            "sphere": precision_study.sphere_case}[case]
    shape, solid, kw = make(scale)
    s = lbm.Solver(shape, solid=solid if solid.any() else None, storage="fp64", root_finder=solver, **kw)
    info = s.info()
    s.step(10)  # past the first steps from the initial equilibrium
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    st = s.step(steps, stats=True)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    last = s.step(1, stats=True)
    fields, tot = s.moments()
    s.close()
    torch.cuda.empty_cache()
    upd = max(1, st.cell_updates)
    res = {"solver": solver, "glups": info.cells * steps / dt / 1e9, "ms_per_step": 1e3 * dt / steps,
           "updates_per_cell": st.iterations / upd, "max_updates": int(st.max_iterations),
           "failed_cell_updates": int(st.failed), "cold_restarts": int(st.cold_restarts),
           "alpha_fraction_last_step": [a / max(1, last.cell_updates) for a in last.alpha_hist],
           "finite": bool(np.all(np.isfinite(tot)))}
    if log:
        log(f"{case} {solver}: {res['glups']:.3f} GLUPS, {res['updates_per_cell']:.2f} updates per cell")
    return fields, solid.reshape(-1) == 0, res


def study(cases=("tgv", "airfoil"), steps=200, scale=1.0, log=None):
    out = {"steps": steps, "scale": scale, "storage": "fp64", "cases": {}}
    for case in cases:
        f_n, fluid, r_n = run(case, "newton", steps, scale, log)
        f_s, _, r_s = run(case, "secant", steps, scale, log)
        diff = precision_study.errors(f_s, f_n, fluid)
        out["cases"][case] = {"newton": r_n, "secant": r_s, "secant_vs_newton": diff,
                              "time_ratio": r_s["ms_per_step"] / r_n["ms_per_step"]}
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--cases", default="tgv,airfoil")
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--scale", type=float, default=1.0)
    args = ap.parse_args()
    import torch
    if not torch.cuda.is_available():
        raise SystemExit("the study needs a GPU")
    torch.cuda.set_device(0)
    res = study(args.cases.split(","), args.steps, args.scale, log=lambda m: print("#", m, file=sys.stderr,
                                                                                    flush=True))
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
