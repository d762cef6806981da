"""Knudsen sensor and Newton iteration fields of the supersonic airfoil.

Sec. 4 of the paper maps the sensor eps (Eq. eq:DeltaAvg) and the Newton
iterations per cell around the NACA0012 at Ma 1.5, Re 1e4 (Fig.
naca-knudsen).  It reports that eps is active only near the shocks, the
airfoil and the wake, and that the solver needs at most four iterations, fewer
than two on average, and none over wide areas.  This runs the full-size case
in FP64 (the paper's tolerance, 1e-12), takes lbm_diagnostics of the next
step, and reports those statistics:

* the histogram of Newton updates per updated cell (fluid, off the frozen
  face layers), their mean and maximum;
* the share of those cells in each alpha branch (eps < 0.01, < 0.1, < 1, >= 1);
* where the sensor is active: the share of cells with eps >= 0.01 that lie
  within a distance of the airfoil, and the x extent of the active region.

    python -m paper_1910_13515_amd.knudsen_map [--steps 20000] [--scale 1] [--png out.png]

Prints one JSON object; with --png also writes the two maps (log10 eps and
iterations) next to each other.
"""
from __future__ import annotations

import argparse
import json
import sys

import numpy as np

from . import lbm, precision_study


def run(steps=20000, scale=1.0, storage="fp64", chunk=1000, log=None, shift_ref=0, newton_tol=0.0, kn_relax=True):
    import torch
    shape, solid, kw = precision_study.airfoil_case(scale)
    kw = dict(kw, kn_relax=kn_relax)
    s = lbm.Solver(shape, solid=solid, storage=storage, shift_ref=shift_ref, newton_tol=newton_tol, **kw)
    done = 0
    while done < steps:
        k = min(chunk, steps - done)
        s.step(k)
        done += k
        if log:
            log(f"{done}/{steps} steps")
    torch.cuda.synchronize()
    eps, iters = s.diagnostics()
    s.close()
    return shape, solid, eps, iters


def summarize(shape, solid, eps, iters, near=8.0):
    nx, ny, _ = shape
    # updated cells: fluid and off the frozen face layers (iterations -1 there)
    fluid = (solid.reshape(-1) == 0) & (iters >= 0)
    it = iters[fluid]
    e = eps[fluid]
    ok = np.isfinite(e)  # NaN: no equilibrium found (the cell is not collided)
    fin = ok
    hist = [int(np.sum(it[ok] == k)) for k in range(5)] + [int(np.sum(it[ok] >= 5))]
    thr = np.array([1e-2, 1e-1, 1.0])
    br = np.digitize(e[fin], thr)
    # distance of every cell to the nearest solid cell (exact, on the 2-D grid)
    from scipy import ndimage
    dist = ndimage.distance_transform_edt(solid.reshape(ny, nx) == 0).reshape(-1)[fluid]
    active = fin & (e >= 1e-2)
    xall = (np.arange(nx * ny) % nx)[fluid]
    xs = xall[active]
    # the free stream ahead of the bow shock: the first 40% of the domain
    # (the leading edge sits at half its length)
    upstream = fin & (xall < 0.4 * nx)
    return {
        "updated_cells": int(fluid.sum()),
        "newton_updates": {"histogram_0_to_4_and_more": hist, "mean": float(it[ok].mean()), "max": int(it[ok].max()),
                           "share_zero": float(np.mean(it[ok] == 0)), "cells_without_equilibrium": int(np.sum(~ok))},
        "alpha_branch_share": [float(np.mean(br == k)) for k in range(4)],
        "upstream_share_alpha_above_1": float(np.mean(e[upstream] >= 1e-2)) if upstream.any() else 0.0,
        "sensor": {"share_active": float(active.mean()),
                   f"share_of_active_within_{near:g}_cells_of_the_airfoil": float(np.mean(dist[active] <= near))
                   if active.any() else 0.0,
                   "active_x_range": [int(xs.min()), int(xs.max())] if active.any() else None,
                   "eps_percentiles_50_90_99": [float(v) for v in np.percentile(e[fin], [50, 90, 99])]},
    }


def save_png(path, shape, solid, eps, iters):
    import matplotlib
    matplotlib.use("Agg")
    import matplotlib.pyplot as plt
    nx, ny, _ = shape
    m = solid.reshape(ny, nx) != 0
    le = np.log10(np.maximum(eps.reshape(ny, nx), 1e-8))
    le[m] = np.nan
    it = iters.reshape(ny, nx).astype(float)
    it[m] = np.nan
    fig, ax = plt.subplots(1, 2, figsize=(14, 4))
    a = ax[0].imshow(le, origin="lower", cmap="viridis", vmin=-6, vmax=0)
    ax[0].set_title("log10 eps")
    fig.colorbar(a, ax=ax[0])
    b = ax[1].imshow(it, origin="lower", cmap="magma", vmin=0, vmax=4)
    ax[1].set_title("Newton updates")
    fig.colorbar(b, ax=ax[1])
    fig.tight_layout()
    fig.savefig(path, dpi=100)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--steps", type=int, default=20000)
    ap.add_argument("--scale", type=float, default=1.0)
    ap.add_argument("--storage", default="fp64", choices=["fp64", "fp32s", "fp16s"])
    ap.add_argument("--png", default=None)
    ap.add_argument("--shift-ref", type=int, default=0, choices=[0, 1],
                    help="reduced precision: deviations from the rest weights (0) or the free stream (1)")
    ap.add_argument("--save", default=None, help="write eps and iterations per cell to this .npz")
    ap.add_argument("--newton-tol", type=float, default=0.0, help="0: the library default of the storage mode")
    ap.add_argument("--plain-bgk", action="store_true", help="alpha(eps) off (the sensor is still reported)")
    args = ap.parse_args()
    import torch
    if not torch.cuda.is_available():
        raise SystemExit("the map needs a GPU")
    torch.cuda.set_device(0)
    shape, solid, eps, iters = run(args.steps, args.scale, args.storage,
                                   log=lambda m: print("#", m, file=sys.stderr, flush=True), shift_ref=args.shift_ref,
                                   newton_tol=args.newton_tol, kn_relax=not args.plain_bgk)
    res = {"case": "airfoil", "storage": args.storage, "shift_ref": args.shift_ref, "newton_tol": args.newton_tol,
           "kn_relax": not args.plain_bgk,
           "steps": args.steps,
           "scale": args.scale, **summarize(shape, solid, eps, iters)}
    if args.save:
        np.savez_compressed(args.save, eps=eps, iters=iters)
    if args.png:
        save_png(args.png, shape, solid, eps, iters)
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
