"""Reduced-precision storage against the FP64 GPU step on two obstacle
flows: the supersonic NACA0012 airfoil of Sec. 4 and a sphere in a
supersonic channel.

Each case is run once per storage mode from the same initial state (uniform
free stream) and the same parameters; the fields (rho, u, T) at the end are
compared with the FP64 run over the fluid cells:

    e_rho = ||rho_m - rho_64||_2 / ||rho_64||_2      (likewise T)
    e_u   = ||u_m - u_64||_2 / ||u_64||_2            (all three components)

plus the maximum absolute differences.  Newton statistics and the histogram of
the relaxation factor alpha(eps) of one further step are reported per mode.

    python -m paper_1910_13515_amd.precision_study --case airfoil [--steps 20000] [--scale 1]
    python -m paper_1910_13515_amd.precision_study --case sphere  [--steps 2000]  [--scale 1] [--mach 1.5]
    python -m paper_1910_13515_amd.precision_study --case tgv     [--steps 1000]  [--mach 0.5] [--plain-bgk]
    python -m paper_1910_13515_amd.precision_study --case airfoil --average 5000 --modes fp64,fp64:1e-13,fp32s

``--average N`` compares time averages over the last N steps instead of end
states (a chaotic wake makes end states of two correct runs differ by as much
as round-off lets them), with the bow shock's position on a few rows ahead of
the body and the alpha(eps) branch shares over the window.

``--scale`` shrinks the domain and the body together (for quick checks).
``--plain-bgk`` turns the Knudsen-dependent relaxation off in every mode, so
that its share in the reduced-precision error can be read off.  ``--every N``
runs the modes side by side instead and reports their errors against FP64
every N steps (the error's course in time).
Prints one JSON object.
"""
from __future__ import annotations

import argparse
import json
import sys
import time

import numpy as np

from . import inputs, lbm

EQ, NEU, PER = lbm.LBM_FACE_EQUILIBRIUM, lbm.LBM_FACE_NEUMANN, lbm.LBM_FACE_PERIODIC


# Reference temperature of both obstacle flows: 2/3, the temperature the
# D3Q39 quadrature is built around.  The paper does not state its lattice
# temperature; with 0.5 (or 0.6, 0.75) the expansion over the airfoil leaves
# the range of (u, T) for which the 13-moment equilibrium exists on this
# lattice, and the run diverges.
T_OBSTACLE = 2.0 / 3.0


def airfoil_case(scale: float = 1.0, mach: float = 1.5):
    """2048 x 1024 x 1, chord 256 with the leading edge at the domain centre,
    Ma 1.5, Re 1e4 on the chord; free-stream equilibrium on the x and y
    faces, z periodic (Sec. 4, supersonic airfoil)."""
    nx, ny = int(round(2048 * scale)), int(round(1024 * scale))
    chord = 256.0 * scale
    solid = inputs.naca_symmetric_mask(nx, ny, 1, chord, 0.12, leading_edge=(nx / 2.0, ny / 2.0))
    kw = dict(gamma=1.4, mach=mach, reynolds=1e4, length_ref=chord, T_ref=T_OBSTACLE, u_dir=(1.0, 0.0, 0.0),
              kn_relax=True, faces=(EQ, EQ, EQ, EQ, PER, PER))
    return (nx, ny, 1), solid, kw


def sphere_case(scale: float = 1.0, mach: float = 1.5):
    """512 x 256 x 256 channel, sphere of radius 24 centred at (128, 128, 128),
    uniform inflow, Re 1e4 on the diameter; equilibrium inflow and far-field
    faces, Neumann outflow.  Mach 1.5 by default: at Mach 2 the flow around
    the sphere leaves the range where the D3Q39 13-moment equilibrium exists
    (in FP64 as well), so a Mach 2 run reports Newton failures and diverges."""
    nx, ny, nz = (int(round(v * scale)) for v in (512, 256, 256))
    r = 24.0 * scale
    solid = inputs.sphere_mask(nx, ny, nz, (128.0 * scale, ny / 2.0, nz / 2.0), r)
    kw = dict(gamma=1.4, mach=mach, reynolds=1e4, length_ref=2.0 * r, T_ref=T_OBSTACLE, u_dir=(1.0, 0.0, 0.0),
              kn_relax=True, faces=(EQ, NEU, EQ, EQ, EQ, EQ))
    return (nx, ny, nz), solid, kw


def tgv_case(scale: float = 1.0, mach: float = 0.5):
    """The benchmark's workload: periodic 128^3 compressible Taylor-Green
    vortex at Ma 0.5, Re 1600, uniform T 0.5 (no obstacle; the mask is
    empty).  The initial fields go in through ``fields``."""
    n = int(round(128 * scale))
    gamma, T0 = 1.4, 0.5
    U = mach * np.sqrt(gamma * T0)
    kw = dict(gamma=gamma, mach=mach, reynolds=1600.0, length_ref=n / (2 * np.pi), T_ref=T0, u_dir=(1.0, 0.0, 0.0),
              kn_relax=True, fields=inputs.taylor_green_fields(n, U, T0))
    return (n, n, n), np.zeros(n ** 3, dtype=np.uint8), kw


CASES = {"airfoil": (airfoil_case, ("fp64", "fp32s"), 20000),
         "sphere": (sphere_case, ("fp64", "fp32s", "fp16s", "fp16s@stream"), 2000),
         "tgv": (tgv_case, ("fp64", "fp32s", "fp16s"), 1000)}


def parse_mode(mode: str):
    """(storage, shift_ref, newton_tol) of a mode string "storage[@stream][:tol]".
    "@stream" stores deviations from the free stream's equilibrium instead of
    the rest weights (shift_ref = 1); ":tol" overrides the Newton threshold
    (0 = the storage mode's default)."""
    base, _, tol = mode.partition(":")
    storage, _, ref = base.partition("@")
    if storage not in lbm.STORAGE or ref not in ("", "stream"):
        raise ValueError(f"unknown mode {mode!r}")
    if ref == "stream" and storage == "fp64":
        raise ValueError("the stream shift applies to the shifted storage modes only")
    return storage, int(ref == "stream"), float(tol) if tol else 0.0


def shock_front(rho, shape, x_end: int, y: int, z: int = 0, rho_inf: float = 1.0) -> float:
    """x of the bow shock on the grid row (y, z), scanned over x < x_end:
    going downstream from the inflow, where the density first reaches halfway
    between the free-stream value and the row's maximum over the scan (the
    shock's mid-point), interpolated linearly between cells.  NaN when the
    row has no such rise."""
    nx, ny, nz = shape
    row = np.asarray(rho).reshape(nz, ny, nx)[z, y, :x_end]
    if row.size < 2:
        return float("nan")
    half = rho_inf + 0.5 * (row.max() - rho_inf)
    idx = np.nonzero(row >= half)[0]
    if idx.size == 0 or idx[0] == 0 or row.max() <= rho_inf * 1.01:
        return float("nan")
    i = int(idx[0])
    return float(i - 1 + (half - row[i - 1]) / (row[i] - row[i - 1]))


def front_rows(case: str, shape, scale: float):
    """(x of the body's front, [(label, y, z, x_end), ...]): the rows on which
    the bow shock is located, each scanned up to x_end.  Airfoil: the
    stagnation row up to the leading edge, rows an eighth and a quarter chord
    off it up to half a chord further (the shock bends back away from the
    axis).  Sphere: rows 0, r/2 and r off the axis, each up to where it meets
    the sphere."""
    nx, ny, nz = shape
    if case == "airfoil":
        c = 256.0 * scale
        x0 = int(np.floor(nx / 2.0))
        offs = [("stagnation", 0, x0), ("+c/8", int(round(c / 8)), x0 + int(c / 2)),
                ("-c/8", -int(round(c / 8)), x0 + int(c / 2)), ("+c/4", int(round(c / 4)), x0 + int(c / 2)),
                ("-c/4", -int(round(c / 4)), x0 + int(c / 2))]
        return x0, [(lab, ny // 2 + d, 0, xe) for lab, d, xe in offs]
    if case == "sphere":
        r = 24.0 * scale
        x0 = int(np.floor(128.0 * scale - r))
        xc = int(np.floor(128.0 * scale))
        # each row up to the sphere's surface on it (where the row meets it)
        offs = [(lab, d, int(np.floor(xc - np.sqrt(max(r * r - d * d, 0.0)))))
                for lab, d in (("stagnation", 0), ("+r/2", int(round(r / 2))), ("-r/2", -int(round(r / 2))),
                               ("+r", int(round(r))), ("-r", -int(round(r))))]
        return x0, [(lab, ny // 2 + d, nz // 2, xe) for lab, d, xe in offs]
    return None, []


def run(shape, solid, kw, storage, steps, chunk=1000, log=None, average=0, sample=50):
    """Runs one mode (see parse_mode); returns (fields[5, N], summary).

    With ``average`` > 0 the fields returned are the time averages of
    (rho, u, T) over the last ``average`` steps, sampled every ``sample``
    steps, and the summary carries the alpha(eps) branch shares over that
    window; otherwise they are the end state."""
    import torch
    mode = storage
    storage, shift_ref, tol = parse_mode(mode)
    s = lbm.Solver(shape, solid=solid if solid.any() else None, storage=storage, shift_ref=shift_ref,
                   **dict(kw, newton_tol=tol))
    info = s.info()
    t0 = time.perf_counter()
    failed = 0
    done = 0
    start_avg = steps - average if average > 0 else steps + 1
    acc, nacc, alpha_win, upd_win = None, 0, np.zeros(4), 0
    stepping = 0.0
    while done < steps:
        k = min(chunk, steps - done)
        if done >= start_avg:
            k = min(k, sample)
        elif done + k > start_avg:
            k = start_avg - done
        ts = time.perf_counter()
        st = s.step(k, stats=True)
        torch.cuda.synchronize()
        stepping += time.perf_counter() - ts
        failed += st.failed
        done += k
        if done > start_avg:
            alpha_win += np.array(st.alpha_hist[:4], dtype=np.float64)
            upd_win += st.cell_updates
            f, _ = s.moments()
            acc = f.copy() if acc is None else acc + f
            nacc += 1
        if log and (done % chunk == 0 or done == steps):
            log(f"{mode}: {done}/{steps} steps, Newton failures so far {failed}")
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    st = s.step(1, stats=True)  # statistics of one further step
    failed += st.failed
    fields, tot = s.moments()
    s.close()
    del s
    torch.cuda.empty_cache()
    upd = max(1, st.cell_updates)
    summary = {
        "storage": storage, "shift": "free stream" if shift_ref else "rest weights", "newton_tol": tol,
        "tau": info.tau, "seconds": dt, "glups": info.cells * steps / stepping / 1e9,
        "newton_failures": int(failed), "newton_iterations_per_cell": st.iterations / upd,
        "newton_max_iterations": int(st.max_iterations),
        "alpha_fraction": [a / upd for a in st.alpha_hist], "totals": [float(v) for v in tot],
        "finite": bool(np.all(np.isfinite(tot))),
    }
    if nacc:
        fields = acc / nacc
        summary["window"] = {"steps": average, "samples": nacc,
                             "alpha_fraction": (alpha_win / max(1, upd_win)).tolist()}
    return fields, summary


def errors(f, ref, fluid):
    """Relative L2 and max-abs differences of rho, u, T over fluid cells."""
    out = {}
    for name, rows in (("rho", [0]), ("u", [1, 2, 3]), ("T", [4])):
        a, b = f[rows][:, fluid], ref[rows][:, fluid]
        d = a - b
        out[f"l2_{name}"] = float(np.sqrt(np.sum(d * d)) / np.sqrt(np.sum(b * b)))
        out[f"max_{name}"] = float(np.max(np.abs(d)))
    return out


def curve(case: str, every: int, steps: int | None = None, scale: float = 1.0, modes=None, mach: float | None = None,
          log=None, plain_bgk: bool = False):
    """All modes side by side from the same state: the relative L2 errors of
    (rho, u, T) against FP64 every `every` steps, with the rms speed of the
    FP64 field.  Returns {"columns": [...], "rows": [[step, ...], ...]}."""
    import torch
    make, default_modes, default_steps = CASES[case]
    steps = default_steps if steps is None else steps
    modes = [m for m in (default_modes if modes is None else modes) if m != "fp64"]
    shape, solid, kw = make(scale) if mach is None else make(scale, mach)
    if plain_bgk:
        kw = dict(kw, kn_relax=False)
    fluid = solid.reshape(-1) == 0
    mask = solid if solid.any() else None
    solvers = {"fp64": lbm.Solver(shape, solid=mask, storage="fp64", **kw)}
    for m in modes:
        storage, shift_ref, tol = parse_mode(m)
        solvers[m] = lbm.Solver(shape, solid=mask, storage=storage, shift_ref=shift_ref, **dict(kw, newton_tol=tol))
    cols = ["step"] + [f"{m}_l2_{q}" for m in modes for q in ("rho", "u", "T")] + ["u_rms_fp64"]
    rows = []
    done = 0
    while done < steps:
        k = min(every, steps - done)
        for s in solvers.values():
            s.step(k)
        done += k
        ref, _ = solvers["fp64"].moments()
        row = [done]
        for m in modes:
            e = errors(solvers[m].moments()[0], ref, fluid)
            row += [e["l2_rho"], e["l2_u"], e["l2_T"]]
        row.append(float(np.sqrt((ref[1:4, fluid] ** 2).sum(0).mean())))
        rows.append(row)
        if log:
            log(" ".join(f"{c} {v:.3g}" for c, v in zip(cols, row)))
    for s in solvers.values():
        s.close()
    torch.cuda.empty_cache()
    return {"case": case, "shape": list(shape), "every": every, "steps": steps, "plain_bgk": plain_bgk,
            "columns": cols, "rows": rows}


def mach_field(f, gamma):
    """Local Mach number |u| / sqrt(gamma T) of a fields array [5, N]."""
    return np.sqrt((f[1:4] ** 2).sum(0) / (gamma * np.maximum(f[4], 1e-300)))


def study(case: str, steps: int | None = None, scale: float = 1.0, modes=None, mach: float | None = None, log=None,
          plain_bgk: bool = False, average: int = 0, sample: int = 50, chunk: int = 1000):
    make, default_modes, default_steps = CASES[case]
    steps = default_steps if steps is None else steps
    modes = default_modes if modes is None else modes
    shape, solid, kw = make(scale) if mach is None else make(scale, mach)
    if plain_bgk:
        kw = dict(kw, kn_relax=False)
    fluid = solid.reshape(-1) == 0
    results = {"case": case, "shape": list(shape), "steps": steps, "scale": scale,
               "solid_cells": int(solid.sum()),
               "params": {k: v for k, v in kw.items() if k not in ("faces", "fields")},
               "faces": list(kw.get("faces", (PER,) * 6)), "modes": {}}
    fields = {}
    x_body, rows = front_rows(case, shape, scale)
    if average > 0:
        results["window"] = {"steps": average, "sample_every": sample,
                             "fields": "time averages of (rho, u, T) over the window"}
    for m in modes:
        f, summ = run(shape, solid, kw, m, steps, chunk=chunk, log=log, average=average, sample=sample)
        fields[m] = f
        if x_body is not None:
            summ["shock_x"] = {lab: shock_front(f[0], shape, xe, y, z) for lab, y, z, xe in rows}
            summ["standoff"] = x_body - summ["shock_x"]["stagnation"]
        results["modes"][m] = summ
    ref = fields.get("fp64")
    if ref is not None:
        for m in modes:
            if m != "fp64":
                e = errors(fields[m], ref, fluid)
                ma, ma_ref = mach_field(fields[m], kw["gamma"])[fluid], mach_field(ref, kw["gamma"])[fluid]
                e["l2_mach"] = float(np.linalg.norm(ma - ma_ref) / np.linalg.norm(ma_ref))
                e["max_mach"] = float(np.max(np.abs(ma - ma_ref)))
                if x_body is not None:
                    sx, sx_ref = results["modes"][m]["shock_x"], results["modes"]["fp64"]["shock_x"]
                    e["shock_x_shift"] = {k: sx[k] - sx_ref[k] for k in sx}
                    if "window" in results["modes"][m]:
                        a, a_ref = (results["modes"][q]["window"]["alpha_fraction"] for q in (m, "fp64"))
                        e["alpha_share_diff"] = [x - y for x, y in zip(a, a_ref)]
                results["modes"][m]["vs_fp64"] = e
    if "fp32s" in fields and "fp16s" in fields:
        results["modes"]["fp16s"]["vs_fp32s"] = errors(fields["fp16s"], fields["fp32s"], fluid)
    return results


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--case", choices=sorted(CASES), required=True)
    ap.add_argument("--steps", type=int, default=None)
    ap.add_argument("--scale", type=float, default=1.0)
    ap.add_argument("--modes", default=None,
                    help="comma-separated modes storage[@stream][:tol] with storage fp64, fp32s or fp16s; @stream "
                         "shifts the stored deviations by the free stream's equilibrium, :tol sets the Newton "
                         "threshold (fp64:1e-13 against fp64 gives the flow's round-off floor)")
    ap.add_argument("--mach", type=float, default=None, help="default: the case's own (1.5; TGV 0.5)")
    ap.add_argument("--plain-bgk", action="store_true",
                    help="relax every cell with 1/tau (alpha(eps) off), in every mode including the FP64 reference")
    ap.add_argument("--average", type=int, default=0,
                    help="compare time averages over the last N steps (sampled every --sample steps) instead of "
                         "the end state, and report the alpha(eps) branch shares over that window")
    ap.add_argument("--sample", type=int, default=50)
    ap.add_argument("--chunk", type=int, default=1000, help="steps per launch batch (and per progress line)")
    ap.add_argument("--every", type=int, default=0,
                    help="instead: run all modes side by side and report their errors every N steps")
    args = ap.parse_args()
    import torch
    if not torch.cuda.is_available():
        raise SystemExit("the precision study needs a GPU")
    torch.cuda.set_device(0)
    modes = args.modes.split(",") if args.modes else None
    if args.every > 0:
        res = curve(args.case, args.every, args.steps, args.scale, modes, args.mach,
                    log=lambda m: print("#", m, file=sys.stderr, flush=True), plain_bgk=args.plain_bgk)
        print(json.dumps(res), flush=True)
        return
    res = study(args.case, args.steps, args.scale, modes, args.mach,
                log=lambda m: print("#", m, file=sys.stderr, flush=True), plain_bgk=args.plain_bgk,
                average=args.average, sample=args.sample, chunk=args.chunk)
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
