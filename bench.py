#!/usr/bin/env python3
"""Throughput of the fused D3Q39 13-moment DDF-LBM step on one MI355X.

Workload (default): periodic 128^3 compressible Taylor-Green vortex, Ma 0.5,
Re 1600, gamma 1.4, FP64 storage and arithmetic (the plain FP64 GPU step).
The same workload is also timed with FP32- and FP16-shifted storage and
reported under "modes", and the serving mix (continuous batching against one
solve at a time) under "serving".  A step is one fused stream-and-collide launch over
all cells (f and g).  Prints one JSON line.

  python bench.py [--gpus 1] [--steps K] [--warmup W] [--mode fp64|fp32s|fp16s]
                  [--n 128] [--no-modes] [--no-cpu] [--no-serving]
                  [--serving-requests 40] [--serving-rate 1.75] [--serving-only]
  python bench.py --serving-only --serving-requests 200 --serving-rate 1.75 \
                  --serving-seeds 2024,2025,2026   (run-to-run spread of the serving figures)
  python bench.py --copy-probe   (plain device copy of 1 GiB x 5, used to
                                  calibrate the FETCH_SIZE / WRITE_SIZE counters)

roofline.traffic is read from profiles/traffic.json (HBM bytes per launch from
rocprofv3 FETCH_SIZE / WRITE_SIZE, scaled by the copy calibration) and is null
unless that file was taken from the current kernel sources.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, vendor figure
# algorithmic bytes per cell update: 78 populations read + written, 13
# multipliers read + written
BYTES_PER_CELL = {"fp64": 2 * 78 * 8 + 2 * 13 * 8, "fp32s": 2 * 78 * 4 + 2 * 13 * 4, "fp16s": 2 * 78 * 2 + 2 * 13 * 4}
DTYPE = {"fp64": "f64", "fp32s": "f32 (fp32-shifted storage)", "fp16s": "f32 (fp16-shifted storage)"}


def tgv_setup(n, ma=0.5, re=1600.0, gamma=1.4, T0=0.5):
    from paper_1910_13515_amd import inputs
    U = ma * math.sqrt(gamma * T0)
    fields = inputs.taylor_green_fields(n, U, T0)
    kw = dict(gamma=gamma, mach=ma, reynolds=re, length_ref=n / (2 * math.pi), T_ref=T0, u_dir=(1, 0, 0),
              kn_relax=True)
    return fields, kw


def run_mode(mode, n, steps, warmup):
    import torch
    from paper_1910_13515_amd import lbm
    fields, kw = tgv_setup(n)
    s = lbm.Solver((n, n, n), fields=fields, storage=mode, **kw)
    cells = n ** 3
    s.step(warmup)
    torch.cuda.synchronize()
    stream = s.stream
    start = torch.cuda.Event(enable_timing=True)
    end = torch.cuda.Event(enable_timing=True)
    start.record(stream)
    s.step(steps)
    end.record(stream)
    end.synchronize()
    torch.cuda.synchronize()
    ms = start.elapsed_time(end)
    st = s.step(1, stats=True)  # statistics of one further step (not timed)
    info = s.info()
    fields, _ = s.moments()  # (rho, u, T) after warmup + steps + 1, for the error against FP64
    s.close()
    del s
    torch.cuda.empty_cache()
    ms_step = ms / steps
    glups = cells * steps / (ms * 1e-3) / 1e9
    bytes_launch = BYTES_PER_CELL[mode] * cells
    achieved = bytes_launch / (ms_step * 1e-3) / 1e9
    return {
        "fields": fields,
        "steps_total": warmup + steps + 1,
        "glups": glups,
        "ms_per_step": ms_step,
        "tau": info.tau,
        "newton_iterations_per_cell": st.iterations / max(1, st.cell_updates),
        "newton_max_iterations": st.max_iterations,
        "alpha_hist": list(st.alpha_hist),
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                     "bytes_per_cell": BYTES_PER_CELL[mode], "cells_per_launch": cells,
                     "floor_ms": bytes_launch / (HBM_PEAK_GBS * 1e9) * 1e3},
    }


def run_case(case, mode, develop, steps):
    """One obstacle workload of the method at its full size (the supersonic
    airfoil of Sec. 4, 2048 x 1024 x 1, or the sphere in a 512 x 256 x 256
    channel) in one storage mode: `develop` untimed steps from the free
    stream, so that the shocks and the wake have formed, then `steps` timed
    ones.  Algorithmic bytes per cell add the 8-byte link mask that an
    obstacle's cells read."""
    import numpy as np
    import torch

    from paper_1910_13515_amd import lbm, precision_study
    make = {"airfoil": precision_study.airfoil_case, "sphere": precision_study.sphere_case}[case]
    shape, solid, kw = make(1.0)
    storage, shift_ref, _ = precision_study.parse_mode(mode)
    s = lbm.Solver(shape, solid=solid, storage=storage, shift_ref=shift_ref, **kw)
    cells = int(np.prod(shape))
    done = 0
    while done < develop:
        k = min(500, develop - done)
        s.step(k)
        done += k
    torch.cuda.synchronize()
    start = torch.cuda.Event(enable_timing=True)
    end = torch.cuda.Event(enable_timing=True)
    start.record(s.stream)
    s.step(steps)
    end.record(s.stream)
    end.synchronize()
    ms = start.elapsed_time(end)
    st = s.step(1, stats=True)
    info = s.info()
    s.close()
    del s
    torch.cuda.empty_cache()
    ms_step = ms / steps
    bpc = BYTES_PER_CELL[storage] + 8
    achieved = bpc * cells / (ms_step * 1e-3) / 1e9
    return {"workload": f"{case} {'x'.join(map(str, shape))}, Ma {kw['mach']}, Re {kw['reynolds']:g}, "
                        f"T_ref {kw['T_ref']:.4g}, {mode}, timed after {develop} steps",
            "glups": cells * steps / (ms * 1e-3) / 1e9, "ms_per_step": ms_step, "steps": steps, "tau": info.tau,
            "newton_iterations_per_cell": st.iterations / max(1, st.cell_updates),
            "failed_cells_next_step": int(st.failed), "alpha_hist": list(st.alpha_hist),
            "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                         "frac": achieved / HBM_PEAK_GBS, "traffic": None, "bytes_per_cell": bpc,
                         "cells_per_launch": cells}}


# device sources, and the host layer that sets their run-time parameters
# (default Newton tolerances change the instruction counts)
KERNEL_SOURCES = ["lbm_kernels.hip", "equilibrium.h", "d3q39.h", "slot.h", "lbm_api.cpp"]


def kernel_hash() -> str:
    """Hash of the kernel sources, to tie counter data to the kernel it came from."""
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_1910_13515_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(mode: str):
    """HBM bytes per launch of the step kernel from the committed counter
    summary, or None when it is missing or was taken from other sources."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    try:
        with open(path) as fh:
            t = json.load(fh)
    except (OSError, ValueError):
        return None
    if t.get("kernel_hash") != kernel_hash() or mode not in t.get("modes", {}):
        return None
    return t["modes"][mode]["hbm_bytes_per_launch"]


def measured_alu(mode: str, ms_per_step: float):
    """Vector-ALU issue rate of the step kernel: VALU instructions per launch
    from the committed counter summary (same kernel sources only) over the
    launch time measured here, against 614.4 G wave instructions/s (one per
    4 cycles per SIMD, 1024 SIMDs at 2.4 GHz)."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    try:
        with open(path) as fh:
            t = json.load(fh)
    except (OSError, ValueError):
        return None
    if t.get("kernel_hash") != kernel_hash():
        return None
    m = t.get("modes", {}).get(mode, {})
    if "valu_instr_per_launch" not in m:
        return None
    peak = 256 * 4 * 2.4e9 / 4.0
    achieved = m["valu_instr_per_launch"] / (ms_per_step * 1e-3)
    return {"valu_instr_per_cell": m["valu_instr_per_cell"], "achieved_ginstr_s": achieved / 1e9,
            "peak_ginstr_s": peak / 1e9, "frac": achieved / peak,
            "floor_ms": m["valu_instr_per_launch"] / peak * 1e3}


def with_ceiling(roof, alu):
    """Names the higher of the two floors (HBM bytes at peak bandwidth, VALU
    instructions at peak issue): the ceiling that binds the launch."""
    if alu is not None:
        alu["binding_ceiling"] = "alu" if alu["floor_ms"] > roof["floor_ms"] else "hbm"
    return alu


def copy_probe(gib=1, reps=5):
    """A plain device-to-device copy of known size (counter calibration)."""
    import torch
    n = gib * (1 << 30) // 4
    a = torch.ones(n, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        b.copy_(a)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    print(json.dumps({"copy_bytes_each_way": n * 4, "reps": reps, "GBps": 2 * n * 4 * reps / dt / 1e9}), flush=True)


SERVING_MIX = dict(tube_cells=(200, 4000), box_cells=(64, 192), steps=(200, 2000), ratio=(2.0, 10.0),
                   mach=(0.3, 1.5), reynolds=(1e3, 1e4))


def serving_leg(count, rate, seed=2024, arena_gib=96, max_slots=64, graph_steps=32, sched="vft", sequential=True,
                batched=True):
    """The serving mix (seeded Poisson arrivals of tubes and boxes, FP32
    shifted storage): continuous batching in the pool against the same trace
    solved one at a time with the plain calls."""
    from paper_1910_13515_amd import inputs, serve
    trace = inputs.serving_trace(seed, count, rate, **SERVING_MIX)
    out = {"trace": {"seed": seed, "requests": count, "rate_per_s": rate, "storage": "fp32s", **SERVING_MIX},
           "pool": {"arena_gib": arena_gib, "max_slots": max_slots, "graph_steps": graph_steps, "sched": sched}}

    def progress(o, name):
        if o.rid % 20 == 19:
            print(f"# serving {name}: request {o.rid + 1} done at {o.done:.1f} s", file=sys.stderr, flush=True)

    if batched:
        out["batched"] = _serve_pool(trace, seed, arena_gib, max_slots, graph_steps, sched, progress)
    if sequential:
        _, seq = serve.serve_sequential(trace, storage="fp32s", progress=lambda o: progress(o, "one at a time"))
        print(f"# serving one-at-a-time: p50 {seq['p50_s']:.3f} s p99 {seq['p99_s']:.3f} s "
              f"{seq['aggregate_glups']:.3f} GLUPS", file=sys.stderr, flush=True)
        out["one_at_a_time"] = seq
    return out


def serving_spread(runs):
    """Min, mean and max over runs (one per trace seed) of each side's p50,
    p99 and aggregate GLUPS, and of the pool's gain over one at a time."""
    out = {}
    for side in ("batched", "one_at_a_time"):
        for key in ("p50_s", "p99_s", "aggregate_glups"):
            v = [r[side][key] for r in runs]
            out[f"{side}.{key}"] = {"min": min(v), "mean": sum(v) / len(v), "max": max(v)}
    for key, better in (("p50_s", "lower"), ("p99_s", "lower"), ("aggregate_glups", "higher")):
        g = [(r["one_at_a_time"][key] / r["batched"][key]) if better == "lower"
             else (r["batched"][key] / r["one_at_a_time"][key]) for r in runs]
        out[f"gain.{key}"] = {"min": min(g), "mean": sum(g) / len(g), "max": max(g)}
    return out


def _serve_pool(trace, seed, arena_gib, max_slots, graph_steps, sched, progress):
    import torch
    from paper_1910_13515_amd import inputs, serve
    pool = serve.Pool(arena_gib << 30, storage="fp32s", max_slots=max_slots, graph_steps=graph_steps, sched=sched)
    # warm the graph and the admission path once (untimed)
    warm = inputs.serving_trace(seed + 1, 2, 1e6, tube_cells=(200, 400), box_cells=(16, 16), steps=(40, 40))
    serve.serve_batched(warm, pool, realtime=False)
    _, batched = serve.serve_batched(trace, pool, progress=lambda o: progress(o, "batched"))
    pool.close()
    del pool
    torch.cuda.empty_cache()
    print(f"# serving batched ({sched}): p50 {batched['p50_s']:.3f} s p99 {batched['p99_s']:.3f} s "
          f"{batched['aggregate_glups']:.3f} GLUPS", file=sys.stderr, flush=True)
    return batched


def cpu_baseline(seconds_target=15.0):
    """The FP64 oracle on the host cores: TGV 32^3 (same Ma, Re), a bounded
    number of steps.  Reported in GLUPS."""
    import oracle
    n = 32
    fields, kw = tgv_setup(n)
    # relaxation time with the same model viscosity as the GPU run
    U = kw["mach"] * math.sqrt(kw["gamma"] * kw["T_ref"])
    tau = oracle.tau_from_reynolds(U, kw["length_ref"], kw["reynolds"], kw["T_ref"])
    o = oracle.Oracle(n, n, n, gamma=kw["gamma"], tau=tau, kn_relax=True, newton_tol=1e-12, newton_maxit=20)
    o.init(*fields)
    t0 = time.perf_counter()
    steps = 0
    while time.perf_counter() - t0 < seconds_target or steps < 1:
        o.step(1)
        steps += 1
    dt = time.perf_counter() - t0
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    return {"value": n ** 3 * steps / dt / 1e9, "unit": "GLUPS", "cores": threads, "kind": "oracle",
            "sample": f"FP64 oracle, TGV {n}^3 Ma 0.5 Re 1600, {steps} steps from the initial state, {dt:.1f} s"}


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_table(single_thread=False, log=None):
    """The FP64 oracle timed on the configurations of the method's workloads
    (bounded step counts; full runs would take hours on the host).  Uses the
    OpenMP threads the process was started with (OMP_NUM_THREADS)."""
    import numpy as np

    import oracle
    from paper_1910_13515_amd import inputs, precision_study
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    eq, neu = oracle.FACE_EQUILIBRIUM, oracle.FACE_NEUMANN

    def timed(name, shape, fields, steps, **okw):
        o = oracle.Oracle(*shape, **okw)
        t0 = time.perf_counter()
        if o.init(*fields) != 0:
            raise RuntimeError("the oracle found no initial equilibrium")
        t_init = time.perf_counter() - t0
        t0 = last = time.perf_counter()
        for k in range(steps):
            o.step(1)
            if log and time.perf_counter() - last > 30.0:
                last = time.perf_counter()
                log(f"oracle {name}: {k + 1}/{steps} steps")
        dt = time.perf_counter() - t0
        n = int(np.prod(shape))
        r = {"case": name, "cells": n, "steps": steps, "seconds": dt, "init_seconds": t_init,
             "mlups": n * steps / dt / 1e6}
        if log:
            log(f"oracle {name}: {r['mlups']:.3f} MLUPS ({steps} steps, {dt:.1f} s)")
        del o
        return r

    rows = []
    # Sod tube 400 x 1 x 1, tau 0.5 with alpha(eps), all 400 steps
    rows.append(timed("Sod 400x1x1", (400, 1, 1), inputs.sod_fields(400, temp_scale=0.5), 400, gamma=1.4, tau=0.5,
                      kn_relax=True, faces=(eq, eq, 0, 0, 0, 0), newton_tol=1e-12))
    # TGV at 32^3 and 128^3 (Ma 0.5, Re 1600)
    for n, steps in ((32, 20),) if single_thread else ((32, 200), (128, 20)):
        fields, kw = tgv_setup(n)
        U = kw["mach"] * math.sqrt(kw["gamma"] * kw["T_ref"])
        tau = oracle.tau_from_reynolds(U, kw["length_ref"], kw["reynolds"], kw["T_ref"])
        rows.append(timed(f"TGV {n}^3", (n, n, n), fields, steps, gamma=kw["gamma"], tau=tau, kn_relax=True,
                          newton_tol=1e-12))
    # the obstacle flows from the free stream, a few steps (the sphere at half
    # its size, 256 x 128 x 128: the cold start of the full grid alone takes
    # minutes on the host)
    cases = [] if single_thread else [("airfoil 2048x1024", precision_study.airfoil_case, 1.0, 5),
                                      ("sphere 256x128x128", precision_study.sphere_case, 0.5, 3)]
    for name, make, scale, steps in cases:
        if log:
            log(f"oracle {name}: cold start")
        shape, solid, kw = make(scale)
        n = int(np.prod(shape))
        U = kw["mach"] * math.sqrt(kw["gamma"] * kw["T_ref"])
        tau = oracle.tau_from_reynolds(U, kw["length_ref"], kw["reynolds"], kw["T_ref"])
        u = np.zeros((3, n))
        u[0] = U
        rows.append(timed(name, shape, (np.ones(n), u, np.full(n, kw["T_ref"])), steps, gamma=kw["gamma"], tau=tau,
                          kn_relax=True, faces=kw["faces"], solid=solid, newton_tol=1e-12))
    return {"oracle_threads": threads, "cpu_model": _cpu_model(), "host_cpus": os.cpu_count(), "rows": rows}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--mode", default="fp64", choices=["fp64", "fp32s", "fp16s"])
    ap.add_argument("--n", type=int, default=128)
    ap.add_argument("--no-modes", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--copy-probe", action="store_true")
    ap.add_argument("--serving-requests", type=int, default=40)
    # 0.8 of the pool's capacity on this mix: about 3.6 GLUPS over a mean of
    # 1.65e9 cell updates per request is 2.2 requests/s
    ap.add_argument("--serving-rate", type=float, default=1.75)
    ap.add_argument("--no-serving", action="store_true")
    ap.add_argument("--no-configs", action="store_true",
                    help="skip the obstacle workloads (FP32 airfoil, FP16 sphere, each beside FP64)")
    ap.add_argument("--serving-only", action="store_true")
    ap.add_argument("--serving-side", default="both", choices=["both", "batched", "sequential"],
                    help="with --serving-only: run one side of the comparison alone (for profiling)")
    ap.add_argument("--serving-sched", default="vft", choices=["vft", "srpt", "all"],
                    help="round selection of the pool (with --serving-only)")
    ap.add_argument("--serving-seeds", default=None,
                    help="with --serving-only: comma-separated trace seeds, one full comparison each, and the "
                         "spread of p50, p99 and throughput over them")
    ap.add_argument("--cpu-table", action="store_true",
                    help="time the FP64 oracle on the workloads' configurations instead (host only)")
    ap.add_argument("--cpu-table-short", action="store_true", help="with --cpu-table: the short set (Sod, TGV 32^3)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: a single domain is not sharded across GPUs here (x-slabs with "
              "a 3-cell halo exchange would be the way); run with --gpus 1", file=sys.stderr)
        sys.exit(2)
    if args.cpu_table:
        res = cpu_table(args.cpu_table_short, log=lambda m: print("#", m, file=sys.stderr, flush=True))
        print(json.dumps({"cpu_table": res}), flush=True)
        return
    import torch
    if not torch.cuda.is_available():
        raise SystemExit("bench.py needs a GPU")
    torch.cuda.set_device(0)
    if args.copy_probe:
        copy_probe()
        return
    from paper_1910_13515_amd import lbm
    lbm.load()
    if args.serving_only:
        if args.serving_seeds:
            runs = [serving_leg(args.serving_requests, args.serving_rate, seed=int(sd), sched=args.serving_sched)
                    for sd in args.serving_seeds.split(",")]
            print(json.dumps({"serving_runs": runs, "spread": serving_spread(runs)}), flush=True)
            return
        print(json.dumps({"serving": serving_leg(args.serving_requests, args.serving_rate, sched=args.serving_sched,
                                                 batched=args.serving_side != "sequential",
                                                 sequential=args.serving_side != "batched")}), flush=True)
        return

    main_res = run_mode(args.mode, args.n, args.steps, args.warmup)
    print(f"# {args.mode}: {main_res['glups']:.3f} GLUPS, {main_res['ms_per_step']:.3f} ms/step", file=sys.stderr,
          flush=True)
    modes = {}
    if not args.no_modes:
        for m in ("fp64", "fp32s", "fp16s"):
            if m == args.mode:
                continue
            r = run_mode(m, args.n, args.steps, args.warmup)
            print(f"# {m}: {r['glups']:.3f} GLUPS, {r['ms_per_step']:.3f} ms/step", file=sys.stderr, flush=True)
            modes[m] = r
    configs = {}
    if not args.no_configs:
        # the airfoil compares FP32-shifted storage with FP64, the sphere
        # FP16-shifted (on the rest weights, and on the free stream's
        # equilibrium) with FP32 and FP64 (each at its full size)
        for case, modes_c, develop, steps_c in (("airfoil", ("fp32s", "fp64"), 2000, 200),
                                                ("sphere", ("fp16s", "fp16s@stream", "fp32s", "fp64"), 500, 20)):
            for m in modes_c:
                r = run_case(case, m, develop, steps_c)
                print(f"# {case} {m}: {r['glups']:.3f} GLUPS, {r['ms_per_step']:.3f} ms/step", file=sys.stderr,
                      flush=True)
                configs[f"{case}_{m}"] = r
    serving = None if args.no_serving else serving_leg(args.serving_requests, args.serving_rate)
    cpu = None if args.no_cpu else cpu_baseline()
    roof = dict(main_res["roofline"])
    roof["traffic"] = measured_traffic(args.mode)
    ref = main_res.pop("fields")
    main_res.pop("steps_total")
    for m, r in modes.items():
        r["roofline"]["traffic"] = measured_traffic(m)
        r["alu"] = with_ceiling(r["roofline"], measured_alu(m, r["ms_per_step"]))
        f = r.pop("fields")
        if args.mode == "fp64":
            # same initial state and step count as the FP64 run: relative L2
            # errors of (rho, u, T) over all cells
            import numpy as np

            from paper_1910_13515_amd import precision_study
            e = precision_study.errors(f, ref, np.ones(f.shape[1], dtype=bool))
            r["vs_fp64"] = {"after_steps": r["steps_total"], **{k: v for k, v in e.items() if k.startswith("l2_")}}
        r.pop("steps_total")
    out = {
        "metric": "GLUPS (D3Q39 f+g) & % HBM roofline, FP32/FP16 vs FP64 at stated error; p99",
        "value": main_res["glups"],
        "unit": "GLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": main_res["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": DTYPE[args.mode],
        "data": "synthetic (analytic Taylor-Green initial fields)",
        "config": {"workload": f"periodic {args.n}^3 compressible Taylor-Green vortex, Ma 0.5, Re 1600, "
                               f"gamma 1.4, {args.mode} step", "cells": args.n ** 3, "storage": args.mode,
                   "tau": main_res["tau"], "newton_iterations_per_cell": main_res["newton_iterations_per_cell"],
                   "alpha_hist": main_res["alpha_hist"]},
        "roofline": roof,
        "alu": with_ceiling(roof, measured_alu(args.mode, main_res["ms_per_step"])),
        "cpu_baseline": cpu,
        "modes": modes,
        "configs": configs,
        "serving": serving,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
