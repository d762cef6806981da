"""Summarise rocprofv3 runs of bench.py into the committed profile files.

Reads, under one output root:

    trace/        rocprofv3 --kernel-trace --stats of bench.py (all three storage modes)
    pmc_FETCH_SIZE/, pmc_WRITE_SIZE/          one counter per run, same bench command
    pmc_FETCH_SIZE_copy/, pmc_WRITE_SIZE_copy/ the same counters over bench.py --copy-probe
    pmc_sq/       (optional) SQ_INSTS_VALU, SQ_INSTS_SALU, SQ_INSTS_LDS, SQ_WAVES over the bench command

and writes ``profiles/step_kernel_tgv128.md`` (durations, counter bytes,
calibration, the commands) and ``profiles/traffic.json`` (HBM bytes per step
launch per mode, tied to a hash of the device sources), which bench.py reads
for roofline.traffic.

The counters are scaled by what they read for a plain device copy of known
size (five copies of 1 GiB).

    python -m paper_1910_13515_amd.profile_summary <root> [--commands file]

With --serving it instead summarises <root>/serve_batched and
<root>/serve_sequential (kernel traces of the two sides of the serving leg)
into ``profiles/serving_mix.md``.
"""
from __future__ import annotations

import argparse
import csv
import glob
import json
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PROFILES = os.path.join(ROOT, "profiles")

# kernel-name fragment -> storage mode
STEP_KERNELS = {"fp64": ("step_kernel_f64",), "fp32s": ("step_kernel_f32",), "fp16s": ("step_kernel_f16",)}
BYTES_PER_CELL = {"fp64": 2 * 78 * 8 + 2 * 13 * 8, "fp32s": 2 * 78 * 4 + 2 * 13 * 4, "fp16s": 2 * 78 * 2 + 2 * 13 * 4}
CELLS = 128 ** 3
COPY_BYTES = 1 << 30
COPY_REPS = 5


def _mode_of(name: str):
    """Storage mode of a timed step kernel: the variant without statistics,
    with the Newton root finder, for grids below 2^28 cells (every template
    flag false or 0)."""
    if "true" in name or "Lb1E" in name or ", 1>" in name or "Li1EE" in name:
        return None
    for m, frags in STEP_KERNELS.items():
        if any(f in name for f in frags):
            return m
    return None


def _one(root, pattern):
    hits = sorted(glob.glob(os.path.join(root, pattern), recursive=True))
    if not hits:
        raise FileNotFoundError(os.path.join(root, pattern))
    return hits[0]


def kernel_stats(root):
    out = {}
    with open(_one(root, "trace/**/tgv128_kernel_stats.csv")) as fh:
        for row in csv.DictReader(fh):
            m = _mode_of(row["Name"])
            if m:
                out[m] = {"kernel": row["Name"], "calls": int(row["Calls"]), "avg_ns": float(row["AverageNs"]),
                          "min_ns": float(row["MinNs"]), "max_ns": float(row["MaxNs"])}
    return out


def counter_per_dispatch(root, sub, counter, select):
    """Mean counter value (KiB) over the dispatches whose kernel name select() maps to a key."""
    sums, counts = {}, {}
    with open(_one(root, f"{sub}/**/tgv128_counter_collection.csv")) as fh:
        for row in csv.DictReader(fh):
            if row["Counter_Name"] != counter:
                continue
            key = select(row["Kernel_Name"])
            if key is None:
                continue
            sums[key] = sums.get(key, 0.0) + float(row["Counter_Value"])
            counts[key] = counts.get(key, 0) + 1
    return {k: (sums[k] / counts[k], counts[k]) for k in sums}


def _copy_select(name):
    return "copy" if "copyBuffer" in name else None


def counter_total(root, sub, counter, select):
    """Sum of a counter (KiB) over the dispatches select() maps to a key."""
    tot = {}
    with open(_one(root, f"{sub}/**/copy_counter_collection.csv")) as fh:
        for row in csv.DictReader(fh):
            if row["Counter_Name"] == counter and select(row["Kernel_Name"]) is not None:
                k = select(row["Kernel_Name"])
                tot[k] = tot.get(k, 0.0) + float(row["Counter_Value"])
    return tot


# VALU issue ceiling: one wave64 vector instruction per 4 cycles per SIMD
# (16 lanes), 4 SIMDs x 256 CUs at 2.4 GHz
VALU_ISSUE_PEAK = 256 * 4 * 2.4e9 / 4.0


def sq_counters(root, sub="pmc_sq"):
    """Mean SQ counts per dispatch of each step kernel (optional runs)."""
    try:
        path = _one(root, sub + "/**/tgv128_counter_collection.csv")
    except FileNotFoundError:
        return {}
    sums, counts = {}, {}
    with open(path) as fh:
        for row in csv.DictReader(fh):
            m = _mode_of(row["Kernel_Name"])
            if m is None:
                continue
            key = (m, row["Counter_Name"])
            sums[key] = sums.get(key, 0.0) + float(row["Counter_Value"])
            counts[key] = counts.get(key, 0) + 1
    out = {}
    for (m, c), v in sums.items():
        out.setdefault(m, {})[c] = v / counts[(m, c)]
    return out


def summarize(root, commands=None):
    sys.path.insert(0, ROOT)
    import bench  # the hash of the device sources the profile belongs to

    ks = kernel_stats(root)
    fetch = counter_per_dispatch(root, "pmc_FETCH_SIZE", "FETCH_SIZE", _mode_of)
    write = counter_per_dispatch(root, "pmc_WRITE_SIZE", "WRITE_SIZE", _mode_of)
    # bench.py --copy-probe: COPY_REPS device copies of 1 GiB (one or more
    # copy dispatches each); calibrate on the totals
    cf = counter_total(root, "pmc_FETCH_SIZE_copy", "FETCH_SIZE", _copy_select)["copy"]
    cw = counter_total(root, "pmc_WRITE_SIZE_copy", "WRITE_SIZE", _copy_select)["copy"]
    f_cal = COPY_REPS * COPY_BYTES / (cf * 1024.0)
    w_cal = COPY_REPS * COPY_BYTES / (cw * 1024.0)
    modes = {}
    for m in ("fp64", "fp32s", "fp16s"):
        if m not in ks or m not in fetch or m not in write:
            continue
        fb = fetch[m][0] * 1024.0 * f_cal
        wb = write[m][0] * 1024.0 * w_cal
        alg = BYTES_PER_CELL[m] * CELLS
        avg_s = ks[m]["avg_ns"] * 1e-9
        modes[m] = {
            "kernel": ks[m]["kernel"], "calls": ks[m]["calls"], "avg_ns": ks[m]["avg_ns"],
            "glups_from_avg": CELLS / avg_s / 1e9,
            "algorithmic_bytes_per_launch": alg, "algorithmic_GBps": alg / avg_s / 1e9,
            "fetch_kib_raw": fetch[m][0], "write_kib_raw": write[m][0], "dispatches_counted": fetch[m][1],
            "hbm_read_bytes": fb, "hbm_write_bytes": wb, "hbm_bytes_per_launch": fb + wb,
            "hbm_GBps": (fb + wb) / avg_s / 1e9, "traffic_over_algorithmic": (fb + wb) / alg,
        }
    sq = sq_counters(root)
    for m, v in modes.items():
        if m in sq and "SQ_INSTS_VALU" in sq[m]:
            valu = sq[m]["SQ_INSTS_VALU"]
            v["valu_instr_per_launch"] = valu
            v["valu_instr_per_cell"] = valu / CELLS
            v["valu_issue_floor_us"] = valu / VALU_ISSUE_PEAK * 1e6
            v["valu_issue_frac"] = (valu / (v["avg_ns"] * 1e-9)) / VALU_ISSUE_PEAK
            for c in ("SQ_INSTS_SALU", "SQ_INSTS_LDS", "SQ_WAVES"):
                if c in sq[m]:
                    v[c.lower()] = sq[m][c]
    # where the waves' resident cycles go (optional second run): the share
    # spent issuing VALU and LDS instructions and waiting to issue
    sq2 = sq_counters(root, "pmc_sq2")
    for m, v in modes.items():
        w = sq2.get(m, {}).get("SQ_WAVE_CYCLES")
        if w:
            for c in ("SQ_ACTIVE_INST_VALU", "SQ_ACTIVE_INST_LDS", "SQ_WAIT_INST_ANY", "SQ_LDS_BANK_CONFLICT",
                      "SQ_BUSY_CYCLES"):
                if c in sq2[m]:
                    v[c.lower()] = sq2[m][c]
            v["wave_cycles"] = w
            v["valu_active_share"] = sq2[m].get("SQ_ACTIVE_INST_VALU", 0.0) / w
            v["lds_active_share"] = sq2[m].get("SQ_ACTIVE_INST_LDS", 0.0) / w
            v["wait_share"] = sq2[m].get("SQ_WAIT_INST_ANY", 0.0) / w
    data = {"kernel_hash": bench.kernel_hash(), "workload": "periodic 128^3 Taylor-Green vortex, Ma 0.5, Re 1600",
            "cells_per_launch": CELLS,
            "calibration": {"copy_bytes_each_way": COPY_BYTES, "copies": COPY_REPS,
                            "fetch_kib_per_copy": cf / COPY_REPS, "write_kib_per_copy": cw / COPY_REPS,
                            "fetch_factor": f_cal, "write_factor": w_cal},
            "modes": modes}
    os.makedirs(PROFILES, exist_ok=True)
    with open(os.path.join(PROFILES, "traffic.json"), "w") as fh:
        json.dump(data, fh, indent=1)
    lines = ["# Fused step kernel, periodic 128^3 Taylor-Green vortex (Ma 0.5, Re 1600)", "",
             f"Device sources hash (bench.kernel_hash): `{data['kernel_hash']}`", "",
             "Per launch = one time step over all 2,097,152 cells, f and g.  Algorithmic bytes: 78 populations "
             "read and written plus 13 multipliers read and written per cell (FP64 1456 B, FP32-shifted 728 B, "
             "FP16-shifted 416 B).  HBM peak 8000 GB/s.", "",
             "| storage | kernel | calls | avg us | GLUPS (avg) | algorithmic GB/s | frac of 8 TB/s | "
             "FETCH KiB raw | WRITE KiB raw | HBM bytes/launch (calibrated) | HBM GB/s | traffic / algorithmic |",
             "|---|---|---|---|---|---|---|---|---|---|---|---|"]
    for m, v in modes.items():
        lines.append(f"| {m} | `{v['kernel']}` | {v['calls']} | {v['avg_ns'] / 1e3:.1f} | {v['glups_from_avg']:.3f} | "
                     f"{v['algorithmic_GBps']:.0f} | {v['algorithmic_GBps'] / 8000:.3f} | {v['fetch_kib_raw']:.0f} | "
                     f"{v['write_kib_raw']:.0f} | {v['hbm_bytes_per_launch']:.4g} | {v['hbm_GBps']:.0f} | "
                     f"{v['traffic_over_algorithmic']:.3f} |")
    if any("valu_instr_per_cell" in v for v in modes.values()):
        lines += ["", "Vector ALU issue (rocprofv3 SQ_INSTS_VALU per dispatch).  Ceiling: one wave64 VALU "
                  "instruction per 4 cycles per SIMD, 1024 SIMDs at 2.4 GHz = 614.4 G instructions/s.", "",
                  "| storage | VALU instr / cell | VALU issue floor (us) | kernel avg (us) | issue rate / ceiling |",
                  "|---|---|---|---|---|"]
        for m, v in modes.items():
            if "valu_instr_per_cell" in v:
                lines.append(f"| {m} | {v['valu_instr_per_cell']:.0f} | {v['valu_issue_floor_us']:.0f} | "
                             f"{v['avg_ns'] / 1e3:.0f} | {v['valu_issue_frac']:.2f} |")
    if any("wave_cycles" in v for v in modes.values()):
        lines += ["", "Where a wave's resident cycles go (rocprofv3 SQ_ACTIVE_INST_VALU, SQ_ACTIVE_INST_LDS, "
                  "SQ_WAIT_INST_ANY over SQ_WAVE_CYCLES, summed over the dispatch's waves; all in the same quad-cycle units), with the waves resident "
                  "per SIMD (SQ_WAVES per dispatch over the 1024 SIMDs, per pass of the persistent grid):", "",
                  "| storage | waves per dispatch | VALU-issuing share | LDS-issuing share | waiting to issue | "
                  "LDS bank conflicts |", "|---|---|---|---|---|---|"]
        for m, v in modes.items():
            if "wave_cycles" in v:
                lines.append(f"| {m} | {v.get('sq_waves', float('nan')):.0f} | {v['valu_active_share']:.2f} | "
                             f"{v['lds_active_share']:.3f} | {v['wait_share']:.2f} | "
                             f"{v.get('sq_lds_bank_conflict', 0.0):.0f} |")
    c = data["calibration"]
    lines += ["", "Counter calibration (plain device copy of 1 GiB, `bench.py --copy-probe`): "
              f"FETCH_SIZE reads {c['fetch_kib_per_copy']:.0f} KiB per copy dispatch (factor {c['fetch_factor']:.3f}), "
              f"WRITE_SIZE {c['write_kib_per_copy']:.0f} KiB (factor {c['write_factor']:.3f}).", ""]
    if commands:
        lines += ["Commands (run from the repository root on the GPU host, `cd /tmp && export TMPDIR=/tmp` first "
                  "for the profiler):", "", "```"] + [ln.rstrip() for ln in open(commands) if ln.strip()] + ["```", ""]
    with open(os.path.join(PROFILES, "step_kernel_tgv128.md"), "w") as fh:
        fh.write("\n".join(lines))
    return data


def _dispatches(path):
    """(name, start_ns, end_ns) of every kernel dispatch of a kernel trace."""
    with open(path) as fh:
        return [(r["Kernel_Name"], int(r["Start_Timestamp"]), int(r["End_Timestamp"])) for r in csv.DictReader(fh)]


def _union_ns(intervals):
    """Length of the union of [start, end) intervals (kernels of two streams
    may overlap in time)."""
    total, cur_s, cur_e = 0, None, None
    for s, e in sorted(intervals):
        if cur_e is None or s > cur_e:
            if cur_e is not None:
                total += cur_e - cur_s
            cur_s, cur_e = s, e
        else:
            cur_e = max(cur_e, e)
    if cur_e is not None:
        total += cur_e - cur_s
    return total


def serving_side(path):
    """GPU activity of one side of the serving leg: step-kernel launches and
    their durations, and how much of the span from the first to the last step
    launch the device was busy (any kernel, and step kernels alone)."""
    d = _dispatches(path)
    steps = [(s, e) for n, s, e in d if "step_kernel" in n]
    if not steps:
        return None
    t0 = min(s for s, _ in steps)
    t1 = max(e for _, e in steps)
    inside = [(max(s, t0), min(e, t1)) for _, s, e in d if e > t0 and s < t1]
    durs = sorted(e - s for s, e in steps)
    starts = sorted(s for s, _ in steps)
    ends = sorted(e for _, e in steps)
    gaps = sorted(max(0, b - a) for a, b in zip(ends[:-1], starts[1:]))
    return {"step_launches": len(steps), "step_avg_us": sum(durs) / len(durs) / 1e3,
            "step_p50_us": durs[len(durs) // 2] / 1e3, "step_max_us": durs[-1] / 1e3,
            "span_s": (t1 - t0) / 1e9, "busy_any_s": _union_ns(inside) / 1e9, "busy_step_s": _union_ns(steps) / 1e9,
            "busy_frac": _union_ns(inside) / (t1 - t0), "step_frac": _union_ns(steps) / (t1 - t0),
            "gap_p50_us": gaps[len(gaps) // 2] / 1e3 if gaps else 0.0,
            "other_kernels": len(inside) - len(steps)}


def serving_summary(root, commands=None):
    """profiles/serving_mix.md from <root>/serve_batched and <root>/serve_sequential."""
    data = {}
    for side in ("batched", "sequential"):
        try:
            data[side] = serving_side(_one(root, f"serve_{side}/**/*kernel_trace.csv"))
        except FileNotFoundError:
            data[side] = None
    lines = ["# Serving mix: GPU activity of continuous batching against one solve at a time", "",
             "rocprofv3 --kernel-trace of `bench.py --serving-only --serving-side <side>` (40 requests of the mix, "
             "Poisson arrivals at 3/s, seed 2024, FP32-shifted storage), one run per side.  The span runs from the "
             "first to the last step-kernel launch; busy time is the union of kernel intervals within it (the pool's "
             "admission stream overlaps its rounds).  The batched side includes the pool's two-request warm-up.", "",
             "| side | step launches | avg step (µs) | median step (µs) | max step (µs) | span (s) | busy, any kernel | "
             "busy, step kernel | median gap between steps (µs) | other kernels |",
             "|---|---|---|---|---|---|---|---|---|---|"]
    for side, r in data.items():
        if r is None:
            continue
        lines.append(f"| {side} | {r['step_launches']} | {r['step_avg_us']:.1f} | {r['step_p50_us']:.1f} | "
                     f"{r['step_max_us']:.1f} | {r['span_s']:.2f} | {r['busy_any_s']:.2f} s ({r['busy_frac']:.0%}) | "
                     f"{r['busy_step_s']:.2f} s ({r['step_frac']:.0%}) | {r['gap_p50_us']:.1f} | {r['other_kernels']} |")
    lines.append("")
    if commands:
        lines += ["Commands (run from the repository root on the GPU host, `cd /tmp && export TMPDIR=/tmp` first "
                  "for the profiler):", "", "```"] + [ln.rstrip() for ln in open(commands) if ln.strip()] + ["```", ""]
    with open(os.path.join(PROFILES, "serving_mix.md"), "w") as fh:
        fh.write("\n".join(lines))
    return data


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("root")
    ap.add_argument("--commands", default=None)
    ap.add_argument("--serving", action="store_true", help="summarise the serving traces instead")
    args = ap.parse_args()
    if args.serving:
        print(json.dumps(serving_summary(args.root, args.commands), indent=1))
        return
    print(json.dumps(summarize(args.root, args.commands), indent=1))


if __name__ == "__main__":
    main()
