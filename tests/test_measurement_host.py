"""Host logic of the measurement tools (no GPU): the binding ceiling of the
bench line, the counter file's tie to the kernel sources, and the serving
trace summary."""
import csv
import json

import bench
from paper_1910_13515_amd import profile_summary


def test_binding_ceiling_is_the_higher_floor():
    alu = {"floor_ms": 0.648}
    assert bench.with_ceiling({"floor_ms": 0.382}, alu)["binding_ceiling"] == "alu"
    alu = {"floor_ms": 0.188}
    assert bench.with_ceiling({"floor_ms": 0.191}, alu)["binding_ceiling"] == "hbm"
    assert bench.with_ceiling({"floor_ms": 1.0}, None) is None


def test_counters_are_used_only_for_the_sources_they_came_from(tmp_path, monkeypatch):
    prof = tmp_path / "profiles"
    prof.mkdir()
    t = {"kernel_hash": bench.kernel_hash(),
         "modes": {"fp32s": {"hbm_bytes_per_launch": 1.5e9, "valu_instr_per_launch": 1.2e8,
                             "valu_instr_per_cell": 55.0}}}
    (prof / "traffic.json").write_text(json.dumps(t))
    # the counter file under a scratch root; the source hash stubbed to match
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    monkeypatch.setattr(bench, "kernel_hash", lambda: t["kernel_hash"])
    assert bench.measured_traffic("fp32s") == 1.5e9
    assert bench.measured_traffic("fp16s") is None
    alu = bench.measured_alu("fp32s", 0.35)
    assert abs(alu["frac"] - 1.2e8 / 0.35e-3 / 614.4e9) < 1e-12
    assert abs(alu["floor_ms"] - 1.2e8 / 614.4e9 * 1e3) < 1e-12
    monkeypatch.setattr(bench, "kernel_hash", lambda: "0" * 16)
    assert bench.measured_traffic("fp32s") is None and bench.measured_alu("fp32s", 0.35) is None


def test_union_of_kernel_intervals():
    assert profile_summary._union_ns([]) == 0
    assert profile_summary._union_ns([(0, 10), (5, 15), (20, 30)]) == 25
    assert profile_summary._union_ns([(20, 30), (0, 10), (10, 12)]) == 22
    assert profile_summary._union_ns([(0, 100), (10, 20), (30, 40)]) == 100


def test_serving_side_summary(tmp_path):
    path = tmp_path / "serve_kernel_trace.csv"
    rows = [("lbm13::step_kernel_f32(x)", 1000, 3000), ("lbm13::init_kernel<float>(y)", 2000, 2500),
            ("lbm13::step_kernel_f32(x)", 3000, 4000), ("lbm13::moments_kernel<float>(z)", 6000, 7000),
            ("lbm13::step_kernel_f32(x)", 8000, 9000), ("lbm13::zero_kernel(w)", 9500, 9900)]
    with open(path, "w", newline="") as fh:
        w = csv.writer(fh)
        w.writerow(["Kernel_Name", "Start_Timestamp", "End_Timestamp"])
        for r in rows:
            w.writerow(r)
    r = profile_summary.serving_side(str(path))
    assert r["step_launches"] == 3
    assert abs(r["step_avg_us"] - (2000 + 1000 + 1000) / 3 / 1e3) < 1e-12
    assert abs(r["span_s"] - 8000e-9) < 1e-18
    # steps cover 1000-4000 and 8000-9000; the moments kernel adds 6000-7000;
    # the kernel after the last step lies outside the span
    assert abs(r["busy_step_s"] - 4000e-9) < 1e-18
    assert abs(r["busy_any_s"] - 5000e-9) < 1e-18
    assert r["other_kernels"] == 2
    assert abs(r["gap_p50_us"] - 4.0) < 1e-12  # gaps 0 and 4000 ns


def test_serving_spread_over_seeds():
    """Min, mean and max of each side's figures over trace seeds, and the
    pool's gain (one-at-a-time over pool for latencies, pool over
    one-at-a-time for throughput)."""
    runs = [{"batched": {"p50_s": 1.0, "p99_s": 10.0, "aggregate_glups": 3.6},
             "one_at_a_time": {"p50_s": 2.0, "p99_s": 11.0, "aggregate_glups": 3.5}},
            {"batched": {"p50_s": 0.5, "p99_s": 12.0, "aggregate_glups": 3.4},
             "one_at_a_time": {"p50_s": 2.0, "p99_s": 12.0, "aggregate_glups": 3.4}}]
    s = bench.serving_spread(runs)
    assert s["batched.p50_s"] == {"min": 0.5, "mean": 0.75, "max": 1.0}
    assert s["one_at_a_time.aggregate_glups"]["max"] == 3.5
    assert s["gain.p50_s"] == {"min": 2.0, "mean": 3.0, "max": 4.0}
    assert abs(s["gain.p99_s"]["min"] - 1.0) < 1e-12 and abs(s["gain.p99_s"]["max"] - 1.1) < 1e-12
    assert abs(s["gain.aggregate_glups"]["mean"] - (3.6 / 3.5 + 1.0) / 2) < 1e-12
