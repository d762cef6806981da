"""Serving pool on the GPU: every solve of a mixed batch gives exactly the
result it gives alone, admission is by HBM footprint, and the continuous
batching loop retires every request of a trace."""
import numpy as np
import pytest

from paper_1910_13515_amd import inputs, lbm

pytestmark = pytest.mark.gpu


def _trace(seed, count, **kw):
    kw.setdefault("tube_cells", (90, 260))
    kw.setdefault("box_cells", (6, 14))
    kw.setdefault("steps", (5, 37))
    kw.setdefault("mach", (0.2, 0.8))
    return inputs.serving_trace(seed, count, rate=1e6, **kw)


def _first(kind, seed=3, **kw):
    return next(r for r in _trace(seed, 16, **kw) if r.kind == kind)


@pytest.mark.parametrize("storage,sched", [("fp64", "all"), ("fp64", "srpt"), ("fp32s", "srpt"), ("fp16s", "srpt"),
                                           ("fp32s", "all"), ("fp32s", "vft")])
def test_mix_equals_alone_bitwise(storage, sched):
    from paper_1910_13515_amd import serve
    trace = _trace(11, 9)
    fps = [serve.footprint(r, storage) for r in trace]
    # room for about half of them at once: admission waits, slots are reused
    room = max(sum(fps) // 2, max(fps)) + (1 << 20)
    # a small SRPT fill bound so that rounds really leave slots waiting
    pool = serve.Pool(lbm.load().lbm_pool_overhead_bytes(4) + room, storage=storage, max_slots=4, graph_steps=8,
                      sched=sched, fill_cells=3000)
    outs, summary = serve.serve_batched(trace, pool, keep_fields=True, realtime=False)
    assert summary["requests"] == len(trace)
    inf = pool.info()
    assert inf.active == 0 and inf.free_bytes == inf.arena_bytes - lbm.load().lbm_pool_overhead_bytes(4)
    pool.close()
    for r, o in zip(trace, outs):
        fields, tot = serve.solve_alone(r, storage)
        assert np.array_equal(o.fields, fields), (r.rid, r.kind, r.shape, r.steps)
        assert np.array_equal(o.totals, tot), r.rid


def test_admission_by_footprint_and_release():
    from paper_1910_13515_amd import serve
    L = lbm.load()
    req = _first("box", box_cells=(12, 12), steps=(10, 10))
    fp = serve.footprint(req, "fp32s")
    head = L.lbm_pool_overhead_bytes(8)
    pool = serve.Pool(head + 2 * fp + 4096, storage="fp32s", max_slots=8, graph_steps=4)
    a = pool.admit(req)
    b = pool.admit(req)
    assert a is not None and b is not None and a != b
    assert pool.admit(req) is None  # no free range: refused, nothing changed
    inf = pool.info()
    assert inf.active == 2 and inf.running == 2 and inf.largest_free < fp
    # storage mismatch is an argument error, not a refusal
    p, _ = serve.request_params(req, "fp64")
    import ctypes
    slot = ctypes.c_int32()
    assert L.lbm_pool_admit(pool.h, ctypes.byref(p), 1, ctypes.byref(slot)) == lbm.LBM_E_INVAL
    # a round in flight: its slots cannot be read or released, admission goes on
    assert pool.launch() == 2
    assert pool.info().in_flight == 1
    with pytest.raises(lbm.LbmError):
        pool.moments(a, 12 ** 3)
    with pytest.raises(lbm.LbmError):
        pool.release(b)
    with pytest.raises(lbm.LbmError):
        pool.launch()
    # a slot that was never admitted: an argument error, reported on the pool
    with pytest.raises(lbm.LbmError) as e:
        pool.release(7)
    assert e.value.code == lbm.LBM_E_INVAL and "invalid slot" in str(e.value)
    done = pool.wait()
    for _ in range(2):
        done += pool.run()
    assert sorted(done) == sorted([a, b])
    assert pool.run() == []  # nothing running: a no-op
    pool.release(a)
    c = pool.admit(req)
    assert c is not None
    assert pool.info().active == 2
    pool.close()


def test_admission_during_round_matches_alone():
    from paper_1910_13515_amd import serve
    first = _first("box", seed=7, box_cells=(14, 14), steps=(24, 24))
    late = _first("tube", seed=8, tube_cells=(150, 150), steps=(17, 17))
    pool = serve.Pool(256 << 20, storage="fp32s", max_slots=4, graph_steps=8, sched="all")
    a = pool.admit(first)
    assert pool.launch() == 1
    b = pool.admit(late)  # created on the admission stream while the round runs
    fin = pool.wait()
    while a not in fin or b not in fin:
        assert pool.launch() >= 1
        fin += pool.wait()
    for slot, r in ((a, first), (b, late)):
        f, tot = pool.moments(slot, int(np.prod(r.shape)), fields=True)
        f1, t1 = serve.solve_alone(r, "fp32s")
        assert np.array_equal(f, f1) and np.array_equal(tot, t1), r.rid
    pool.close()


def test_zero_step_request_keeps_initial_state():
    from paper_1910_13515_amd import serve
    req = _first("box", seed=5, box_cells=(8, 8), steps=(1, 1))
    req.steps = 0
    pool = serve.Pool(64 << 20, storage="fp64", max_slots=2, graph_steps=4)
    slot = pool.admit(req)
    assert pool.run() == []
    f0, t0 = pool.moments(slot, int(np.prod(req.shape)), fields=True)
    p, keep = serve.request_params(req, "fp64")
    s = lbm.Solver.from_params(p)
    f1, t1 = s.moments()
    assert np.array_equal(f0, f1) and np.array_equal(t0, t1)
    s.close()
    pool.release(slot)
    # the serving loop retires a zero-step request at admission
    outs, summary = serve.serve_batched([req], pool, realtime=False)
    assert summary["requests"] == 1 and np.array_equal(outs[0].totals, t1)
    pool.close()


def test_realtime_trace_latencies():
    from paper_1910_13515_amd import serve
    trace = inputs.serving_trace(21, 12, rate=200.0, tube_cells=(90, 200), box_cells=(8, 16), steps=(20, 60),
                                 mach=(0.2, 0.6))
    pool = serve.Pool(256 << 20, storage="fp32s", max_slots=16, graph_steps=16)
    outs, summary = serve.serve_batched(trace, pool)
    pool.close()
    assert summary["requests"] == 12
    assert 0.0 < summary["p50_s"] <= summary["p99_s"] <= summary["max_s"]
    for o in outs:
        assert o.arrival <= o.admitted <= o.done
        assert np.all(np.isfinite(o.totals))
