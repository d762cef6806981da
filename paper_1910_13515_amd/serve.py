"""Continuous-batching serving of independent D3Q39 solves on one GPU.

Requests (``inputs.Request``: a 1-D Riemann tube or a periodic 3-D box with
its own grid, flow parameters and step count) arrive on a seeded Poisson
trace.  ``serve_batched`` admits each arrival into the resident pool of the C
ABI (``lbm_pool_*``) as soon as a slot and a large enough free range of the
arena exist (admission by HBM footprint), advances every admitted solve
together with one graph launch of the batched step kernel per round, and
retires solves as they reach their step count, freeing their memory for the
next arrivals.  ``serve_sequential`` runs the same trace one solve at a time
with the plain ``lbm_create`` / ``lbm_step`` / ``lbm_moments`` calls.  Both
report time to solution (arrival to moments on the host) as p50/p99 and the
aggregate throughput in GLUPS.

Argument marshalling and scheduling only: all arithmetic runs in the HIP
library.
"""
from __future__ import annotations

import collections
import ctypes
import math
import time
from dataclasses import dataclass, field

import numpy as np

from . import lbm

def _lib():
    return lbm.load()


def request_params(req, storage: str = "fp32s"):
    """lbm_params for a serving request, plus the host arrays that must stay
    alive until the solve is created.  Tubes are x-periodic (a double Riemann
    problem) with the sound speed at the reference temperature as reference
    speed and L = n/8; boxes are periodic with L = n/2pi and the drawn Mach
    number."""
    nx, ny, nz = req.shape
    if req.kind == "tube":
        p = lbm.make_params(req.shape, storage=storage, gamma=req.gamma, mach=1.0, reynolds=req.reynolds,
                            length_ref=nx / 8.0, T_ref=req.T_ref, u_dir=(1.0, 0.0, 0.0), kn_relax=True)
    else:
        p = lbm.make_params(req.shape, storage=storage, gamma=req.gamma, mach=req.mach, reynolds=req.reynolds,
                            length_ref=nx / (2.0 * math.pi), T_ref=req.T_ref, u_dir=(1.0, 0.0, 0.0),
                            kn_relax=True)
    keep = []
    if req.rho is not None:
        rho = np.ascontiguousarray(req.rho, dtype=np.float64).reshape(-1)
        u = np.ascontiguousarray(req.u, dtype=np.float64).reshape(-1)
        T = np.ascontiguousarray(req.T, dtype=np.float64).reshape(-1)
        keep = [rho, u, T]
        p.init_rho, p.init_u, p.init_T = rho.ctypes.data, u.ctypes.data, T.ctypes.data
    return p, keep


class Pool:
    """A serving pool over a torch-owned device arena."""

    def __init__(self, arena_bytes: int, storage: str = "fp32s", max_slots: int = 64, graph_steps: int = 32,
                 sched: str = "vft", fill_cells: int = 0, stream=None):
        import torch
        L = _lib()
        self.storage = storage
        self.max_slots = max_slots
        self.arena = torch.empty(int(arena_bytes) + 256, dtype=torch.uint8, device="cuda")
        base = (self.arena.data_ptr() + 255) // 256 * 256
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        h = ctypes.c_void_p()
        code = L.lbm_pool_create(lbm.STORAGE[storage], max_slots, graph_steps, lbm.SCHED[sched], int(fill_cells),
                                 ctypes.c_void_p(base), int(arena_bytes), ctypes.c_void_p(self.stream.cuda_stream),
                                 ctypes.byref(h))
        if code != 0:
            raise lbm.LbmError(code, L.lbm_pool_last_error(None).decode())
        self.h = h
        self._finished = (ctypes.c_int32 * max_slots)()

    def _check(self, code):
        if code < 0:
            raise lbm.LbmError(code, _lib().lbm_pool_last_error(self.h).decode())
        return code

    def admit(self, req):
        """Slot index, or None when the request does not fit right now."""
        p, keep = request_params(req, self.storage)
        slot = ctypes.c_int32()
        code = _lib().lbm_pool_admit(self.h, ctypes.byref(p), int(req.steps), ctypes.byref(slot))
        del keep
        if code == lbm.LBM_E_NOMEM:
            return None
        self._check(code)
        return slot.value

    def launch(self) -> int:
        """Start a round without waiting; number of slots it advances."""
        n = ctypes.c_int32()
        self._check(_lib().lbm_pool_launch(self.h, ctypes.byref(n)))
        return n.value

    def wait(self):
        """Wait for the round in flight; slots that reached their step count."""
        nf = ctypes.c_int32()
        self._check(_lib().lbm_pool_wait(self.h, self._finished, ctypes.byref(nf)))
        return [self._finished[k] for k in range(nf.value)]

    def run(self):
        """One round, waited for; finished slots."""
        nf = ctypes.c_int32()
        self._check(_lib().lbm_pool_run(self.h, self._finished, ctypes.byref(nf)))
        return [self._finished[k] for k in range(nf.value)]

    def moments(self, slot: int, n: int, fields: bool = False):
        """(fields[5, n] or None, totals[5]); non-finite moments are
        returned as they are (the caller sees NaN/inf in the totals)."""
        out = np.empty(5 * n) if fields else None
        tot = np.empty(5)
        code = _lib().lbm_pool_moments(self.h, slot, lbm._ptr(out), lbm._ptr(tot))
        if code != lbm.LBM_E_NONFINITE:
            self._check(code)
        return (None if out is None else out.reshape(5, n)), tot

    def release(self, slot: int):
        self._check(_lib().lbm_pool_release(self.h, slot))

    def info(self) -> lbm.lbm_pool_info:
        inf = lbm.lbm_pool_info()
        self._check(_lib().lbm_pool_get_info(self.h, ctypes.byref(inf)))
        return inf

    def close(self):
        if getattr(self, "h", None) is not None:
            _lib().lbm_pool_destroy(self.h)
            self.h = None
            self.arena = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


@dataclass
class Outcome:
    rid: int
    kind: str
    cells: int
    steps: int
    arrival: float
    admitted: float = math.nan
    done: float = math.nan
    totals: np.ndarray = field(default=None, repr=False)
    fields: np.ndarray = field(default=None, repr=False)

    @property
    def latency(self) -> float:
        return self.done - self.arrival


def summarize(outcomes, t_first: float, t_last: float) -> dict:
    lat = np.array([o.latency for o in outcomes])
    work = sum(o.cells * o.steps for o in outcomes)
    span = max(t_last - t_first, 1e-9)
    finite = sum(bool(o.totals is not None and np.all(np.isfinite(o.totals))) for o in outcomes)
    return {
        "requests": len(outcomes),
        "finite_results": int(finite),
        "p50_s": float(np.percentile(lat, 50)),
        "p99_s": float(np.percentile(lat, 99)),
        "mean_s": float(lat.mean()),
        "max_s": float(lat.max()),
        "makespan_s": span,
        "cell_updates": int(work),
        "aggregate_glups": work / span / 1e9,
    }


def _cells(req):
    return req.shape[0] * req.shape[1] * req.shape[2]


def serve_batched(trace, pool, keep_fields: bool = False, realtime: bool = True, progress=None):
    """Continuous batching over a pool.  With realtime, requests become
    visible at their arrival times (relative to the start); otherwise all are
    visible at once.  Arrivals are admitted in arrival order as soon as their
    footprint fits, also while a round is in flight; as soon as a round ends
    the next one is launched, and the finished solves are read back and
    released while it runs.  Returns (outcomes, summary)."""
    pending = collections.deque(sorted(trace, key=lambda r: r.arrival))
    waiting = collections.deque()
    active = {}
    outcomes = {}
    t0 = time.perf_counter()
    now = lambda: time.perf_counter() - t0  # noqa: E731
    in_flight = False

    def retire(slots):
        for slot in slots:
            r = active.pop(slot)
            o = outcomes[r.rid]
            f, tot = pool.moments(slot, _cells(r), fields=keep_fields)
            o.done = now()
            o.totals, o.fields = tot, f
            pool.release(slot)
            if progress:
                progress(o)

    while pending or waiting or active:
        t = now()
        while pending and (not realtime or pending[0].arrival <= t):
            r = pending.popleft()
            waiting.append(r)
            outcomes[r.rid] = Outcome(r.rid, r.kind, _cells(r), r.steps, r.arrival if realtime else 0.0)
        # admission in arrival order, by footprint (overlaps a round in flight)
        zero = []
        while waiting:
            slot = pool.admit(waiting[0])
            if slot is None:
                break
            r = waiting.popleft()
            active[slot] = r
            outcomes[r.rid].admitted = now()
            if r.steps == 0:
                zero.append(slot)
        retire(zero)
        if not in_flight and active:
            in_flight = pool.launch() > 0
            if not in_flight:
                raise RuntimeError("admitted solves with steps left, but the pool launched nothing")
        if in_flight:
            finished = pool.wait()
            in_flight = pool.launch() > 0  # next round first, then read back
            retire(finished)
        elif waiting and not active:
            raise RuntimeError(f"request {waiting[0].rid} does not fit in an empty pool")
        elif pending and not active:
            time.sleep(max(0.0, pending[0].arrival - now()))
    outs = [outcomes[r.rid] for r in trace]
    t_first = min(o.arrival for o in outs)
    t_last = max(o.done for o in outs)
    return outs, summarize(outs, t_first, t_last)


def serve_sequential(trace, storage: str = "fp32s", keep_fields: bool = False, realtime: bool = True,
                     progress=None):
    """The same trace, one solve at a time with the plain calls."""
    pending = sorted(trace, key=lambda r: r.arrival)
    outcomes = []
    t0 = time.perf_counter()
    now = lambda: time.perf_counter() - t0  # noqa: E731
    for r in pending:
        if realtime and now() < r.arrival:
            time.sleep(r.arrival - now())
        o = Outcome(r.rid, r.kind, _cells(r), r.steps, r.arrival if realtime else 0.0)
        o.admitted = now()
        p, keep = request_params(r, storage)
        s = lbm.Solver.from_params(p)
        del keep
        s.step(r.steps)
        f, tot = s.moments(fields=keep_fields)
        o.done = now()
        o.totals, o.fields = tot, f
        s.close()
        outcomes.append(o)
        if progress:
            progress(o)
    by_id = {o.rid: o for o in outcomes}
    outs = [by_id[r.rid] for r in trace]
    t_first = min(o.arrival for o in outs)
    t_last = max(o.done for o in outs)
    return outs, summarize(outs, t_first, t_last)


def solve_alone(req, storage: str = "fp32s", fields: bool = True):
    """One request run by itself with the plain calls (reference for tests)."""
    p, keep = request_params(req, storage)
    s = lbm.Solver.from_params(p)
    del keep
    s.step(req.steps)
    out = s.moments(fields=fields)
    s.close()
    return out


def footprint(req, storage: str = "fp32s") -> int:
    p, keep = request_params(req, storage)
    return lbm.lbm_required_bytes(p)
