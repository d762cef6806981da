"""The continuous-batching loop, driven by a host-only stand-in for the
device pool: arrival-order admission by footprint, retirement at the step
count, memory never over-committed, every request served once."""
import numpy as np

from paper_1910_13515_amd import inputs, serve


class FakePool:
    """Host model of lbm_pool: a byte budget, max_slots, graph_steps per run."""

    def __init__(self, budget, max_slots, graph_steps, footprint):
        self.budget, self.max_slots, self.k = budget, max_slots, graph_steps
        self.footprint = footprint
        self.slots = {}
        self.used = 0
        self.peak = 0
        self.runs = 0
        self.admit_order = []
        self.round = []
        self.in_flight = False

    def admit(self, req):
        need = self.footprint(req)
        free = [i for i in range(self.max_slots) if i not in self.slots]
        if not free or self.used + need > self.budget:
            return None
        s = free[0]
        self.slots[s] = [req, need, req.steps]
        self.used += need
        self.peak = max(self.peak, self.used)
        self.admit_order.append(req.rid)
        return s

    def launch(self):
        assert not self.in_flight
        self.round = [s for s, v in self.slots.items() if v[2] > 0]
        self.in_flight = bool(self.round)
        if self.in_flight:
            self.runs += 1
        return len(self.round)

    def wait(self):
        done = []
        for s in self.round:
            v = self.slots[s]
            v[2] -= min(self.k, v[2])
            if v[2] == 0:
                done.append(s)
        self.round, self.in_flight = [], False
        return done

    def moments(self, slot, n, fields=False):
        assert slot not in self.round
        req = self.slots[slot][0]
        return None, np.array([float(req.rid), n, 0.0, 0.0, 0.0])

    def release(self, slot):
        assert slot not in self.round
        self.used -= self.slots.pop(slot)[1]


def _fp(req):
    return 100 * int(np.prod(req.shape))


def test_batched_loop_serves_every_request_in_arrival_order():
    trace = inputs.serving_trace(4, 40, rate=1e9, tube_cells=(50, 400), box_cells=(4, 10), steps=(0, 90),
                                 with_fields=False)
    budget = max(_fp(r) for r in trace) * 3
    pool = FakePool(budget, 5, 16, _fp)
    outs, summary = serve.serve_batched(trace, pool, realtime=False)
    assert summary["requests"] == len(trace)
    assert pool.peak <= budget and pool.used == 0 and not pool.slots
    assert pool.admit_order == sorted(pool.admit_order)  # FIFO admission
    for r, o in zip(trace, outs):
        assert o.rid == r.rid and o.totals[0] == r.rid
        assert o.admitted <= o.done
    # runs needed: at least the longest request's rounds
    assert pool.runs >= max(-(-r.steps // 16) for r in trace)


def test_summary_percentiles():
    outs = [serve.Outcome(i, "box", 8, 10, arrival=0.0, admitted=0.0, done=float(i + 1)) for i in range(100)]
    s = serve.summarize(outs, 0.0, 100.0)
    assert s["p50_s"] == np.percentile(np.arange(1, 101), 50)
    assert s["p99_s"] == np.percentile(np.arange(1, 101), 99)
    assert s["cell_updates"] == 8000 and abs(s["aggregate_glups"] - 8000 / 100 / 1e9) < 1e-18
