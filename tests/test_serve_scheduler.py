"""Scheduling logic of the continuous-batching server, driven on the CPU by a stand-in
executor and a simulated clock: FIFO admission, the HBM ledger never exceeds its budget,
requests that do not fit wait (none is dropped), completions free memory."""
import numpy as np
import pytest

from paper_2510_09997_amd import synth
from paper_2510_09997_amd.serve import Scheduler, summarize


class SimClock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        return self.t

    def sleep(self, dt):
        self.t += max(dt, 1e-6)


class FakeExecutor:
    """Batches take a fixed setup time plus a per-megapixel time; each request costs its
    pixel count in 'bytes'."""

    def __init__(self, clock, setup_s=1e-3, per_mpx_s=2e-3):
        self.clock, self.setup, self.per = clock, setup_s, per_mpx_s
        self.launched = []
        self.busy_until = 0.0

    def cost(self, r):
        return r.view.width * r.view.height

    def start(self):
        self.t0 = self.clock()

    def launch(self, batch):
        mpx = sum(self.cost(r) for r in batch) / 1e6
        begin = max(self.clock(), self.busy_until - 0.5 * self.setup)   # overlaps the previous tail
        done = begin + self.setup + self.per * mpx
        self.busy_until = done
        self.launched.append([r.rid for r in batch])
        return dict(done=done)

    def poll(self, h):
        return h["done"] - self.t0 if self.clock() >= h["done"] else None

    def finish(self):
        pass


def requests(count=300, rate=200.0, seed=0):
    return synth.poisson_requests(seed, count, rate_hz=rate)


def test_fifo_admission_all_served_and_budget_respected():
    clk = SimClock()
    ex = FakeExecutor(clk)
    budget = 3 * 3840 * 2160                          # at most three 4K requests in flight
    sch = Scheduler(ex, budget, max_batch=4, max_inflight=3)
    reqs = requests()
    recs = sch.run(reqs, clock=clk, sleep=clk.sleep)
    assert all(np.isfinite(r.done_s) for r in recs)
    assert sch.peak_in_use <= budget
    order = [rid for b in ex.launched for rid in b]
    assert order == sorted(order) == [r.rid for r in sorted(reqs, key=lambda r: r.arrival_s)]
    for r in recs:
        assert r.done_s >= r.arrival_s and r.admitted_s >= r.arrival_s - 1e-12
    s = summarize(recs)
    assert s["requests"] == len(reqs) and s["p99_ms"] >= s["p50_ms"] > 0


def test_budget_shortfall_defers_requests_without_dropping():
    clk = SimClock()
    ex = FakeExecutor(clk, setup_s=5e-3)
    budget = 3840 * 2160                              # exactly one 4K request, or a few smaller
    sch = Scheduler(ex, budget, max_batch=8, max_inflight=3)
    reqs = requests(count=120, rate=2000.0)           # a burst far above capacity
    recs = sch.run(reqs, clock=clk, sleep=clk.sleep)
    assert all(np.isfinite(r.done_s) for r in recs)
    assert sch.peak_in_use <= budget
    for b in ex.launched:
        assert sum(next(r for r in reqs if r.rid == i).view.width * next(r for r in reqs if r.rid == i).view.height
                   for i in b) <= budget
    waited = [r.admitted_s - r.arrival_s for r in recs]
    assert max(waited) > 10 * 5e-3                    # requests were deferred


def test_continuous_batching_beats_one_at_a_time_under_load():
    reqs = requests(count=400, rate=1500.0, seed=3)
    res = {}
    for name, mb, mi in (("continuous", 8, 3), ("plain", 1, 1)):
        clk = SimClock()
        ex = FakeExecutor(clk)
        sch = Scheduler(ex, 1 << 40, max_batch=mb, max_inflight=mi)
        res[name] = summarize(sch.run(reqs, clock=clk, sleep=clk.sleep))
    assert res["continuous"]["p99_ms"] < res["plain"]["p99_ms"]
    assert res["continuous"]["frames_per_s"] >= res["plain"]["frames_per_s"]


def test_request_larger_than_budget_is_an_error():
    clk = SimClock()
    sch = Scheduler(FakeExecutor(clk), 1000, max_batch=2)
    with pytest.raises(ValueError):
        sch.run(requests(count=3), clock=clk, sleep=clk.sleep)
