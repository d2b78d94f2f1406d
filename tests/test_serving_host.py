"""Scheduler logic of the continuous-batching server, on the CPU with a fake
executor whose launches take a modelled time on a manually advanced clock."""
import math

import pytest

from paper_2202_03411_amd.serving import Request, Scheduler, poisson_arrivals, summarize


class Clock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        return self.t


class FakeExecutor:
    """Launch of a batch takes the sum of its requests' durations; footprint and
    duration (also the work estimate) from the request key."""

    def __init__(self, clock, foot, dur):
        self.clock, self.foot, self.dur = clock, foot, dur
        self.launches = []

    def footprint(self, req):
        return self.foot[req.key]

    def cost(self, req):
        return self.dur[req.key]

    def launch(self, batch):
        h = {"end": self.clock() + sum(self.dur[r.key] for r in batch), "ids": [r.rid for r in batch]}
        self.launches.append(h)
        return h

    def poll(self, h):
        return self.clock() >= h["end"]

    def finish(self, h, batch):
        for r in batch:
            r.result = ("done", r.rid)


def _drive(sched, clock, reqs, dt=0.001, horizon=100.0):
    reqs = sorted(reqs, key=lambda r: r.arrival)
    i = 0
    max_used = 0
    while (i < len(reqs) or not sched.idle()) and clock.t < horizon:
        while i < len(reqs) and reqs[i].arrival <= clock.t:
            sched.submit(reqs[i])
            i += 1
        sched.step()
        max_used = max(max_used, sched.used)
        assert len(sched.inflight) <= sched.max_inflight
        clock.t += dt
    return max_used


def _reqs(keys, arrivals):
    return [Request(k, a, key) for k, (key, a) in enumerate(zip(keys, arrivals))]


def test_budget_never_exceeded_and_all_complete():
    clock = Clock()
    ex = FakeExecutor(clock, {"s": 10, "m": 30, "l": 60}, {"s": 0.01, "m": 0.03, "l": 0.06})
    sched = Scheduler(ex, hbm_budget=100, max_inflight=3, max_batch=4, clock=clock)
    keys = ["s", "m", "l", "m", "s", "l", "l", "s", "m", "s"] * 3
    arr = list(poisson_arrivals(len(keys), rate=50.0, seed=1))
    reqs = _reqs(keys, arr)
    max_used = _drive(sched, clock, reqs)
    assert max_used <= 100
    assert len(sched.completed) == len(reqs) and not sched.rejected
    assert all(r.done >= r.admitted >= r.arrival for r in reqs)
    assert sched.used == 0


def test_fifo_admission_order_and_batch_limit():
    clock = Clock()
    ex = FakeExecutor(clock, {"a": 1}, {"a": 0.05})
    sched = Scheduler(ex, hbm_budget=1000, max_inflight=2, max_batch=3, clock=clock)
    reqs = _reqs(["a"] * 11, [0.0] * 11)
    _drive(sched, clock, reqs)
    order = [rid for h in ex.launches for rid in h["ids"]]
    assert order == list(range(11))
    assert all(len(h["ids"]) <= 3 for h in ex.launches)


def test_arrivals_join_while_earlier_work_runs():
    # the second request arrives while the first launch is still running and is
    # admitted into a new launch before the first completes
    clock = Clock()
    ex = FakeExecutor(clock, {"a": 1}, {"a": 0.2})
    sched = Scheduler(ex, hbm_budget=10, max_inflight=2, max_batch=8, clock=clock)
    r0, r1 = Request(0, 0.0, "a"), Request(1, 0.05, "a")
    _drive(sched, clock, [r0, r1])
    assert r1.admitted < r0.done
    assert len(ex.launches) == 2


def test_waits_for_memory_then_runs():
    clock = Clock()
    ex = FakeExecutor(clock, {"big": 80}, {"big": 0.1})
    sched = Scheduler(ex, hbm_budget=100, max_inflight=4, max_batch=4, clock=clock)
    reqs = _reqs(["big"] * 3, [0.0, 0.0, 0.0])
    _drive(sched, clock, reqs)
    # only one fits at a time: each starts after the previous one finished
    reqs.sort(key=lambda r: r.admitted)
    for a, b in zip(reqs, reqs[1:]):
        assert b.admitted >= a.done - 1e-12


def test_oversize_request_refused_not_blocking():
    clock = Clock()
    ex = FakeExecutor(clock, {"huge": 500, "s": 1}, {"huge": 1.0, "s": 0.01})
    sched = Scheduler(ex, hbm_budget=100, clock=clock)
    reqs = _reqs(["s", "huge", "s"], [0.0, 0.0, 0.0])
    _drive(sched, clock, reqs)
    assert [r.rid for r in sched.rejected] == [1]
    assert sorted(r.rid for r in sched.completed) == [0, 2]


def test_work_quantum_keeps_expensive_requests_apart():
    # launches group cheap requests up to the work limit; an expensive request gets a
    # launch of its own (and is never split or skipped: FIFO still holds)
    clock = Clock()
    ex = FakeExecutor(clock, {"s": 1, "l": 1}, {"s": 0.01, "l": 0.5})
    sched = Scheduler(ex, hbm_budget=1000, max_inflight=8, max_batch=24, clock=clock,
                      max_batch_cost=0.045)
    keys = ["s"] * 6 + ["l"] + ["s"] * 3
    for r in _reqs(keys, [0.0] * len(keys)):
        sched.submit(r)
    sched.step()
    assert [h["ids"] for h in ex.launches] == [[0, 1, 2, 3], [4, 5], [6], [7, 8, 9]]


def test_one_large_runs_expensive_requests_in_order_and_lets_cheap_ones_pass():
    clock = Clock()
    ex = FakeExecutor(clock, {"s": 1, "l": 1}, {"s": 0.01, "l": 0.5})
    sched = Scheduler(ex, hbm_budget=1000, max_inflight=4, max_batch=24, clock=clock,
                      max_batch_cost=0.045, one_large=True)
    keys = ["l", "l", "s", "s", "l", "s"]
    for r in _reqs(keys, [0.0] * len(keys)):
        sched.submit(r)
    sched.step()
    # the first expensive request runs; the second waits, the cheap ones behind it start
    assert [h["ids"] for h in ex.launches] == [[0], [2, 3], [5]]
    assert [r.rid for r in sched.queue] == [1, 4]
    clock.t = 0.6
    sched.step()
    assert [h["ids"] for h in ex.launches][3:] == [[1]]
    clock.t = 1.2
    sched.step()
    assert [h["ids"] for h in ex.launches][4:] == [[4]]


def test_invalid_limits():
    with pytest.raises(ValueError):
        Scheduler(None, 10, max_inflight=0)


def test_summary_percentiles():
    reqs = [Request(k, 0.0, "a") for k in range(100)]
    for k, r in enumerate(reqs):
        r.done = (k + 1) * 1e-3
    s = summarize(reqs, 0.0, 0.1)
    assert s["requests"] == 100
    assert math.isclose(s["p50_ms"], 50.0) and math.isclose(s["p99_ms"], 99.0)
    assert math.isclose(s["patterns_per_s"], 1000.0)
