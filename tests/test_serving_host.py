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
    """A launch takes the modelled time of its items (blocks x per-block time);
    memory and size of a request come from its key: key -> (io bytes, scratch bytes,
    blocks, seconds per block)."""

    def __init__(self, clock, spec):
        self.clock, self.spec = clock, spec
        self.launches = []
        self.completed = []

    def describe(self, req):
        req.io_bytes, req.ws_bytes, req.blocks, req.block_cost = self.spec[req.key][:4]
        req.wave_blocks = self.spec[req.key][4] if len(self.spec[req.key]) > 4 else 1

    def launch(self, items):
        dur = sum((b1 - b0) * r.block_cost for r, b0, b1 in items)
        h = {"end": self.clock() + dur, "ids": [r.rid for r, _, _ in items],
             "items": [(r.rid, b0, b1) for r, b0, b1 in items]}
        self.launches.append(h)
        return h

    def poll(self, h):
        return self.clock() >= h["end"]

    def finish(self, h, items):
        pass

    def complete(self, req):
        req.result = ("done", req.rid)
        self.completed.append(req.rid)


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
    ex = FakeExecutor(clock, {"s": (6, 4, 1, 0.01), "m": (20, 10, 3, 0.01), "l": (40, 20, 6, 0.01)})
    sched = Scheduler(ex, hbm_budget=100, max_inflight=3, max_batch=4, clock=clock, quantum=0.02)
    keys = ["s", "m", "l", "m", "s", "l", "l", "s", "m", "s"] * 3
    arr = list(poisson_arrivals(len(keys), rate=50.0, seed=1))
    reqs = _reqs(keys, arr)
    max_used = _drive(sched, clock, reqs)
    assert max_used <= 100
    assert len(sched.completed) == len(reqs) and not sched.rejected
    assert all(r.done >= r.admitted >= r.arrival for r in reqs)
    assert sched.used == 0


def test_fifo_order_and_batch_limit_without_quantum():
    clock = Clock()
    ex = FakeExecutor(clock, {"a": (1, 0, 5, 0.01)})
    sched = Scheduler(ex, hbm_budget=1000, max_inflight=2, max_batch=3, clock=clock)
    reqs = _reqs(["a"] * 11, [0.0] * 11)
    _drive(sched, clock, reqs)
    order = [rid for h in ex.launches for rid in h["ids"]]
    assert order == list(range(11))
    assert all(len(h["ids"]) <= 3 for h in ex.launches)
    # nothing is sliced without a quantum
    assert all(b0 == 0 and b1 == 5 for h in ex.launches for _, b0, b1 in h["items"])


def test_arrivals_join_while_earlier_work_runs():
    # the second request arrives while the first launch is still running and is
    # admitted into a new launch before the first completes
    clock = Clock()
    ex = FakeExecutor(clock, {"a": (1, 0, 1, 0.2)})
    sched = Scheduler(ex, hbm_budget=10, max_inflight=2, max_batch=8, clock=clock)
    r0, r1 = Request(0, 0.0, "a"), Request(1, 0.05, "a")
    _drive(sched, clock, [r0, r1])
    assert r1.admitted < r0.done
    assert len(ex.launches) == 2


def test_waits_for_memory_then_runs():
    clock = Clock()
    ex = FakeExecutor(clock, {"big": (60, 20, 1, 0.1)})
    sched = Scheduler(ex, hbm_budget=100, max_inflight=4, max_batch=4, clock=clock)
    reqs = _reqs(["big"] * 3, [0.0, 0.0, 0.0])
    _drive(sched, clock, reqs)
    # only one fits at a time: each starts after the previous one finished
    reqs.sort(key=lambda r: r.admitted)
    for a, b in zip(reqs, reqs[1:]):
        assert b.admitted >= a.done - 1e-12


def test_oversize_request_refused_not_blocking():
    clock = Clock()
    ex = FakeExecutor(clock, {"huge": (400, 100, 1, 1.0), "s": (1, 0, 1, 0.01)})
    sched = Scheduler(ex, hbm_budget=100, clock=clock)
    reqs = _reqs(["s", "huge", "s"], [0.0, 0.0, 0.0])
    _drive(sched, clock, reqs)
    assert [r.rid for r in sched.rejected] == [1]
    assert sorted(r.rid for r in sched.completed) == [0, 2]


def test_cheap_requests_grouped_up_to_the_quantum():
    # cheap requests share launches up to the work limit, in arrival order
    clock = Clock()
    ex = FakeExecutor(clock, {"s": (1, 1, 1, 0.01)})
    sched = Scheduler(ex, hbm_budget=1000, max_inflight=8, max_batch=24, clock=clock,
                      quantum=0.045)
    for r in _reqs(["s"] * 10, [0.0] * 10):
        sched.submit(r)
    sched.step()
    assert [h["ids"] for h in ex.launches] == [[0, 1, 2, 3], [4, 5, 6, 7], [8, 9]]


def test_expensive_requests_are_sliced_and_cheap_ones_pass_between_slices():
    clock = Clock()
    # l: 10 blocks of 0.01 s = 0.1 s of work, quantum 0.03 s -> slices of 3 blocks
    ex = FakeExecutor(clock, {"s": (1, 1, 1, 0.01), "l": (5, 2, 10, 0.01)})
    sched = Scheduler(ex, hbm_budget=1000, max_inflight=2, max_batch=24, clock=clock,
                      quantum=0.03)
    reqs = _reqs(["l", "l"], [0.0, 0.0])
    for r in reqs:
        sched.submit(r)
    sched.step()
    # one launch slot stays free for cheap arrivals: one slice of the oldest request
    assert [h["items"] for h in ex.launches] == [[(0, 0, 3)]]
    cheap = Request(2, 0.0, "s")
    sched.submit(cheap)
    sched.step()
    assert ex.launches[-1]["items"] == [(2, 0, 1)]
    _drive(sched, clock, [])
    slices = [it for h in ex.launches for it in h["items"]]
    # every block of each expensive request launched exactly once, oldest request first
    for rid in (0, 1):
        got = sorted((b0, b1) for r, b0, b1 in slices if r == rid)
        assert got == [(0, 3), (3, 6), (6, 9), (9, 10)]
    first1 = min(k for k, (r, _, _) in enumerate(slices) if r == 1)
    last0 = max(k for k, (r, _, _) in enumerate(slices) if r == 0)
    assert first1 > last0
    assert cheap.done < reqs[0].done
    assert all(r.done >= r.admitted for r in reqs) and sched.used == 0
    assert sorted(ex.completed) == [0, 1, 2]


def test_slices_of_one_request_charge_its_inputs_once():
    clock = Clock()
    ex = FakeExecutor(clock, {"l": (50, 10, 8, 0.01)})
    sched = Scheduler(ex, hbm_budget=75, max_inflight=3, max_batch=4, clock=clock, quantum=0.02)
    r = Request(0, 0.0, "l")
    sched.submit(r)
    sched.step()
    # inputs (50) once plus two slices' scratch (10 each) fit in 75; a third would not
    assert sched.used == 70 and len(sched.inflight) == 2
    _drive(sched, clock, [])
    assert r.done > 0 and sched.used == 0


def test_invalid_limits():
    with pytest.raises(ValueError):
        Scheduler(None, 10, max_inflight=0)
    with pytest.raises(ValueError):
        Scheduler(None, 10, quantum=0.0)


def test_summary_percentiles():
    reqs = [Request(k, 0.0, "a") for k in range(100)]
    for k, r in enumerate(reqs):
        r.done = (k + 1) * 1e-3
    s = summarize(reqs, 0.0, 0.1)
    assert s["requests"] == 100
    assert math.isclose(s["p50_ms"], 50.0) and math.isclose(s["p99_ms"], 99.0)
    assert math.isclose(s["patterns_per_s"], 1000.0)


def test_slices_are_whole_device_waves():
    # 40 blocks, 4 run at once (one wave = 4 x 0.01 s): a 0.09 s quantum gives slices
    # of two waves (8 blocks); a quantum below one wave still gives one whole wave
    clock = Clock()
    ex = FakeExecutor(clock, {"l": (5, 2, 40, 0.01, 4), "m": (5, 2, 10, 0.01, 4)})
    sched = Scheduler(ex, hbm_budget=1000, max_inflight=2, max_batch=4, clock=clock, quantum=0.09)
    sched.submit(Request(0, 0.0, "l"))
    _drive(sched, clock, [])
    sizes = [b1 - b0 for h in ex.launches for _, b0, b1 in h["items"]]
    assert sizes == [8, 8, 8, 8, 8]
    ex.launches.clear()
    sched = Scheduler(ex, hbm_budget=1000, max_inflight=2, max_batch=4, clock=clock, quantum=0.015)
    sched.submit(Request(1, clock.t, "m"))
    _drive(sched, clock, [])
    assert [b1 - b0 for h in ex.launches for _, b0, b1 in h["items"]] == [4, 4, 2]


def test_latency_log_one_line_per_request():
    import io
    import json
    clock = Clock()
    spec = {"a": (10, 5, 4, 0.002), "b": (10, 5, 40, 0.002), "huge": (10 ** 6, 0, 1, 0.001)}
    ex = FakeExecutor(clock, spec)
    log = io.StringIO()
    sched = Scheduler(ex, hbm_budget=100, max_inflight=2, max_batch=4, clock=clock, quantum=0.02,
                      latency_log=log)
    reqs = [Request(k, 0.003 * k, "a" if k % 3 else "b") for k in range(9)] + [Request(99, 0.01, "huge")]
    _drive(sched, clock, reqs)
    recs = [json.loads(line) for line in log.getvalue().splitlines()]
    assert len(recs) == len(reqs)
    by = {r["rid"]: r for r in recs}
    assert by[99]["status"] == "rejected" and by[99]["latency_ms"] is None and by[99]["launches"] == 0
    for r in sched.completed:
        e = by[r.rid]
        assert e["status"] == "completed"
        assert math.isclose(e["latency_ms"], 1e3 * r.latency, rel_tol=1e-12)
        assert 0.0 <= e["queue_ms"] <= e["latency_ms"]
        assert e["blocks"] == r.blocks and e["launches"] >= 1
    # an expensive request went out in several slices
    assert max(by[r.rid]["launches"] for r in sched.completed if r.key == "b") > 1
    # completed lines come in completion order
    done = [e["done_s"] for e in recs if e["status"] == "completed"]
    assert done == sorted(done)
