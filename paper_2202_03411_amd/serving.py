"""Continuous-batching server for MSFT pattern requests.

Requests of uneven grid and detector sizes arrive over time (the candidate
simulations of forward fitting, Sec. 6).  The scheduler keeps one plan per
geometry resident (q map and twiddle tables), admits queued requests while the
in-flight HBM footprint stays under a budget and a launch slot is free, and
runs each admitted group as one batched launch
(``msft_simulate_batch``).  Several launches can be in flight on separate
streams, so requests that arrive while others are on the GPU start as soon as
a slot and memory free up and their work overlaps the tail of earlier
launches.  Per-request latency is arrival -> completion as seen by the host.

The scheduler talks to an executor object; ``GpuExecutor`` drives the library,
tests use a fake one with modelled durations.
"""
from __future__ import annotations

import collections
import dataclasses
import json
import math
import time
from typing import Callable


@dataclasses.dataclass
class Request:
    rid: int
    arrival: float                 # seconds, on the server clock
    key: tuple                     # geometry key: (wavelength, theta, det_n, grid, pitch, mode)
    payload: object = None         # executor inputs: a shape to render, or device (delta, beta)
    admitted: float = math.nan     # first work launched
    done: float = math.nan
    io_bytes: int = 0              # inputs and outputs, held from the first launch to completion
    ws_bytes: int = 0              # scratch of one launch item of this request
    blocks: int = 1                # pixel blocks (work items) of the request
    block_cost: float = 0.0        # executor's estimate of one block's device time (s)
    wave_blocks: int = 1           # blocks the device runs at once: slices are multiples of it
    next_block: int = 0            # first block not launched yet
    open_items: int = 0            # launched items not finished yet
    launches: int = 0              # launches that carried some of its blocks
    result: object = None
    state: object = None           # executor's per-request device state

    @property
    def latency(self):
        return self.done - self.arrival

    @property
    def cost(self):
        return self.blocks * self.block_cost

    @property
    def footprint(self):
        return self.io_bytes + self.ws_bytes


@dataclasses.dataclass
class Batch:
    items: list                    # (request, first block, end block)
    handle: object
    footprint: int
    launched: float
    large: bool = False


class Scheduler:
    """Admission + batching policy, independent of the device.

    executor must provide:
      describe(req)    fill req.io_bytes, req.ws_bytes, req.blocks, req.block_cost,
                       req.wave_blocks
      launch(items) -> handle                 (asynchronous; items: (req, b0, b1))
      poll(handle) -> bool                    (True once finished)
      finish(handle, items)                   (release the launch's buffers)
      complete(req)                           (all of req's blocks are done: set req.result)

    A launch holds at most `quantum` seconds of estimated device work.  A request
    whose whole cost fits the quantum is cheap: cheap requests are grouped in arrival
    order, up to the quantum and max_batch, and go first.  An expensive request is cut
    into slices of pixel blocks worth about one quantum each (a whole number of device
    waves of blocks, at least one, so that a slice fills the device), launched one
    slice per launch, oldest request first; cheap requests that arrive meanwhile start between
    its slices instead of waiting for all of it.  At most max_inflight launches are in
    flight, so the device always has queued work; expensive slices leave one launch
    slot to cheap arrivals.  Memory: a request's inputs and outputs are charged from
    its first launch to its completion, each launch item's scratch while it runs; the
    total stays within hbm_budget.  With quantum None nothing is sliced and requests
    are grouped first-come first-served up to max_batch.

    latency_log, a writable text stream, receives one JSON line per finished request
    (completed or rejected), in the order they finish: its id, geometry key, arrival,
    first launch and completion times (seconds on the scheduler's clock), latency and
    queueing time (ms), pixel blocks and the number of launches that carried them.
    """

    def __init__(self, executor, hbm_budget: int, max_inflight: int = 3, max_batch: int = 24,
                 clock: Callable[[], float] = time.perf_counter, quantum=None, latency_log=None):
        if max_inflight < 1 or max_batch < 1:
            raise ValueError("max_inflight and max_batch must be >= 1")
        if quantum is not None and not quantum > 0:
            raise ValueError("quantum must be > 0 or None")
        self.ex = executor
        self.budget = int(hbm_budget)
        self.max_inflight = max_inflight
        self.max_batch = max_batch
        self.quantum = quantum
        self.clock = clock
        self.queue: list = []          # requests with blocks not launched yet, arrival order
        self.inflight: list = []
        self.used = 0
        self.completed: list = []
        self.rejected: list = []
        self.log = latency_log

    def _log(self, r, status):
        if self.log is None:
            return

        def num(v):
            return None if v is None or (isinstance(v, float) and math.isnan(v)) else v
        done, adm = num(r.done), num(r.admitted)
        rec = {"rid": r.rid, "status": status, "key": repr(r.key), "arrival_s": r.arrival,
               "admitted_s": adm, "done_s": done,
               "latency_ms": None if done is None else 1e3 * (done - r.arrival),
               "queue_ms": None if adm is None else 1e3 * (adm - r.arrival),
               "blocks": r.blocks, "launches": r.launches}
        self.log.write(json.dumps(rec) + "\n")

    def submit(self, req: Request):
        self.ex.describe(req)
        req.next_block = 0
        req.open_items = 0
        req.launches = 0
        if req.footprint > self.budget:
            # could never be admitted: refuse instead of blocking the queue
            self.rejected.append(req)
            self._log(req, "rejected")
            return False
        self.queue.append(req)
        return True

    def retire(self):
        now = self.clock()
        still = []
        for b in self.inflight:
            if self.ex.poll(b.handle):
                self.ex.finish(b.handle, b.items)
                self.used -= b.footprint
                for r, _, _ in b.items:
                    r.open_items -= 1
                    if r.open_items == 0 and r.next_block == r.blocks:
                        r.done = now
                        self.ex.complete(r)
                        self.used -= r.io_bytes
                        self.completed.append(r)
                        self._log(r, "completed")
            else:
                still.append(b)
        self.inflight = still

    def _cheap(self, r):
        return self.quantum is None or (r.next_block == 0 and r.cost <= self.quantum)

    def _take(self, items, r, b0, b1):
        items.append((r, b0, b1))
        r.next_block = b1
        r.open_items += 1
        r.launches += 1
        need = r.ws_bytes + (r.io_bytes if b0 == 0 else 0)
        return need

    def admit_and_launch(self):
        """Form at most one launch: cheap requests first (arrival order), else one
        slice of the oldest expensive request."""
        if len(self.inflight) >= self.max_inflight or not self.queue:
            return None
        items, foot, cost = [], 0, 0.0
        k = 0
        while k < len(self.queue) and len(items) < self.max_batch:
            r = self.queue[k]
            if not self._cheap(r):
                k += 1
                continue
            need = r.io_bytes + r.ws_bytes
            if self.used + foot + need > self.budget:
                break
            if items and self.quantum is not None and cost + r.cost > self.quantum:
                break
            foot += self._take(items, r, 0, r.blocks)
            cost += r.cost
            del self.queue[k]
        large = False
        if not items:
            big = [r for r in self.queue if not self._cheap(r)]
            n_large = sum(1 for b in self.inflight if b.large)
            if big and (self.max_inflight == 1 or n_large < self.max_inflight - 1):
                r = big[0]
                wave = max(1, r.wave_blocks)
                per = (max(1, int(self.quantum / (r.block_cost * wave))) * wave
                       if r.block_cost > 0 else r.blocks)
                b0 = r.next_block
                b1 = min(r.blocks, b0 + per)
                need = r.ws_bytes + (r.io_bytes if b0 == 0 else 0)
                if self.used + need <= self.budget:
                    foot += self._take(items, r, b0, b1)
                    if b1 == r.blocks:
                        self.queue.remove(r)
                    large = True
        if not items:
            return None
        now = self.clock()
        for r, b0, _ in items:
            if b0 == 0:
                r.admitted = now
        handle = self.ex.launch(items)
        ws = sum(r.ws_bytes for r, _, _ in items)
        b = Batch(items, handle, ws, now, large)
        self.inflight.append(b)
        self.used += foot
        return b

    def idle(self):
        return not self.queue and not self.inflight

    def step(self):
        self.retire()
        launched = 0
        while self.admit_and_launch() is not None:
            launched += 1
        return launched


def run_stream(scheduler: Scheduler, requests, poll_sleep: float = 2e-4, progress=None):
    """Replay requests at their arrival times (seconds from start) through a scheduler.
    `progress(done, total)` is called whenever another 512 requests have completed."""
    pending = sorted(requests, key=lambda r: r.arrival)
    t0 = scheduler.clock()
    for r in pending:
        r.arrival += t0
    i = 0
    reported = 0
    while i < len(pending) or not scheduler.idle():
        if progress is not None and len(scheduler.completed) >= reported + 512:
            reported = len(scheduler.completed) // 512 * 512
            progress(reported, len(pending))
        now = scheduler.clock()
        while i < len(pending) and pending[i].arrival <= now:
            scheduler.submit(pending[i])
            i += 1
        launched = scheduler.step()
        if not launched and i < len(pending) and scheduler.idle():
            wait = pending[i].arrival - scheduler.clock()
            if wait > 0:
                time.sleep(min(wait, 0.01))
        elif not launched:
            time.sleep(poll_sleep)
    return t0


def poisson_arrivals(n: int, rate: float, seed: int):
    """Arrival times (s) of a Poisson process of the given rate."""
    import numpy as np
    rng = np.random.default_rng(seed)
    return np.cumsum(rng.exponential(1.0 / rate, size=n))


def summarize(requests, t0: float, t_end: float):
    lat = sorted(r.latency for r in requests)

    def pct(p):
        if not lat:
            return math.nan
        k = min(len(lat) - 1, max(0, int(math.ceil(p / 100.0 * len(lat))) - 1))
        return lat[k]

    span = t_end - t0
    return {"requests": len(lat), "makespan_s": span,
            "patterns_per_s": len(lat) / span if span > 0 else math.nan,
            "p50_ms": 1e3 * pct(50), "p99_ms": 1e3 * pct(99), "max_ms": 1e3 * (lat[-1] if lat else math.nan),
            "mean_ms": 1e3 * (sum(lat) / len(lat) if lat else math.nan)}


# ---------------------------------------------------------------------------
# GPU executor
# ---------------------------------------------------------------------------

class PlanCache:
    """One resident plan per (geometry, precision); plans are built on first use.

    With calibrate (the default) a new plan times two forward passes of an empty
    volume on the device, and the second one's duration per pixel block becomes the
    plan's block_cost: the scheduler's work estimates are the plan's measured rate,
    not a constant."""

    def __init__(self, msft, precision: str, device: int = 0, calibrate: bool = True):
        self.msft = msft
        self.precision = precision
        self.device = device
        self.calibrate = calibrate
        self.plans = {}
        self.block_cost = {}

    def get(self, key):
        p = self.plans.get(key)
        if p is None:
            wavelength, theta, det_n, grid, pitch, mode = key
            p = self.msft.Plan(wavelength, theta, det_n, grid, pitch, self.precision, mode,
                               self.device)
            self.plans[key] = p
            self.block_cost[key] = self._measure(p) if self.calibrate else 0.0
        return p

    def blocks(self, key):
        return -(-self.get(key).npix // self.msft.msft_pixel_block())

    def _measure(self, p):
        import torch
        dev = p.device
        d = torch.zeros(p.grid, dtype=torch.float32, device=dev)
        I = torch.empty(p.npix, dtype=torch.float32, device=dev)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        p.simulate(d, d, out=I)
        e0.record()
        p.simulate(d, d, out=I)
        e1.record()
        torch.cuda.synchronize(dev)
        return e0.elapsed_time(e1) * 1e-3 / (-(-p.npix // self.msft.msft_pixel_block()))

    def resident_bytes(self):
        return sum(p.resident_bytes for p in self.plans.values())

    def close(self):
        for p in self.plans.values():
            p.close()
        self.plans.clear()
        self.block_cost.clear()


@dataclasses.dataclass
class Shape:
    """A request's target, rendered on the device when its first work is launched:
    an ellipsoid (semi-axes `axes`, body axes the columns of `rot`) or a star body
    r0 (1 + sum c_lm Y_lm) (`coeffs`: (lmax + 1)^2 values at l*l + l + m)."""
    kind: str
    axes: object = None
    rot: object = None
    r0: float = 0.0
    coeffs: object = None
    lmax: int = 8
    delta0: float = 0.01
    beta0: float = 0.02


class _ReqState:
    __slots__ = ("delta", "beta", "out", "ready", "stream")

    def __init__(self):
        self.delta = self.beta = self.out = self.ready = None
        self.stream = -1


class GpuExecutor:
    """Runs each launch's items (request, pixel blocks) as one msft_simulate_batch.

    Every in-flight launch owns one stream of a small pool (default priority) and
    its own workspace, so launches overlap on the device.  A request's target is
    rendered (msft_render_ellipsoid / msft_render_sh) on the stream of its first
    launch, into buffers that live until the request completes; later slices of
    the request on other streams wait for that render.  With ``batched=False``
    every request is its own render + msft_simulate on one stream (the plain
    one-pattern-per-launch form), reusing the plan's workspace.  keep_inputs keeps
    each request's rendered delta and beta on the request after it completes.
    """

    def __init__(self, plans: PlanCache, torch, nstreams: int = 3, batched: bool = True,
                 keep_inputs: bool = False):
        self.plans = plans
        self.torch = torch
        self.msft = plans.msft
        self.batched = batched
        self.keep_inputs = keep_inputs
        n = nstreams if batched else 1
        self.streams = [torch.cuda.Stream() for _ in range(n)]
        self.free = list(range(n))
        # pixel blocks resident at once: compute units x workgroups per CU of the
        # contraction (two of the FP32 three-product kernel, one of the BF16 kernel)
        cus = torch.cuda.get_device_properties(plans.device).multi_processor_count
        self.wave_blocks = cus * (2 if plans.precision == "fp32" else 1)

    def describe(self, req):
        p = self.plans.get(req.key)
        V = p.grid[0] * p.grid[1] * p.grid[2]

        def r256(b):
            return -(-b // 256) * 256
        req.io_bytes = 2 * r256(4 * V) + r256(4 * p.npix)
        # msft_plan_query's per-request bytes less the inputs, intensity and
        # amplitude: the forward scratch of one batch item
        req.ws_bytes = p.per_request_bytes - 2 * r256(4 * V) - r256(4 * p.npix) - r256(8 * p.npix)
        if not self.batched:
            req.ws_bytes = 0           # one stream: the plan's own workspace
        req.blocks = self.plans.blocks(req.key)
        req.block_cost = self.plans.block_cost.get(req.key, 0.0)
        req.wave_blocks = self.wave_blocks

    def _render(self, req, p):
        torch, msft = self.torch, self.msft
        st = _ReqState()
        sh = req.payload
        if isinstance(sh, Shape):
            g = msft.make_shape_grid(p.grid, p.pitch, 0.0, sh.delta0, sh.beta0)
            st.delta = torch.empty(p.grid, dtype=torch.float32, device=p.device)
            st.beta = torch.empty_like(st.delta)
            if sh.kind == "ellipsoid":
                msft.msft_render_ellipsoid(g, sh.axes, sh.rot, st.delta, st.beta)
            else:
                c = torch.from_numpy(sh.coeffs).to(p.device)
                msft.msft_render_sh(g, sh.lmax, sh.r0, c, st.delta, st.beta)
        else:
            st.delta, st.beta = sh
        st.out = torch.empty(p.npix, dtype=torch.float32, device=p.device)
        return st

    def launch(self, items):
        torch = self.torch
        sidx = self.free.pop() if self.batched else 0
        s = self.streams[sidx]
        reqs, keep = [], []
        with torch.cuda.stream(s):
            for r, b0, b1 in items:
                p = self.plans.get(r.key)
                if r.state is None:
                    r.state = self._render(r, p)
                    r.state.stream = sidx
                    if self.batched and b1 < r.blocks:
                        r.state.ready = torch.cuda.Event()
                        r.state.ready.record(s)
                elif r.state.stream != sidx and r.state.ready is not None:
                    s.wait_event(r.state.ready)
                st = r.state
                if self.batched:
                    reqs.append((p.handle, st.delta, st.beta, st.out, None, (b0, b1)))
                else:
                    self.msft.msft_simulate(p.handle, st.delta, st.beta, st.out, None,
                                            p.workspace(), stream=s)
            if self.batched:
                ws = self.msft.workspace_tensor(self.msft.msft_batch_query(reqs), p.device)
                self.msft.msft_simulate_batch(reqs, ws, stream=s)
                keep.append(ws)
            ev = torch.cuda.Event()
            ev.record(s)
        return {"event": ev, "stream": sidx, "keep": keep}

    def poll(self, handle):
        return handle["event"].query()

    def finish(self, handle, items):
        handle["keep"].clear()
        if self.batched:
            self.free.append(handle["stream"])

    def complete(self, req):
        st = req.state
        req.result = st.out
        req.state = None
        if self.keep_inputs:
            req.payload = (st.delta, st.beta)


# ---------------------------------------------------------------------------
# seeded request streams (a fresh shape per request, rendered on the device)
# ---------------------------------------------------------------------------

SERVE_GRIDS = (64, 96, 128, 192)
SERVE_DETS = (256, 512, 1024)


def random_shape(rng, box=700.0, delta0=0.01, beta0=0.02):
    """Half ellipsoids (semi-axes U[80, 250] nm, Haar-random orientation), half
    l <= 8 harmonic bodies (R0 ~ U[80, 170] nm, c ~ N(0, 0.08^2) for 1 <= l <= 8,
    redrawn until r_max <= 340 nm), in the fixed box shared by every request."""
    import numpy as np

    from . import inputs
    if rng.random() < 0.5:
        return Shape("ellipsoid", axes=rng.uniform(80.0, 250.0, size=3),
                     rot=inputs.haar_rotation(rng), delta0=delta0, beta0=beta0)
    while True:
        r0 = float(rng.uniform(80.0, 170.0))
        coeffs = inputs.sh_coefficients(rng, 1, 8, 0.08)
        _, rmax = inputs.sh_radius_range(coeffs, r0, 91, 181)
        if rmax <= 0.5 * box - 10.0:
            break
    cvec = np.zeros(81, np.float32)
    for l, m, v in coeffs:
        cvec[l * l + l + m] = v
    return Shape("harmonic", r0=r0, coeffs=cvec, lmax=8, delta0=delta0, beta0=beta0)


def make_requests(count, seed, rate=None, wavelength=45.0, theta=60.0, grids=SERVE_GRIDS,
                  dets=SERVE_DETS, box=700.0):
    """Seeded requests: uniform grid and detector size, a fresh random shape each;
    Poisson arrivals at `rate` per second, or all at t = 0 when rate is None."""
    import numpy as np
    rng = np.random.default_rng(seed)
    arr = poisson_arrivals(count, rate, seed + 1) if rate else np.zeros(count)
    out = []
    for k in range(count):
        n = int(rng.choice(grids))
        det = int(rng.choice(dets))
        pitch = box / n
        key = (wavelength, theta, det, (n, n, n), (pitch, pitch, pitch), "msft")
        out.append(Request(k, float(arr[k]), key, random_shape(rng, box)))
    return out


def serve(torch, msft, plans, requests, batched=True, hbm_budget=16 << 30, slots=4, max_batch=24,
          quantum_s=0.005, progress=None, keep_inputs=False, latency_log=None):
    """Run a request list through the server; returns (summary, requests).  A batched
    launch holds at most quantum_s of the plans' measured work: expensive requests
    are sliced into pixel-block ranges of that size (None: no slicing).  latency_log:
    a text stream for the per-request JSON lines (Scheduler)."""
    ex = GpuExecutor(plans, torch, nstreams=slots, batched=batched, keep_inputs=keep_inputs)
    sched = Scheduler(ex, hbm_budget, max_inflight=slots if batched else 1 << 30,
                      max_batch=max_batch if batched else 1,
                      quantum=quantum_s if batched else None, latency_log=latency_log)
    t0 = run_stream(sched, requests, progress=progress)
    torch.cuda.synchronize()
    t_end = max(r.done for r in sched.completed) if sched.completed else t0
    s = summarize(sched.completed, t0, t_end)
    s["rejected"] = len(sched.rejected)
    s["mode"] = "batched" if batched else "plain"
    return s, sched.completed


class _TaggedLog:
    """Adds the run's name to each JSON line written through it."""

    def __init__(self, f, run):
        self.f, self.run = f, run

    def write(self, line):
        rec = json.loads(line)
        rec["run"] = self.run
        self.f.write(json.dumps(rec) + "\n")


def benchmark(count=96, precision="fp32", loads=(0.8,), seed=20220205, device=0, plain=True,
              log=None, capacity=None, latency_log=None):
    """The mixed-size stream served three ways: offline (all requests at t = 0),
    whose batched throughput is the measured capacity, then Poisson arrivals at
    each offered load rho * capacity.  Every stream runs batched and, if `plain`,
    as one pattern per launch on one stream.  A given capacity (patterns/s, from an
    earlier offline run of the same stream) skips the offline runs.  latency_log: a
    path that receives every run's per-request JSON lines, each tagged with its run."""
    import torch

    from . import msft
    plans = PlanCache(msft, precision, device)
    probe = make_requests(count, seed, None)
    for r in probe:
        plans.get(r.key)          # plans and twiddles resident before the clock starts
    out = {"precision": precision, "requests": count, "resident_plans": len(plans.plans),
           "resident_bytes": plans.resident_bytes(),
           "stream": "C3 families: grids {64,96,128,192}^3 in a 700 nm box, detectors "
                     "{256,512,1024}^2 to 60 deg, lambda 45 nm, a fresh seeded ellipsoid or "
                     "l <= 8 harmonic body per request rendered on the GPU at launch"}

    def run(name, rate, batched):
        reqs = make_requests(count, seed, rate)
        mode = "batched" if batched else "plain"
        prog = (lambda d, n: log(f"{name} {mode}: {d}/{n} done")) if log else None
        if latency_log:
            with open(latency_log, "a") as f:
                s, _ = serve(torch, msft, plans, reqs, batched=batched, progress=prog,
                             latency_log=_TaggedLog(f, f"{name}_{mode}"))
        else:
            s, _ = serve(torch, msft, plans, reqs, batched=batched, progress=prog)
        out[f"{name}_{s['mode']}"] = s
        if log:
            log(f"{name} {mode}: {s['patterns_per_s']:.2f} patterns/s, p50 {s['p50_ms']:.1f} ms, "
                f"p99 {s['p99_ms']:.1f} ms")
        return s

    if capacity is None:
        cap = run("offline", None, True)["patterns_per_s"]
        if plain:
            run("offline", None, False)
    else:
        cap = float(capacity)
    out["capacity_patterns_per_s"] = cap
    for rho in loads:
        rate = rho * cap
        out[f"offered_rate_rho{rho:g}_per_s"] = rate
        run(f"poisson_rho{rho:g}", rate, True)
        if plain:
            run(f"poisson_rho{rho:g}", rate, False)
    plans.close()
    return out


if __name__ == "__main__":
    import argparse
    import json
    import sys
    ap = argparse.ArgumentParser(description="serve a seeded stream of MSFT requests")
    ap.add_argument("--requests", type=int, default=96)
    ap.add_argument("--precision", choices=["fp32", "bf16x3"], default="fp32")
    ap.add_argument("--loads", type=float, nargs="+", default=[0.8],
                    help="offered loads as fractions of the measured batched capacity")
    ap.add_argument("--no-plain", action="store_true", help="skip the one-pattern-per-launch runs")
    ap.add_argument("--capacity", type=float, default=None,
                    help="batched capacity (patterns/s) of an earlier offline run: skip the offline runs")
    ap.add_argument("--latency-log", default=None,
                    help="append one JSON line per request (every run, tagged) to this file")
    args = ap.parse_args()
    res = benchmark(args.requests, args.precision, tuple(args.loads), plain=not args.no_plain,
                    log=lambda m: print(f"[serving] {m}", file=sys.stderr, flush=True),
                    capacity=args.capacity, latency_log=args.latency_log)
    print(json.dumps(res))
