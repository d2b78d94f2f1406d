"""GPU serving and batching, through the C ABI.

* Requests of mixed grid and detector sizes arrive over time and are served in
  overlapping batched launches, expensive ones cut into pixel-block slices:
  every result must equal, bit for bit, the same request simulated alone.
* Batched and served results against the FP64 oracle: one msft_simulate_batch
  over plans of different grids and detectors (one request split into tile
  ranges), and a served stream of the serving workload's families (a fresh
  seeded ellipsoid or harmonic body per request, rendered on the GPU at launch),
  each request compared with the oracle on its own seeded pixels.
Tolerances are the relative L2 intensity errors required of the two precisions.
"""
import numpy as np
import pytest

import oracle
from paper_2202_03411_amd import inputs

pytestmark = pytest.mark.gpu

TOL = {"fp32": 1e-5, "bf16x3": 1e-3}


@pytest.fixture(scope="module")
def env():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2202_03411_amd import msft, serving
    return torch, msft, serving


def _check_alone(torch, plans, done):
    for r in done:
        p = plans.get(r.key)
        d, b = r.payload
        alone = p.simulate(d, b)
        torch.cuda.synchronize()
        assert torch.equal(alone, r.result), f"request {r.rid} differs alone vs in the mix"


def _rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


@pytest.mark.parametrize("precision", ["fp32", "bf16x3"])
@pytest.mark.parametrize("quantum", [None, 1e-5])
def test_stream_results_equal_alone(env, precision, quantum):
    torch, msft, serving = env
    plans = serving.PlanCache(msft, precision)
    try:
        reqs = serving.make_requests(40, seed=11, rate=400.0, grids=(48, 64, 80),
                                     dets=(16, 33, 48))
        kw = {} if quantum is None else {"quantum_s": quantum}
        s, done = serving.serve(torch, msft, plans, reqs, batched=True, slots=3, max_batch=6,
                                keep_inputs=True, **kw)
        print(f"  {precision} quantum {quantum}: {s}", flush=True)
        assert s["requests"] == 40 and s["rejected"] == 0
        _check_alone(torch, plans, done)
    finally:
        plans.close()


def test_small_budget_waits_and_plain_mode(env):
    torch, msft, serving = env
    plans = serving.PlanCache(msft, "fp32")
    try:
        reqs = serving.make_requests(16, seed=12, rate=None, grids=(48, 64, 80), dets=(16, 33, 48))
        ex = serving.GpuExecutor(plans, torch, nstreams=3, batched=True)
        for r in reqs:
            ex.describe(r)
        biggest = max(r.footprint for r in reqs)
        s, done = serving.serve(torch, msft, plans, reqs, batched=True, hbm_budget=2 * biggest,
                                keep_inputs=True)
        assert s["requests"] == 16
        _check_alone(torch, plans, done)
        reqs = serving.make_requests(16, seed=12, rate=None, grids=(48, 64, 80), dets=(16, 33, 48))
        s, done = serving.serve(torch, msft, plans, reqs, batched=False, keep_inputs=True)
        assert s["requests"] == 16
        _check_alone(torch, plans, done)
    finally:
        plans.close()


@pytest.mark.parametrize("precision", ["fp32", "bf16x3"])
def test_batch_across_plans_matches_oracle(env, precision):
    # one msft_simulate_batch over three plans of different grids and detectors, the
    # second request split into two tile ranges of the same launch
    torch, msft, serving = env
    cases = [((64, 64, 64), 96, 700.0 / 64, 51), ((48, 40, 56), 200, 8.0, 52),
             ((96, 96, 96), 64, 700.0 / 96, 53)]
    plans, reqs, keep = [], [], []
    try:
        for shape, det, pitch, seed in cases:
            rng = np.random.default_rng(inputs.SEED_BASE + seed)
            d = rng.uniform(0.0, 0.05, shape).astype(np.float32)
            b = rng.uniform(0.0, 0.05, shape).astype(np.float32)
            p = msft.Plan(45.0, 60.0, det, shape, (pitch,) * 3, precision, "msft")
            plans.append(p)
            dt, bt = torch.from_numpy(d).cuda(), torch.from_numpy(b).cuda()
            I = torch.full((p.npix,), float("nan"), device="cuda")
            keep.append((p, d, b, I, det, pitch))
            nb = -(-p.npix // msft.msft_pixel_block())
            if len(keep) == 2:
                cut = nb // 3
                reqs += [(p.handle, dt, bt, I, None, (0, cut)), (p.handle, dt, bt, I, None, (cut, nb))]
            else:
                reqs.append((p.handle, dt, bt, I, None))
        print(f"[gpu] batch of {len(reqs)} items over 3 plans, {precision}", flush=True)
        ws = msft.workspace_tensor(msft.msft_batch_query(reqs), "cuda")
        msft.msft_simulate_batch(reqs, ws)
        torch.cuda.synchronize()
        for k, (p, d, b, I, det, pitch) in enumerate(keep):
            Ig = I.cpu().numpy().astype(np.float64)
            assert not np.isnan(Ig).any()
            pix = inputs.random_pixels(det, 96, seed=60 + k)
            Io, _ = oracle.simulate(oracle.MSFT, 45.0, 60.0, det, d.astype(np.float64),
                                    b.astype(np.float64), (pitch,) * 3, pixels=pix)
            err = _rel(Ig[pix], Io)
            print(f"  plan {k}: grid {d.shape} det {det}: rel L2 {err:.2e}", flush=True)
            assert err <= TOL[precision], (k, err)
    finally:
        for p in plans:
            p.close()


@pytest.mark.parametrize("precision", ["fp32", "bf16x3"])
def test_served_stream_matches_oracle(env, precision):
    # 36 requests of the serving workload's families arriving as a Poisson stream;
    # grids 64-128^3 in the 700 nm box and 256^2 / 512^2 detectors to 60 deg, every
    # request its own seeded shape; expensive requests are sliced (5 ms quantum)
    torch, msft, serving = env
    plans = serving.PlanCache(msft, precision)
    try:
        reqs = serving.make_requests(36, seed=71, rate=60.0, grids=(64, 96, 128), dets=(256, 512))
        s, done = serving.serve(torch, msft, plans, reqs, batched=True, keep_inputs=True)
        print(f"[gpu] served stream {precision}: {s}", flush=True)
        assert s["requests"] == 36 and s["rejected"] == 0
        kinds = set()
        worst = 0.0
        for r in done:
            wavelength, theta, det, grid, pitch, mode = r.key
            d, b = (t.cpu().numpy().astype(np.float64) for t in r.payload)
            assert d.any(), f"request {r.rid}: empty target"
            kinds.add(d.shape)
            pix = inputs.random_pixels(det, 48, seed=1000 + r.rid)
            Io, _ = oracle.simulate(oracle.MSFT, wavelength, theta, det, d, b, pitch, pixels=pix)
            err = _rel(r.result.cpu().numpy().astype(np.float64)[pix], Io)
            worst = max(worst, err)
            assert err <= TOL[precision], (r.rid, r.key, err)
        print(f"  worst rel L2 over {len(done)} requests: {worst:.2e}", flush=True)
        assert len(kinds) == 3
    finally:
        plans.close()
