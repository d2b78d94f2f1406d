"""GPU serving: requests of mixed grid and detector sizes arriving over time,
served in overlapping batched launches; every result must equal, bit
for bit, the same request simulated alone."""
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2202_03411_amd import msft, serving
    pool = serving.ShapePool(torch, grids=(48, 64, 80), per_kind=2, box=700.0, seed=3)
    return torch, msft, serving, pool


def _check_alone(torch, plans, done):
    for r in done:
        p = plans.get(r.key)
        d, b = r.payload
        alone = p.simulate(d, b)
        torch.cuda.synchronize()
        assert torch.equal(alone, r.result), f"request {r.rid} differs alone vs in the mix"


@pytest.mark.parametrize("precision", ["fp32", "bf16x3"])
def test_stream_results_equal_alone(env, precision):
    torch, msft, serving, pool = env
    plans = serving.PlanCache(msft, precision)
    try:
        reqs = serving.make_requests(pool, 40, seed=11, rate=400.0, grids=(48, 64, 80),
                                     dets=(16, 33, 48))
        s, done = serving.serve(torch, msft, plans, reqs, batched=True, slots=3, max_batch=6)
        print(f"  {precision}: {s}")
        assert s["requests"] == 40 and s["rejected"] == 0
        _check_alone(torch, plans, done)
    finally:
        plans.close()


def test_small_budget_waits_and_plain_mode(env):
    torch, msft, serving, pool = env
    plans = serving.PlanCache(msft, "fp32")
    try:
        reqs = serving.make_requests(pool, 16, seed=12, rate=None, grids=(48, 64, 80),
                                     dets=(16, 33, 48))
        ex = serving.GpuExecutor(plans, torch, nstreams=3, batched=True)
        biggest = max(ex.footprint(r) for r in reqs)
        s, done = serving.serve(torch, msft, plans, reqs, batched=True, hbm_budget=2 * biggest)
        assert s["requests"] == 16
        _check_alone(torch, plans, done)
        reqs = serving.make_requests(pool, 16, seed=12, rate=None, grids=(48, 64, 80),
                                     dets=(16, 33, 48))
        s, done = serving.serve(torch, msft, plans, reqs, batched=False)
        assert s["requests"] == 16
        _check_alone(torch, plans, done)
    finally:
        plans.close()
