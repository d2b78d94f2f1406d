"""The machine-peak probes behind bench.py's `peaks` field: the streaming copy
moves every byte exactly, and the matrix-core loop leaves finite sums and reports
the flops it executes."""
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2202_03411_amd import msft
    return torch, msft


@pytest.mark.parametrize("n", [4, 1000, 1 << 20, (1 << 20) + 12])
def test_copy_is_exact(env, n):
    torch, msft = env
    g = torch.Generator(device="cuda").manual_seed(n)
    src = torch.rand(n, device="cuda", generator=g)
    dst = torch.full_like(src, -1.0)
    msft.msft_copy(src, dst)
    torch.cuda.synchronize()
    assert torch.equal(src, dst)


@pytest.mark.parametrize("prec,per", [("fp32", 2 * 32 * 32 * 2), ("bf16x3", 2 * 32 * 32 * 16)])
def test_peak_probe_counts_and_finishes(env, prec, per):
    torch, msft = env
    nblocks, iters = 8, 50
    sink = torch.full((nblocks * 256,), float("nan"), device="cuda")
    flops = msft.msft_peak_mfma(prec, iters, nblocks, sink)
    torch.cuda.synchronize()
    # four chains per wave, four waves per workgroup
    assert flops == per * 4 * iters * 4 * nblocks
    assert bool(torch.isfinite(sink).all())
