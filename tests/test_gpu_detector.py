"""GPU Ideal detector against the FP64 oracle's (Sec. 5.2, photon statistics).

Both sides draw from their own Philox4x64-10 stream per pixel and decide every
count in FP64, so the counts agree exactly; the expected counts agree to FP32
rounding.  Intensities are seeded and synthetic (log-uniform over the range of a
diffraction pattern, with zero, negative and non-finite pixels), so no input of
the oracle comes from the library.
"""
import math

import numpy as np
import pytest

import oracle

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2202_03411_amd import msft
    return torch, msft


def _intensity(n, seed, lo=-4.0, hi=20.0):
    rng = np.random.default_rng(seed)
    I = np.exp(rng.uniform(lo, hi, n * n)).astype(np.float32)
    I[rng.integers(0, n * n, 8)] = 0.0
    return I


def _detect(env, n, theta, wl, I, fluence, seed):
    torch, msft = env
    with msft.Plan(wl, theta, n, (4, 4, 4), (2.0, 2.0, 2.0), "fp32", "msft") as plan:
        counts, mu = plan.detect_ideal(torch.from_numpy(I).cuda(), fluence, seed, expected=True)
        torch.cuda.synchronize()
        return counts.cpu().numpy().astype(np.float64), mu.cpu().numpy()


CASES = [
    # (N, theta_max, wavelength, fluence, seed)
    (37, 60.0, 45.0, 1e2, 11),
    (64, 30.0, 45.0, 1e4, 12),
    (1, 45.0, 13.5, 1e6, 13),
    (512, 60.0, 45.0, 1e2, 20220203),
    (1024, 80.0, 13.5, 3.0, 20220206),
]


@pytest.mark.parametrize("case", CASES, ids=[f"n{c[0]}" for c in CASES])
def test_ideal_matches_oracle(env, case):
    n, theta, wl, fluence, seed = case
    I = _intensity(n, seed)
    print(f"[gpu] ideal detector N={n} theta={theta} fluence={fluence:g}", flush=True)
    counts, mu = _detect(env, n, theta, wl, I, fluence, seed)
    omu, ocounts = oracle.detect_ideal(wl, theta, n, I.astype(np.float64), fluence, seed)
    assert np.allclose(mu, omu, rtol=3e-7, atol=0)
    small = int((omu < 10).sum())
    print(f"  {n * n} px: {small} by inversion, {n * n - small} by rejection; "
          f"max mean {omu.max():.3g}; counts identical: {np.array_equal(counts, ocounts)}")
    assert np.array_equal(counts, ocounts.astype(np.float32).astype(np.float64))


def test_ideal_edge_values_and_seeds(env):
    torch, msft = env
    n = 16
    I = _intensity(n, 21, lo=0.0, hi=14.0)
    I[:4] = [0.0, -3.0, np.nan, np.inf]
    c1, _ = _detect(env, n, 60.0, 45.0, I, 1e2, 5)
    c2, _ = _detect(env, n, 60.0, 45.0, I, 1e2, 5)
    c3, _ = _detect(env, n, 60.0, 45.0, I, 1e2, 6)
    assert np.array_equal(c1, c2) and not np.array_equal(c1, c3)
    assert np.all(c1[:4] == 0.0)
    _, oc = oracle.detect_ideal(45.0, 60.0, n, I.astype(np.float64), 1e2, 5)
    assert np.array_equal(c1, oc)
    # no fluence, no photons
    c0, mu0 = _detect(env, n, 60.0, 45.0, I, 0.0, 5)
    assert np.all(c0 == 0.0) and np.all(mu0[4:] == 0.0)


def test_ideal_argument_errors(env):
    torch, msft = env
    I = torch.ones(8 * 8, device="cuda")
    with msft.Plan(45.0, 60.0, 8, (4, 4, 4), (2.0, 2.0, 2.0), "fp32", "msft",
                   detector="uniform_q") as plan:
        with pytest.raises(msft.MSFTError):
            plan.detect_ideal(I, 1.0, 0)
    q = oracle.qmap(45.0, 60.0, 8)
    with msft.Plan(45.0, 60.0, 0, (4, 4, 4), (2.0, 2.0, 2.0), "fp32", "msft", q=q) as plan:
        with pytest.raises(msft.MSFTError):
            plan.detect_ideal(I, 1.0, 0)
    with msft.Plan(45.0, 60.0, 8, (4, 4, 4), (2.0, 2.0, 2.0), "fp32", "msft") as plan:
        for bad in (-1.0, math.inf, math.nan):
            with pytest.raises(msft.MSFTError):
                plan.detect_ideal(I, bad, 0)
