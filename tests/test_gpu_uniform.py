"""GPU parity of the uniform transverse-q detector (the separable two-stage
contraction) against the FP64 oracle's direct sum over the same q.

Pixels with an outgoing wave are compared as relative L2 of the intensity:
1e-5 (FP32) and 1e-3 (BF16 split), as for the flat detector; pixels beyond the
Ewald sphere's rim must be exactly zero.  The oracle sees only its own q map
(oracle.qmap_uniform) and the seeded voxels.
"""
import numpy as np
import pytest

import oracle
from paper_2202_03411_amd import inputs

pytestmark = pytest.mark.gpu

TOL = {"fp32": 1e-5, "bf16x3": 1e-3}
MODES = {inputs.MODE_MSFT: "msft", inputs.MODE_BORN: "born", inputs.MODE_DENSITY: "density"}


@pytest.fixture(scope="module")
def env():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2202_03411_amd import msft
    return torch, msft


def _rel(a, b):
    a, b = np.ravel(a), np.ravel(b)
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def _field(grid, seed):
    rng = np.random.default_rng(seed)
    return (rng.uniform(0.0, 0.05, grid).astype(np.float32),
            rng.uniform(0.0, 0.05, grid).astype(np.float32))


def _gpu(env, wl, precision, amplitude=True):
    torch, msft = env
    print(f"[gpu] uniform-q {wl.name} grid={wl.grid} det={wl.det_n} {precision}", flush=True)
    with msft.Plan(wl.wavelength, wl.theta_max_deg, wl.det_n, wl.grid, wl.pitch, precision,
                   MODES[wl.mode], detector="uniform_q") as plan:
        d = torch.from_numpy(wl.delta).cuda()
        b = torch.from_numpy(wl.beta).cuda()
        I, A = plan.simulate(d, b, amplitude=True)
        torch.cuda.synchronize()
        return I.cpu().numpy().astype(np.float64), A.cpu().numpy().astype(np.complex128)


def _oracle(wl, pixels=None):
    q = oracle.qmap_uniform(wl.wavelength, wl.theta_max_deg, wl.det_n)
    if pixels is not None:
        q = q[pixels]
    ok = ~np.isnan(q[:, 2])
    w = oracle.strength(wl.mode, wl.delta.astype(np.float64), wl.beta.astype(np.float64),
                        wl.pitch, wl.wavelength)
    A = np.zeros(q.shape[0], np.complex128)
    A[ok] = oracle.amplitude(q[ok], w, wl.pitch, 1)
    return np.abs(A) ** 2, A, ok


SMALL = [
    # (name, grid, det, pitch, mode, seed, theta)
    ("ragged", (37, 29, 45), 23, (9.0, 8.0, 7.0), inputs.MODE_MSFT, 51, 60.0),
    ("chunks", (150, 70, 40), 20, (3.0, 3.0, 3.0), inputs.MODE_MSFT, 52, 60.0),
    ("two_blocks", (24, 24, 24), 150, (10.0, 10.0, 10.0), inputs.MODE_BORN, 53, 30.0),
    ("tiny", (1, 1, 1), 1, (10.0, 10.0, 10.0), inputs.MODE_MSFT, 54, 60.0),
    ("thin_z", (9, 70, 3), 31, (6.0, 5.0, 12.0), inputs.MODE_DENSITY, 55, 80.0),
    # six z blocks: BF16 stage 2 reads the Tz table at blocks 0 and 4 and rotates between
    ("deep_z", (12, 10, 170), 20, (8.0, 8.0, 6.0), inputs.MODE_MSFT, 57, 60.0),
    # more than 128 rows y: FP32 leaves the three-product form for the four-product one
    ("tall_y", (10, 140, 20), 24, (6.0, 5.0, 7.0), inputs.MODE_MSFT, 56, 60.0),
]


@pytest.mark.parametrize("precision", ["fp32", "bf16x3"])
@pytest.mark.parametrize("case", SMALL, ids=[c[0] for c in SMALL])
def test_uniform_parity_small(env, case, precision):
    name, grid, det, pitch, mode, seed, theta = case
    d, b = _field(grid, seed)
    wl = inputs.Workload(name, 45.0, theta, det, pitch, mode, d, b)
    I, A = _gpu(env, wl, precision)
    Io, Ao, ok = _oracle(wl)
    err = _rel(I[ok], Io[ok])
    print(f"  rel L2 intensity {err:.3e}  amplitude {_rel(A[ok], Ao[ok]):.3e}  "
          f"beyond the rim {int((~ok).sum())} px")
    assert err <= TOL[precision]
    assert _rel(A[ok], Ao[ok]) <= TOL[precision]
    assert np.all(I[~ok] == 0.0) and np.all(A[~ok] == 0.0)


def test_uniform_equals_direct_sum_kernel(env):
    # the same q through the flat-detector kernel (an explicit q list): the separable
    # contraction and the direct per-pixel contraction agree to FP32 rounding
    torch, msft = env
    d, b = _field((40, 33, 50), 56)
    wl = inputs.Workload("same_q", 45.0, 60.0, 40, (7.0, 7.0, 7.0), inputs.MODE_MSFT, d, b)
    I, _ = _gpu(env, wl, "fp32")
    q = oracle.qmap_uniform(45.0, 60.0, 40)
    ok = ~np.isnan(q[:, 2])
    with msft.Plan(45.0, 60.0, 0, wl.grid, wl.pitch, "fp32", "msft", q=q[ok]) as plan:
        Iq = plan.simulate(torch.from_numpy(d).cuda(), torch.from_numpy(b).cuda())
        Iq = Iq.cpu().numpy().astype(np.float64)
    err = _rel(I[ok], Iq)
    print(f"  separable vs direct kernel rel L2 {err:.3e}")
    assert err <= 1e-5


@pytest.mark.parametrize("precision", ["fp32", "bf16x3"])
def test_uniform_pattern_sampled(env, precision):
    # the 128^3 star body on a 512^2 uniform-q detector to 60 deg, seeded pixels
    base = inputs.pattern_workload()
    wl = inputs.Workload("star_uniform", base.wavelength, base.theta_max_deg, base.det_n,
                         base.pitch, base.mode, base.delta, base.beta)
    pix = inputs.random_pixels(wl.det_n, 1024, seed=81)
    I, _ = _gpu(env, wl, precision)
    Io, _, ok = _oracle(wl, pixels=pix)
    err = _rel(I[pix][ok], Io[ok])
    print(f"  rel L2 {err:.3e} on {int(ok.sum())} pixels; {int((~ok).sum())} beyond the rim")
    assert err <= TOL[precision]
    assert np.all(I[pix][~ok] == 0.0)


@pytest.mark.parametrize("n", [511, 383, 255])
def test_uniform_column_groups(env, n):
    # Detector sides whose second stage leaves a last, partial group of columns: the
    # BF16 split runs 2, 2 and 1 columns per workgroup (row blocks of 128: 4, 3, 2),
    # the FP32 three-product form 8, 4 and 2 (row blocks of 64: 8, 6, 4; last groups
    # of 7, 3 and 1 columns).  ny = 70 gives full and partial y chunks in both.
    # Seeded pixels plus every row of the last three columns and of column 0.
    d, b = _field((20, 70, 33), 60 + n)
    wl = inputs.Workload(f"cols{n}", 45.0, 60.0, n, (9.0, 7.0, 8.0), inputs.MODE_MSFT, d, b)
    rows = np.arange(n)
    pix = np.concatenate([inputs.random_pixels(n, 400, seed=n)] +
                         [rows * n + i for i in (0, n - 3, n - 2, n - 1)])
    Io, _, ok = _oracle(wl, pixels=pix)
    for precision in ("fp32", "bf16x3"):
        I, _ = _gpu(env, wl, precision)
        err = _rel(I[pix][ok], Io[ok])
        print(f"  N={n} {precision}: rel L2 {err:.3e} on {int(ok.sum())} pixels")
        assert err <= TOL[precision]
        assert np.all(I[pix][~ok] == 0.0)


def test_uniform_repeatable(env):
    d, b = _field((40, 30, 50), 57)
    wl = inputs.Workload("rep", 45.0, 60.0, 37, (7.0, 7.0, 7.0), inputs.MODE_MSFT, d, b)
    I1, _ = _gpu(env, wl, "bf16x3")
    I2, _ = _gpu(env, wl, "bf16x3")
    assert np.array_equal(I1, I2)


@pytest.mark.parametrize("grid,det,pitch", [((30, 26, 35), 24, (9.0, 8.0, 7.0)),
                                             ((22, 30, 18), 37, (7.0, 6.0, 8.0)),
                                             ((10, 140, 20), 37, (6.0, 5.0, 7.0))],
                         ids=["three_product", "three_product_odd_side", "tall_y"])
def test_uniform_backward_matches_oracle(env, grid, det, pitch):
    # the separable adjoint on ragged uniform-q plans (pixels beyond the rim carry
    # A = 0, N not a multiple of the column chunk, an odd N whose last column pair
    # holds one column, two row chunks); more than 128 rows y take FP32 out of the
    # three-product form
    torch, msft = env
    d, b = _field(grid, 58)
    g = np.random.default_rng(59).normal(size=det * det)
    with msft.Plan(45.0, 60.0, det, grid, pitch, "fp32", "msft", detector="uniform_q") as plan:
        dt, bt = torch.from_numpy(d).cuda(), torch.from_numpy(b).cuda()
        _, A = plan.simulate(dt, bt, amplitude=True)
        gd, gb = torch.empty_like(dt), torch.empty_like(bt)
        msft.msft_backward(plan.handle, dt, bt, torch.view_as_real(A).contiguous(),
                           torch.from_numpy(g.astype(np.float32)).cuda(), gd, gb, plan.workspace())
        torch.cuda.synchronize()
        gd, gb = gd.cpu().numpy().astype(np.float64), gb.cpu().numpy().astype(np.float64)
    q = oracle.qmap_uniform(45.0, 60.0, det)
    ok = ~np.isnan(q[:, 2])
    d64, b64 = d.astype(np.float64), b.astype(np.float64)
    w = oracle.strength(oracle.MSFT, d64, b64, pitch, 45.0)
    Ao = oracle.amplitude(q[ok], w, pitch, 1)
    od, ob = oracle.backward(oracle.MSFT, q[ok], g[ok], Ao, d64, b64, pitch, 45.0)
    print(f"  rel L2 d/delta {_rel(gd, od):.3e}  d/beta {_rel(gb, ob):.3e}")
    assert _rel(gd, od) <= 1e-3
    assert _rel(gb, ob) <= 1e-3


def test_uniform_backward_sampled_columns(env):
    # a 64^3 star body on a 128^2 uniform-q detector to 60 deg: the separable adjoint
    # against the oracle's gradient on seeded columns through the object
    torch, msft = env
    wl = inputs.star_workload(n=64, det_n=128, seed=inputs.SEED_BASE + 9)
    g = np.random.default_rng(60).normal(size=wl.det_n ** 2)
    print(f"[gpu] uniform-q backward {wl.grid} det={wl.det_n}", flush=True)
    with msft.Plan(wl.wavelength, wl.theta_max_deg, wl.det_n, wl.grid, wl.pitch, "fp32", "msft",
                   detector="uniform_q") as plan:
        dt, bt = torch.from_numpy(wl.delta).cuda(), torch.from_numpy(wl.beta).cuda()
        _, A = plan.simulate(dt, bt, amplitude=True)
        gd, gb = torch.empty_like(dt), torch.empty_like(bt)
        msft.msft_backward(plan.handle, dt, bt, torch.view_as_real(A).contiguous(),
                           torch.from_numpy(g.astype(np.float32)).cuda(), gd, gb, plan.workspace())
        torch.cuda.synchronize()
        gd, gb = gd.cpu().numpy().astype(np.float64), gb.cpu().numpy().astype(np.float64)
    q = oracle.qmap_uniform(wl.wavelength, wl.theta_max_deg, wl.det_n)
    ok = ~np.isnan(q[:, 2])
    d64, b64 = wl.delta.astype(np.float64), wl.beta.astype(np.float64)
    w = oracle.strength(oracle.MSFT, d64, b64, wl.pitch, wl.wavelength)
    Ao = oracle.amplitude(q[ok], w, wl.pitch, 1)
    nx, ny, nz = wl.grid
    rng = np.random.default_rng(61)
    cols = [int(a * ny + b) for a, b in zip(rng.integers(nx // 4, 3 * nx // 4, 24),
                                             rng.integers(ny // 4, 3 * ny // 4, 24))]
    od, ob = oracle.backward(oracle.MSFT, q[ok], g[ok], Ao, d64, b64, wl.pitch, wl.wavelength,
                             cols=cols)
    sd = gd.reshape(nx * ny, nz)[cols]
    sb = gb.reshape(nx * ny, nz)[cols]
    print(f"  rel L2 d/delta {_rel(sd, od):.3e}  d/beta {_rel(sb, ob):.3e} on {len(cols)} columns")
    assert _rel(sd, od) <= 1e-3
    assert _rel(sb, ob) <= 1e-3
