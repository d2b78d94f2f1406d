"""GPU parity: the HIP path through the C ABI against the FP64 oracle.

Tolerances are the relative L2 norms of the intensity error, ||I - I_ref|| / ||I_ref||:
1e-5 for the FP32 contraction and 1e-3 for the BF16 hi+lo split, as required
for this model.  Inputs are seeded; the oracle never sees a GPU result.
"""
import numpy as np
import pytest

import oracle
from paper_2202_03411_amd import inputs

pytestmark = pytest.mark.gpu

TOL = {"fp32": 1e-5, "bf16x3": 1e-3}


@pytest.fixture(scope="module")
def msft():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2202_03411_amd import msft as m
    return m


def _rel(a, b):
    a, b = np.ravel(a), np.ravel(b)
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def _random_field(shape, seed, lo=0.0, hi=0.05, sparsity=0.0):
    rng = np.random.default_rng(seed)
    d = rng.uniform(lo, hi, shape).astype(np.float32)
    b = rng.uniform(lo, hi, shape).astype(np.float32)
    if sparsity:
        mask = rng.random(shape) < sparsity
        d[mask] = 0
        b[mask] = 0
    return d, b


def _run(msft, wl, precision, amplitude=True, pixels=None):
    import torch
    print(f"[gpu] {wl.name} grid={wl.grid} det={wl.det_n} mode={wl.mode} {precision}", flush=True)
    with msft.Plan.for_workload(wl, precision) as plan:
        d = torch.from_numpy(wl.delta).cuda()
        b = torch.from_numpy(wl.beta).cuda()
        I, A = plan.simulate(d, b, amplitude=True)
        torch.cuda.synchronize()
        I, A = I.cpu().numpy(), A.cpu().numpy()
    if pixels is not None:
        I, A = I[pixels], A[pixels]
    return I.astype(np.float64), A.astype(np.complex128)


def _oracle(wl, pixels=None):
    I, A = oracle.simulate(wl.mode, wl.wavelength, wl.theta_max_deg, wl.det_n,
                           wl.delta.astype(np.float64), wl.beta.astype(np.float64), wl.pitch,
                           pixels=pixels)
    return I, A


def _workload(name, grid, det, pitch, mode, seed, theta=60.0, wavelength=45.0, sparsity=0.0):
    d, b = _random_field(grid, seed, sparsity=sparsity)
    return inputs.Workload(name, wavelength, theta, det, pitch, mode, d, b)


SMALL = [
    # (name, grid, det, pitch, mode, seed)
    ("ragged_msft", (37, 29, 45), 23, (9.0, 8.0, 7.0), inputs.MODE_MSFT, 1),
    ("xchunks_msft", (150, 5, 33), 20, (3.0, 9.0, 8.0), inputs.MODE_MSFT, 2),
    ("cube_born", (24, 24, 24), 40, (10.0, 10.0, 10.0), inputs.MODE_BORN, 3),
    ("tiny", (1, 1, 1), 1, (10.0, 10.0, 10.0), inputs.MODE_MSFT, 4),
    ("thin_z", (9, 70, 3), 31, (6.0, 5.0, 12.0), inputs.MODE_DENSITY, 5),
]


@pytest.mark.parametrize("precision", ["fp32", "bf16x3"])
@pytest.mark.parametrize("case", SMALL, ids=[c[0] for c in SMALL])
def test_parity_small(msft, case, precision):
    wl = _workload(*case)
    I, A = _run(msft, wl, precision)
    Io, Ao = _oracle(wl)
    err = _rel(I, Io)
    print(f"  rel L2 intensity {err:.3e}  amplitude {_rel(A, Ao):.3e}")
    assert err <= TOL[precision]
    assert _rel(A, Ao) <= TOL[precision]


@pytest.mark.parametrize("precision", ["fp32", "bf16x3"])
def test_parity_sphere_born(msft, precision):
    wl = inputs.sphere_workload(n=32, det_n=64)
    I, _ = _run(msft, wl, precision)
    Io, _ = _oracle(wl)
    err = _rel(I, Io)
    print(f"  sphere rel L2 {err:.3e}")
    assert err <= TOL[precision]


@pytest.mark.parametrize("precision", ["fp32", "bf16x3"])
def test_parity_pattern_sampled(msft, precision):
    # the 128^3 star body on the 512^2 detector, compared on seeded pixels
    wl = inputs.pattern_workload()
    pix = inputs.random_pixels(wl.det_n, 1024, seed=77)
    I, A = _run(msft, wl, precision, pixels=pix)
    Io, Ao = _oracle(wl, pixels=pix)
    err = _rel(I, Io)
    q = oracle.qmap(wl.wavelength, wl.theta_max_deg, wl.det_n)[pix]
    k0 = 2 * np.pi / wl.wavelength
    theta = np.degrees(np.arccos((q[:, 2] + k0) / k0))
    ring = theta > 0.75 * wl.theta_max_deg
    print(f"  rel L2 {err:.3e}  ring {_rel(I[ring], Io[ring]):.3e}  "
          f"max pixel {np.max(np.abs(I - Io) / Io):.3e}")
    assert err <= TOL[precision]
    assert _rel(I[ring], Io[ring]) <= TOL[precision]


# Per-pixel error model: the contraction's rounding leaves an absolute amplitude
# error of a few units in the last place of the brightest amplitude |A|_max (the
# partial sums are of that size), so a pixel's relative intensity error grows as the
# pixel gets darker: |dI| / I <= 2 |dA| / |A| = c sqrt(I_max / I).  Measured on the
# 128^3 body, c reaches 1.8e-7 (FP32) and 1.1e-6 (BF16 split); the bounds below are
# 16 and 128 units of FP32 rounding (2^-24), five to seven times that.  The same
# FP32 bound holds on the fit's 32^3 body, whose darkest pixels (1e-12 of the peak)
# come out within about 4e-3 of the oracle; accumulating the y and z sums in FP64
# instead moved none of those dark-pixel errors (they come from the FP32 operands
# and the matrix cores' FP32 sums over x).
PIXEL_C = {"fp32": 16 * 2.0 ** -24, "bf16x3": 128 * 2.0 ** -24}


def _decades(I, Io):
    """max relative error per decade of I / I_max (I_max: brightest sampled pixel)."""
    imax = Io.max()
    rel = np.abs(I - Io) / Io
    dec = np.floor(-np.log10(Io / imax)).astype(int)
    return {int(k): (int((dec == k).sum()), float(rel[dec == k].max()),
                     float(np.max(rel[dec == k] * np.sqrt(Io[dec == k] / imax))))
            for k in np.unique(dec)}, rel, imax


@pytest.mark.parametrize("precision", ["fp32", "bf16x3"])
def test_pixel_error_by_intensity_decade(msft, precision):
    # the 128^3 star body on the 512^2 detector: 16384 seeded pixels plus the forward
    # pixel, every one within c sqrt(I_max / I) of the FP64 oracle
    wl = inputs.pattern_workload()
    n = wl.det_n
    pix = np.unique(np.concatenate([inputs.random_pixels(n, 16384, seed=91),
                                    [(n // 2) * n + n // 2]]))
    I, _ = _run(msft, wl, precision, pixels=pix)
    Io, _ = _oracle(wl, pixels=pix)
    table, rel, imax = _decades(I, Io)
    for k, (cnt, mx, scaled) in table.items():
        print(f"  I/I_max 1e-{k}: {cnt:5d} px  max rel {mx:.2e}  max rel*sqrt(I/I_max) {scaled:.2e}")
    bound = PIXEL_C[precision] * np.sqrt(imax / Io)
    worst = int(np.argmax(rel / bound))
    assert np.all(rel <= bound), (pix[worst], rel[worst], bound[worst])


def test_pixel_error_floor_of_the_fit_case(msft):
    # the fit's 32^3 soft star on a 48^2 detector in nm, whose pattern spans 13
    # decades: every pixel within the FP32 bound above
    import torch

    from paper_2202_03411_amd import fit
    star = fit.SoftStar(32, 680.0, 4, r0=200.0, device="cuda")
    rng = np.random.default_rng(10)
    c = torch.tensor(rng.normal(0, 0.08, star.ncoef), dtype=torch.float32, device="cuda")
    c[0] = 0.0
    d, b = star.voxelize(c)
    wl = inputs.Workload("fit32", 45.0, 60.0, 48, (star.pitch,) * 3, inputs.MODE_MSFT,
                         d.cpu().numpy(), b.cpu().numpy())
    I, _ = _run(msft, wl, "fp32")
    Io, _ = _oracle(wl)
    table, rel, imax = _decades(I, Io)
    for k, (cnt, mx, scaled) in table.items():
        print(f"  I/I_max 1e-{k}: {cnt:5d} px  max rel {mx:.2e}  max rel*sqrt(I/I_max) {scaled:.2e}")
    assert max(table) >= 12
    assert np.all(rel <= PIXEL_C["fp32"] * np.sqrt(imax / Io))


def test_plain_bf16_is_the_unsplit_reference(msft):
    # single BF16 products: about 1e-3 of the intensity, clearly behind the split form
    wl = inputs.pattern_workload()
    pix = inputs.random_pixels(wl.det_n, 512, seed=79)
    Io, _ = _oracle(wl, pixels=pix)
    e_plain = _rel(_run(msft, wl, "bf16", pixels=pix)[0], Io)
    e_split = _rel(_run(msft, wl, "bf16x3", pixels=pix)[0], Io)
    print(f"  plain bf16 {e_plain:.3e}  split {e_split:.3e}")
    assert e_plain <= 1e-2
    assert e_split < 0.1 * e_plain


def test_qlist_small_angle_is_fft(msft):
    # explicit q list on the Fourier grid with q_z = 0: |A|^2 = |fft2(projection)|^2
    import torch
    nx, ny, nz = 16, 12, 8
    dx, dy, dz = 3.0, 2.0, 4.0
    d, b = _random_field((nx, ny, nz), 11)
    kx, ky = np.meshgrid(np.arange(nx), np.arange(ny), indexing="ij")
    q = np.stack([2 * np.pi * kx / (nx * dx), 2 * np.pi * ky / (ny * dy),
                  np.zeros(kx.shape)], axis=-1).reshape(-1, 3)
    with msft.Plan(45.0, 60.0, 0, (nx, ny, nz), (dx, dy, dz), "fp32", "msft", q=q,
                   allow_alias=True) as plan:
        I = plan.simulate(torch.from_numpy(d).cuda(), torch.from_numpy(b).cuda())
        I = I.cpu().numpy().astype(np.float64)
    w = oracle.strength(oracle.MSFT, d.astype(np.float64), b.astype(np.float64), (dx, dy, dz), 45.0)
    F = np.abs(np.fft.fft2(w.sum(axis=2))) ** 2
    assert _rel(I, F.ravel()) <= 1e-5


@pytest.mark.parametrize("precision", ["fp32", "bf16x3"])
def test_batch_bitwise_equals_single(msft, precision):
    import torch
    print(f"[gpu] batch of 3 plans, {precision}", flush=True)
    wls = [_workload("b0", (37, 29, 45), 23, (9.0, 8.0, 7.0), inputs.MODE_MSFT, 21),
           _workload("b1", (64, 16, 40), 48, (5.0, 5.0, 5.0), inputs.MODE_MSFT, 22),
           _workload("b2", (20, 20, 20), 33, (8.0, 8.0, 8.0), inputs.MODE_BORN, 23)]
    plans = [msft.Plan.for_workload(w, precision) for w in wls]
    try:
        singles, reqs, outs = [], [], []
        for p, w in zip(plans, wls):
            d = torch.from_numpy(w.delta).cuda()
            b = torch.from_numpy(w.beta).cuda()
            I, A = p.simulate(d, b, amplitude=True)
            singles.append((I.clone(), A.clone()))
            Ib = torch.full_like(I, float("nan"))
            Ab = torch.full((p.npix, 2), float("nan"), device="cuda")
            reqs.append((p.handle, d, b, Ib, Ab))
            outs.append((Ib, Ab))
        ws = msft.workspace_tensor(msft.msft_batch_query(reqs), "cuda")
        msft.msft_simulate_batch(reqs, ws)
        torch.cuda.synchronize()
        for (Is, As), (Ib, Ab) in zip(singles, outs):
            assert torch.equal(Is, Ib)
            assert torch.equal(torch.view_as_real(As), Ab)
    finally:
        for p in plans:
            p.close()


def test_batch_tile_ranges(msft):
    import torch
    w = _workload("split", (33, 20, 40), 40, (6.0, 6.0, 6.0), inputs.MODE_MSFT, 31)
    with msft.Plan.for_workload(w, "fp32") as p:
        d = torch.from_numpy(w.delta).cuda()
        b = torch.from_numpy(w.beta).cuda()
        I = p.simulate(d, b)
        nb = -(-p.npix // msft.msft_pixel_block())
        Ib = torch.full_like(I, -1.0)
        cut = nb // 2
        reqs = [(p.handle, d, b, Ib, None, (0, cut)), (p.handle, d, b, Ib, None, (cut, nb))]
        ws = msft.workspace_tensor(msft.msft_batch_query(reqs), "cuda")
        msft.msft_simulate_batch(reqs, ws)
        torch.cuda.synchronize()
        assert torch.equal(I, Ib)


@pytest.mark.parametrize("precision", ["fp32", "bf16x3"])
def test_empty_volume_and_empty_requests(msft, precision):
    # A volume with no material scatters nothing: every strength is exactly zero, so
    # every sum is.  An empty batch and an empty tile range launch nothing and leave
    # their outputs as they were.
    import torch
    print(f"[gpu] empty inputs, {precision}", flush=True)
    w = _workload("zero", (33, 20, 40), 40, (6.0, 6.0, 6.0), inputs.MODE_MSFT, 51)
    with msft.Plan.for_workload(w, precision) as p:
        d = torch.zeros(w.grid, device="cuda")
        b = torch.zeros(w.grid, device="cuda")
        I, A = p.simulate(d, b, amplitude=True)
        torch.cuda.synchronize()
        assert torch.count_nonzero(I).item() == 0 and torch.count_nonzero(A).item() == 0
        ws = msft.workspace_tensor(msft.msft_batch_query([]), "cuda")
        msft.msft_simulate_batch([], ws)
        nb = -(-p.npix // msft.msft_pixel_block())
        Ib = torch.full_like(I, -1.0)
        reqs = [(p.handle, d, b, Ib, None, (nb, nb)), (p.handle, d, b, Ib, None, (0, 0))]
        ws = msft.workspace_tensor(msft.msft_batch_query(reqs), "cuda")
        msft.msft_simulate_batch(reqs, ws)
        torch.cuda.synchronize()
        assert torch.all(Ib == -1.0).item()
        with pytest.raises(msft.MSFTError):
            msft.msft_simulate_batch([(p.handle, d, b, Ib, None, (1, 0))], ws)
        with pytest.raises(msft.MSFTError):
            msft.msft_simulate_batch([(p.handle, d, b, Ib, None, (0, nb + 1))], ws)


def test_repeatable(msft):
    import torch
    w = _workload("rep", (40, 30, 50), 37, (7.0, 7.0, 7.0), inputs.MODE_MSFT, 41)
    with msft.Plan.for_workload(w, "bf16x3") as p:
        d = torch.from_numpy(w.delta).cuda()
        b = torch.from_numpy(w.beta).cuda()
        I1 = p.simulate(d, b).clone()
        I2 = p.simulate(d, b)
        torch.cuda.synchronize()
        assert torch.equal(I1, I2)


@pytest.fixture(scope="module")
def large_wl():
    # l <= 10 harmonic body with three voids, 256^3, 1024^2 detector to 80 deg at 13.5 nm
    return inputs.large_workload()


@pytest.mark.parametrize("precision", ["fp32", "bf16x3"])
def test_parity_large_sampled(msft, large_wl, precision):
    wl = large_wl
    pix = inputs.random_pixels(wl.det_n, 384, seed=78)
    I, A = _run(msft, wl, precision, pixels=pix)
    Io, Ao = _oracle(wl, pixels=pix)
    err = _rel(I, Io)
    print(f"  large pattern rel L2 {err:.3e}  amplitude {_rel(A, Ao):.3e}")
    assert err <= TOL[precision]


@pytest.mark.parametrize("precision", ["fp32", "bf16x3"])
def test_parity_2048_detector_sampled(msft, precision):
    # the paper's largest detector (2048 x 2048, Sec. 6) on the 128^3 star body to
    # 60 deg: 32768 pixel blocks, seeded pixels against the oracle
    wl = inputs.star_workload(n=128, det_n=2048, seed=inputs.SEED_BASE + 11, name="star_2048")
    pix = inputs.random_pixels(wl.det_n, 384, seed=79)
    I, A = _run(msft, wl, precision, pixels=pix)
    Io, Ao = _oracle(wl, pixels=pix)
    err = _rel(I, Io)
    print(f"  2048^2 detector rel L2 {err:.3e}  amplitude {_rel(A, Ao):.3e}")
    assert err <= TOL[precision]
