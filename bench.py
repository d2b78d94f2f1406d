#!/usr/bin/env python3
"""MSFT forward-model benchmark on one MI355X.

Workload: a star-shaped harmonic body (l <= 6, R0 = 200 nm, delta = 0.01,
beta = 0.02) on a 128^3 voxel grid, lambda = 45 nm, flat 512 x 512 detector to
60 deg.  One step = one pattern through the whole forward path: column scan,
MFMA contraction with the fused y/z reduction, |A|^2.  Inputs are resident in
HBM before timing starts.  Prints ONE JSON line.

Reported beside the headline (FP32, one pattern per launch; 100 timed patterns
after 10 warm-ups by default):
  - the BF16 hi+lo split contraction and plain BF16,
  - a batch of patterns in one batched launch against the same patterns
    launched one by one, and the FP32 adjoint,
  - the dominant kernel against the FP32 matrix-core roofline (HIP events on
    the stream the kernel runs on), with its HBM traffic from the committed
    counter summary,
  - the served stream (batched against plain), the uniform-q detector, the shape
    renderers and the Ideal detector,
  - the FP64 CPU oracle timed on a bounded pixel sample (cpu_baseline).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "MSFT patterns/s at 128³ grid, 512² detector (FP32 vs BF16-split vs plain); p99 ms"
PEAK_TFLOPS = {"fp32": 157.3, "bf16x3": 2500.0, "bf16": 2500.0}   # MI355X dense matrix peaks
# real flops the contraction executes on the matrix cores per voxel-pixel term
EXEC_PER_TERM = {"fp32": 6, "bf16x3": 24, "bf16": 8}
HBM_PEAK_GBS = 8000.0


def profiled_traffic(prec):
    """HBM bytes per launch of the contraction kernel from the committed counter
    summary, or None when the kernel source has changed since it was counted."""
    import hashlib
    import re
    kernel = "fwd_g3_kernel_fp32" if prec == "fp32" else f"fwd_pair_kernel_{prec}"
    path = os.path.join(ROOT, "profiles", f"{kernel}_star128_det512_traffic.md")
    if not os.path.exists(path):
        return None
    text = open(path).read()
    m = re.search(r"^fwd[^\n]*traffic per launch[^:]*:\s*([0-9.eE+]+) bytes", text, re.M)
    h = re.search(r"sha256 when counted:\s*([0-9a-f]{64})", text)
    # the FP32 contraction is the three-product kernel of gauss.hip
    src = os.path.join(ROOT, "paper_2202_03411_amd", "csrc",
                       "gauss.hip" if prec == "fp32" else "kernels.hip")
    if not m or not h or hashlib.sha256(open(src, "rb").read()).hexdigest() != h.group(1):
        return None
    return float(m.group(1))


def _pct(xs, p):
    xs = sorted(xs)
    k = min(len(xs) - 1, max(0, int(round(p / 100.0 * (len(xs) - 1)))))
    return xs[k]


def time_single(msft, torch, plan, d, b, steps, warmup):
    """Time `steps` patterns, one msft_simulate_scan + msft_simulate_contract pair each."""
    ws = plan.workspace()
    I = torch.empty(plan.npix, dtype=torch.float32, device="cuda")
    for _ in range(warmup):
        msft.msft_simulate(plan.handle, d, b, I, None, ws)
    torch.cuda.synchronize()
    ev = [[torch.cuda.Event(enable_timing=True) for _ in range(3)] for _ in range(steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(steps):
        ev[k][0].record()
        msft.msft_simulate_scan(plan.handle, d, b, ws)
        ev[k][1].record()
        msft.msft_simulate_contract(plan.handle, ws, I, None)
        ev[k][2].record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    step_ms = [e[0].elapsed_time(e[2]) for e in ev]
    scan_ms = [e[0].elapsed_time(e[1]) for e in ev]
    contract_ms = [e[1].elapsed_time(e[2]) for e in ev]
    return {"wall_s": wall, "step_ms": step_ms, "scan_ms": scan_ms, "contract_ms": contract_ms,
            "intensity": I}


def time_batch(msft, torch, plan, ds, bs, steps, warmup):
    """The same patterns: one persistent launch for all, then one launch each."""
    n = len(ds)
    outs = [torch.empty(plan.npix, dtype=torch.float32, device="cuda") for _ in range(n)]
    reqs = [(plan.handle, ds[k], bs[k], outs[k], None) for k in range(n)]
    wsb = msft.workspace_tensor(msft.msft_batch_query(reqs), "cuda")
    ws = plan.workspace()
    for _ in range(warmup):
        msft.msft_simulate_batch(reqs, wsb)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(steps):
        msft.msft_simulate_batch(reqs, wsb)
    e1.record()
    torch.cuda.synchronize()
    batched_ms = e0.elapsed_time(e1) / steps
    e0.record()
    for _ in range(steps):
        for k in range(n):
            msft.msft_simulate(plan.handle, ds[k], bs[k], outs[k], None, ws)
    e1.record()
    torch.cuda.synchronize()
    plain_ms = e0.elapsed_time(e1) / steps
    return batched_ms, plain_ms


def time_backward(msft, torch, plan, d, b, steps, warmup):
    """Time msft_backward (adjoint of one pattern) with a fixed seeded dL/dI."""
    I, A = plan.simulate(d, b, amplitude=True)
    A = torch.view_as_real(A).contiguous()
    gen = torch.Generator(device="cuda").manual_seed(7)
    g = torch.randn(plan.npix, device="cuda", generator=gen)
    gd, gb = torch.empty_like(d), torch.empty_like(b)
    ws = plan.workspace()
    for _ in range(warmup):
        msft.msft_backward(plan.handle, d, b, A, g, gd, gb, ws)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(steps):
        msft.msft_backward(plan.handle, d, b, A, g, gd, gb, ws)
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / steps


def time_fit(torch, batch, steps, warmup, log, detector="flat"):
    """One iteration of the differentiable fit: `batch` l <= 8 soft-voxelized
    shapes (81 coefficients, edge width one pitch) in a 680 nm box on 128^3,
    512^2 detector to 60 deg at 45 nm; loss = mean squared log-intensity error
    against seeded targets; adjoint through msft_backward and the soft
    voxelization; one Adam step.  Shapes go through the GPU one at a time and
    their gradients accumulate, so the batch never has to be resident at once."""
    import numpy as np

    from paper_2202_03411_amd import fit, inputs, msft
    n, det, box, lmax, r0 = 128, 512, 680.0, 8, 200.0
    star = fit.SoftStar(n, box, lmax, r0)
    plan = msft.Plan(45.0, 60.0, det, (n, n, n), (star.pitch,) * 3, "fp32", "msft",
                     detector=detector)
    rng = np.random.default_rng(inputs.SEED_BASE + 4)
    ncoef = (lmax + 1) ** 2
    tc = rng.normal(0.0, 0.08, size=(batch, ncoef))
    tc[:, 0] = 0.0
    targets = []
    with torch.no_grad():
        for k in range(batch):
            dk, bk = star.voxelize(torch.tensor(tc[k], dtype=torch.float32, device="cuda"))
            targets.append(plan.simulate(dk.contiguous(), bk.contiguous()).clone())
    coeffs = torch.zeros(batch, ncoef, device="cuda", requires_grad=True)
    opt = torch.optim.Adam([coeffs], lr=1e-3)

    def iteration():
        opt.zero_grad()
        for k in range(batch):
            dk, bk = star.voxelize(coeffs[k])
            I = fit.simulate(dk.contiguous(), bk.contiguous(), plan)
            (fit.log_mse_loss(I, targets[k]) / batch).backward()
        opt.step()

    for _ in range(warmup):
        iteration()
    torch.cuda.synchronize()
    times = []
    for it in range(steps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        iteration()
        e1.record()
        torch.cuda.synchronize()
        times.append(e0.elapsed_time(e1) / 1e3)
        log(f"fit iteration {it + 1}/{steps}: {times[-1]:.2f} s")
    plan.close()
    s = sum(times) / len(times)
    P, V = det * det, n ** 3
    return {"batch": batch, "detector": detector, "iterations": steps, "s_per_iteration": s,
            "shapes_per_s": batch / s,
            "tflops_fwd_plus_bwd": 2 * 8.0 * P * V * batch / s / 1e12,
            "flops_basis": "direct sum" if detector == "flat" else "direct-sum equivalent"}


def time_uniform(msft, torch, wl, d, b, prec, steps, warmup):
    """The same body on the uniform transverse-q detector of the slice-transform
    algorithm (separable two-stage contraction), checked on seeded pixels."""
    import numpy as np

    import oracle
    from paper_2202_03411_amd import inputs
    with msft.Plan(wl.wavelength, wl.theta_max_deg, wl.det_n, wl.grid, wl.pitch, prec, "msft",
                   detector="uniform_q") as plan:
        r = time_single(msft, torch, plan, d, b, steps, warmup)
        I = r["intensity"].cpu().numpy().astype(np.float64)
    n, (nx, ny, nz) = wl.det_n, wl.grid
    flops = 8.0 * n * nx * ny * nz + 8.0 * n * n * ny * nz   # stage 1 + stage 2
    ms = sum(r["step_ms"]) / len(r["step_ms"])
    cms = sum(r["contract_ms"]) / len(r["contract_ms"])
    bms = None
    if prec == "fp32":
        with msft.Plan(wl.wavelength, wl.theta_max_deg, wl.det_n, wl.grid, wl.pitch, prec, "msft",
                       detector="uniform_q") as plan:
            bms = time_backward(msft, torch, plan, d, b, max(3, steps), 1)
    pix = inputs.random_pixels(n, 256, seed=83)
    q = oracle.qmap_uniform(wl.wavelength, wl.theta_max_deg, n)[pix]
    ok = ~np.isnan(q[:, 2])
    w = oracle.strength(wl.mode, wl.delta.astype(np.float64), wl.beta.astype(np.float64),
                        wl.pitch, wl.wavelength)
    Io = np.abs(oracle.amplitude(q[ok], w, wl.pitch, 1)) ** 2
    err = float(np.linalg.norm(I[pix][ok] - Io) / np.linalg.norm(Io))
    return {"ms_per_step": ms, "patterns_per_s": 1000.0 / ms,
            "p50_ms": _pct(r["step_ms"], 50), "p99_ms": _pct(r["step_ms"], 99),
            "contract_ms": cms, "separable_flops": flops,
            "contract_tflops": flops / (cms * 1e-3) / 1e12,
            "direct_equivalent_terms_per_s": n * n * nx * ny * nz / (ms * 1e-3),
            "backward_ms": bms,
            "error_vs_fp64_oracle": {"rel_l2_intensity": err, "pixels": int(ok.sum())}}


def time_peaks(msft, torch):
    """What this device sustains: pure matrix-core loops (four accumulator chains per
    wave, four waves per workgroup, four workgroups per CU, no memory traffic) in FP32
    and BF16, and the HBM rate of a 1 GiB device copy (bytes read plus written)."""
    cus = torch.cuda.get_device_properties(0).multi_processor_count
    nblocks = 4 * cus
    sink = torch.empty(nblocks * 256, dtype=torch.float32, device="cuda")
    out = {}
    for prec, name, iters in (("fp32", "fp32_mfma_tflops", 20000), ("bf16x3", "bf16_mfma_tflops", 40000)):
        msft.msft_peak_mfma(prec, 100, nblocks, sink)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        fl = sum(msft.msft_peak_mfma(prec, iters, nblocks, sink) for _ in range(3))
        e1.record()
        torch.cuda.synchronize()
        out[name] = fl / (e0.elapsed_time(e1) * 1e-3) / 1e12
    n = 1 << 28
    src = torch.ones(n, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    msft.msft_copy(src, dst)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(5):
        msft.msft_copy(src, dst)
    e1.record()
    torch.cuda.synchronize()
    out["hbm_copy_gbs"] = 2 * 4 * n * 5 / (e0.elapsed_time(e1) * 1e-3) / 1e9
    out["copy_bytes"] = 2 * 4 * n
    del src, dst
    torch.cuda.empty_cache()
    return out


def time_render(msft, torch, steps):
    """The fit's star-body renderer on 128^3 (l <= 8, soft edge of one pitch), its
    coefficient gradient, and a 96^3 volume map resampled onto the same grid."""
    import numpy as np
    n, box, lmax = 128, 680.0, 8
    g = msft.make_shape_grid((n, n, n), (box / n,) * 3, box / n, 0.01, 0.02)
    c = torch.tensor(np.random.default_rng(3).normal(0, 0.08, 81), dtype=torch.float32, device="cuda")
    d = torch.empty((n, n, n), device="cuda")
    b = torch.empty_like(d)
    gc = torch.empty_like(c)
    ws = msft.workspace_tensor(msft.msft_render_sh_query(lmax), "cuda")
    rng = torch.Generator(device="cuda").manual_seed(4)
    vd = torch.rand((96, 96, 96), device="cuda", generator=rng) * 0.03
    vb = torch.rand((96, 96, 96), device="cuda", generator=rng) * 0.03
    out = {}
    for name, call in (("render_ms", lambda: msft.msft_render_sh(g, lmax, 200.0, c, d, b)),
                       ("gradient_ms", lambda: msft.msft_render_sh_backward(g, lmax, 200.0, c, d, b,
                                                                           gc, ws)),
                       ("volume_map_ms", lambda: msft.msft_render_volume(g, vd, vb, (box / 96,) * 3,
                                                                         d, b))):
        call()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(steps):
            call()
        e1.record()
        torch.cuda.synchronize()
        out[name] = e0.elapsed_time(e1) / steps
    out["voxels"] = n ** 3
    out["voxels_per_s"] = n ** 3 / (out["render_ms"] * 1e-3)
    return out


def time_detector(msft, torch, wl, intensity, steps):
    """The Ideal detector (Poisson counts) over the benchmark pattern at the paper's
    example photon density, 100 photons/nm^2."""
    with msft.Plan.for_workload(wl, "fp32") as plan:
        counts = plan.detect_ideal(intensity, 1e2, 1)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for k in range(steps):
            plan.detect_ideal(intensity, 1e2, k)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / steps
    return {"ms": ms, "photons": float(counts.double().sum()), "photon_density_per_nm2": 1e2,
            "pixels": wl.det_n ** 2}


def oracle_error(wl, I_gpu, npix=256):
    """Relative L2 intensity error of a GPU pattern against the FP64 oracle on
    seeded pixels (all of them and the wide-angle ring theta > 3/4 theta_max)."""
    import numpy as np

    import oracle
    from paper_2202_03411_amd import inputs

    pix = inputs.random_pixels(wl.det_n, npix, seed=31)
    Io, _ = oracle.simulate(wl.mode, wl.wavelength, wl.theta_max_deg, wl.det_n,
                            wl.delta.astype(np.float64), wl.beta.astype(np.float64), wl.pitch,
                            pixels=pix)
    Ig = I_gpu.detach().cpu().numpy().astype(np.float64)[pix]
    q = oracle.qmap(wl.wavelength, wl.theta_max_deg, wl.det_n)[pix]
    k0 = 2 * np.pi / wl.wavelength
    ring = np.degrees(np.arccos((q[:, 2] + k0) / k0)) > 0.75 * wl.theta_max_deg

    def rel(a, b):
        return float(np.linalg.norm(a - b) / np.linalg.norm(b))

    return {"pixels": int(npix), "rel_l2": rel(Ig, Io), "rel_l2_ring": rel(Ig[ring], Io[ring]),
            "max_pixel_rel": float(np.max(np.abs(Ig - Io) / Io))}


def cpu_baseline(wl, target_s):
    """Time the FP64 oracle on a seeded pixel sample of the same pattern."""
    import numpy as np

    import oracle
    from paper_2202_03411_amd import inputs

    q = oracle.qmap(wl.wavelength, wl.theta_max_deg, wl.det_n)
    P = q.shape[0]
    t = time.perf_counter()
    w = oracle.strength(wl.mode, wl.delta.astype(np.float64), wl.beta.astype(np.float64), wl.pitch,
                        wl.wavelength)
    t_strength = time.perf_counter() - t
    cal = inputs.random_pixels(wl.det_n, 512, seed=5)
    t = time.perf_counter()
    oracle.amplitude(q[cal], w, wl.pitch, 1)
    per_px = (time.perf_counter() - t) / cal.size
    n = int(min(P, max(512, target_s / max(per_px, 1e-9))))
    pix = inputs.random_pixels(wl.det_n, n, seed=6)
    t = time.perf_counter()
    oracle.amplitude(q[pix], w, wl.pitch, 1)
    dt = time.perf_counter() - t
    sec_per_pattern = t_strength + dt * P / n
    return {"value": 1.0 / sec_per_pattern, "unit": "patterns/s", "cores": oracle.threads(),
            "kind": "oracle",
            "sample": f"{n} of {P} seeded pixels of the same pattern (separable FP64 sum, "
                      f"{dt:.1f} s) plus the full column scan, scaled to one whole pattern"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100,
                    help="timed patterns; the paper averages 100 repetitions")
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--batch", type=int, default=8, help="patterns per persistent batch launch")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--only", choices=["fp32", "bf16x3", "bf16", "uniform_fp32", "uniform_bf16x3",
                                       "backward_fp32"],
                    default=None,
                    help="time one precision only (profiling runs)")
    ap.add_argument("--serving", type=int, default=64,
                    help="requests of the mixed-size serving stream (0 = skip)")
    ap.add_argument("--no-large", dest="large", action="store_false",
                    help="skip the 256^3 / 1024^2 pattern (l <= 10 body with voids, 80 deg)")
    ap.add_argument("--fit", type=int, default=256, metavar="B",
                    help="time iterations of the differentiable fit with batch B on the flat and "
                         "the uniform-q detector (0 = skip; the flat batch of 256 takes about 35 s)")
    ap.add_argument("--fit-steps", type=int, default=1)
    ap.add_argument("--fit-detector", choices=["flat", "uniform_q", "both"], default="both")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="first run one 256 MiB device-to-device copy, the reference for "
                         "scaling hardware byte counters")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported "
              "(the forward model shards by pattern, so N GPUs would run N independent copies)",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2202_03411_amd import inputs, msft

    if args.calibrate_copy:
        src = torch.ones(64 * 1024 * 1024, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    wl = inputs.pattern_workload()
    P = wl.det_n ** 2
    V = int(np.prod(wl.grid))
    flops = 8.0 * P * V     # one complex multiply-add per voxel-pixel term
    d = torch.from_numpy(wl.delta).cuda()
    b = torch.from_numpy(wl.beta).cuda()
    print(f"[bench] workload {wl.name} grid {wl.grid} det {wl.det_n}^2, {P * V:.3e} terms/pattern",
          file=sys.stderr, flush=True)

    if args.only and args.only.startswith("uniform_"):
        prec = args.only.split("_", 1)[1]
        u = time_uniform(msft, torch, wl, d, b, prec, args.steps, args.warmup)
        print(f"[bench] uniform-q {prec}: {u['ms_per_step']:.3f} ms/pattern, "
              f"{u['contract_tflops']:.1f} TFLOP/s, backward {u['backward_ms']} ms",
              file=sys.stderr, flush=True)
        print(json.dumps({"metric": "MSFT patterns/s, uniform-q detector, 128³ grid, 512²",
                          "value": u["patterns_per_s"], "unit": "patterns/s", "n_gpus": 1,
                          "steps": args.steps, "warmup": args.warmup, "dtype": "f32",
                          "higher_is_better": True, "uniform_q": {prec: u}}))
        return

    if args.only == "backward_fp32":
        with msft.Plan.for_workload(wl, "fp32") as plan:
            ms = time_backward(msft, torch, plan, d, b, args.steps, args.warmup)
        print(f"[bench] fp32 backward: {ms:.3f} ms/pattern, {flops / (ms * 1e-3) / 1e12:.1f} TFLOP/s "
              "algorithmic", file=sys.stderr, flush=True)
        print(json.dumps({"metric": "MSFT adjoint patterns/s, 128³ grid, 512² detector",
                          "value": 1000.0 / ms, "unit": "patterns/s", "n_gpus": 1, "steps": args.steps,
                          "warmup": args.warmup, "dtype": "f32", "higher_is_better": True,
                          "ms_per_step": ms, "tflops_algorithmic": flops / (ms * 1e-3) / 1e12}))
        return

    results = {}
    precisions = [args.only] if args.only else ["fp32", "bf16x3", "bf16"]
    for prec in precisions:
        with msft.Plan.for_workload(wl, prec) as plan:
            r = time_single(msft, torch, plan, d, b, args.steps, args.warmup)
            ms = sum(r["step_ms"]) / len(r["step_ms"])
            cms = sum(r["contract_ms"]) / len(r["contract_ms"])
            sms = sum(r["scan_ms"]) / len(r["scan_ms"])
            res = {"ms_per_step": ms, "patterns_per_s": 1000.0 / ms,
                   "p50_ms": _pct(r["step_ms"], 50), "p99_ms": _pct(r["step_ms"], 99),
                   "contract_ms": cms, "scan_ms": sms, "wall_s": r["wall_s"],
                   "terms_per_s": P * V / (ms * 1e-3),
                   "contract_tflops": flops / (cms * 1e-3) / 1e12,
                   "resident_bytes": plan.resident_bytes, "workspace_bytes": plan.workspace_bytes,
                   "error_vs_fp64_oracle": oracle_error(wl, r["intensity"]),
                   "intensity": r["intensity"]}
            print(f"[bench] {prec}: {ms:.3f} ms/pattern (contract {cms:.3f} ms, scan {sms:.4f} ms), "
                  f"{res['contract_tflops']:.1f} TFLOP/s algorithmic", file=sys.stderr, flush=True)
            if prec == "fp32" and not args.only:
                bms_adj = time_backward(msft, torch, plan, d, b, max(3, args.steps // 4), 1)
                res["backward"] = {"ms_per_pattern": bms_adj,
                                   "tflops_algorithmic": flops / (bms_adj * 1e-3) / 1e12,
                                   "tflops_executed": 0.75 * flops / (bms_adj * 1e-3) / 1e12,
                                   "frac_fp32_mfma_peak": 0.75 * flops / (bms_adj * 1e-3) / 1e12 /
                                   PEAK_TFLOPS["fp32"]}
                print(f"[bench] fp32 backward: {bms_adj:.3f} ms/pattern, "
                      f"{res['backward']['tflops_algorithmic']:.1f} TFLOP/s algorithmic",
                      file=sys.stderr, flush=True)
            if args.batch > 1 and not args.only:
                ds = [torch.roll(d, shifts=k, dims=0) for k in range(args.batch)]
                bs = [torch.roll(b, shifts=k, dims=0) for k in range(args.batch)]
                bms, pms = time_batch(msft, torch, plan, ds, bs, max(2, args.steps // args.batch),
                                      1)
                res["batched"] = {"patterns": args.batch, "ms_per_batch": bms,
                                  "patterns_per_s": args.batch * 1000.0 / bms,
                                  "plain_ms_per_batch": pms,
                                  "plain_patterns_per_s": args.batch * 1000.0 / pms}
                print(f"[bench] {prec}: batch of {args.batch}: {bms:.2f} ms vs {pms:.2f} ms plain",
                      file=sys.stderr, flush=True)
            results[prec] = res

    head = results.get("fp32") or results[precisions[0]]
    head_prec = "fp32" if "fp32" in results else precisions[0]
    # scan: delta and beta in (8 B per voxel), w out in the tile layout (8 B per voxel:
    # FP32 re/im, or BF16 hi/lo re/im)
    scan_bytes = 16.0 * V
    line = {
        "metric": METRIC,
        "value": head["patterns_per_s"],
        "unit": "patterns/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": head["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if head_prec == "fp32" else "bf16x3",
        "data": "synthetic",
        "config": {"workload": wl.name, "grid": list(wl.grid), "detector": [wl.det_n, wl.det_n],
                   "wavelength_nm": wl.wavelength, "theta_max_deg": wl.theta_max_deg,
                   "pitch_nm": wl.pitch[0], "precision": head_prec, "launch": "one pattern per launch"},
        "p50_ms": head["p50_ms"],
        "p99_ms": head["p99_ms"],
        "terms_per_s": head["terms_per_s"],
        # The contraction's roofline is the matrix cores' peak for its dtype against the
        # flops the kernel executes on them: 6 real flops per voxel-pixel term for the
        # FP32 three-product form, 24 for the BF16 hi+lo split (three 8-flop products).
        # The 8-flop count of one complex multiply-add is reported beside it.
        "roofline": {"bound": "mfma", "achieved": head["contract_tflops"] * EXEC_PER_TERM[head_prec] / 8.0,
                     "peak": PEAK_TFLOPS[head_prec], "unit": "TFLOP/s",
                     "frac": head["contract_tflops"] * EXEC_PER_TERM[head_prec] / 8.0
                     / PEAK_TFLOPS[head_prec],
                     "traffic": profiled_traffic(head_prec),
                     "kernel": "fwd_g3_kernel" if head_prec == "fp32" else f"fwd_pair_kernel<{head_prec}>",
                     "per_launch": f"{flops * EXEC_PER_TERM[head_prec] / 8.0:.4e} executed flops "
                                   f"({EXEC_PER_TERM[head_prec]} per voxel-pixel term, {P * V:.4e} terms)",
                     "achieved_algorithmic": head["contract_tflops"],
                     "algorithmic_flops_per_term": 8},
        "scan": {"ms": head["scan_ms"], "gbs": scan_bytes / (head["scan_ms"] * 1e-3) / 1e9,
                 "frac_hbm": scan_bytes / (head["scan_ms"] * 1e-3) / 1e9 / HBM_PEAK_GBS},
        "variants": results,
    }
    if not args.only and head.get("intensity") is not None:
        line["ideal_detector"] = time_detector(msft, torch, wl, head["intensity"], args.steps)
        print(f"[bench] ideal detector 512^2: {line['ideal_detector']['ms'] * 1e3:.1f} us, "
              f"{line['ideal_detector']['photons']:.4g} photons", file=sys.stderr, flush=True)
    for v in line["variants"].values():
        v.pop("intensity", None)
    for prec, r in results.items():
        r["roofline_frac_executed"] = (r["contract_tflops"] * EXEC_PER_TERM[prec] / 8.0
                                       / PEAK_TFLOPS[prec])
        r["executed_flops_per_term"] = EXEC_PER_TERM[prec]
    if args.large and not args.only:
        lw = inputs.large_workload()
        lP, lV = lw.det_n ** 2, int(np.prod(lw.grid))
        ld, lb = torch.from_numpy(lw.delta).cuda(), torch.from_numpy(lw.beta).cuda()
        line["large"] = {"workload": lw.name, "grid": list(lw.grid), "detector": [lw.det_n] * 2,
                         "terms": lP * lV}
        for prec in ("fp32", "bf16x3"):
            with msft.Plan.for_workload(lw, prec) as plan:
                r = time_single(msft, torch, plan, ld, lb, 3, 1)
            ms = sum(r["step_ms"]) / len(r["step_ms"])
            cms = sum(r["contract_ms"]) / len(r["contract_ms"])
            line["large"][prec] = {"ms_per_pattern": ms, "patterns_per_s": 1000.0 / ms,
                                   "contract_tflops": 8.0 * lP * lV / (cms * 1e-3) / 1e12}
            print(f"[bench] large {prec}: {ms:.1f} ms/pattern, "
                  f"{line['large'][prec]['contract_tflops']:.1f} TFLOP/s algorithmic",
                  file=sys.stderr, flush=True)
        del ld, lb
    if args.serving > 0 and not args.only:
        from paper_2202_03411_amd import serving
        line["serving"] = serving.benchmark(
            args.serving, "fp32", loads=(0.8,),
            log=lambda m: print(f"[bench] serving {m}", file=sys.stderr, flush=True))
        line["serving"]["subset"] = (f"the first {args.serving} requests of the seeded serving "
                                     "stream (the full stream is 4096 requests)")
    if not args.only:
        line["uniform_q"] = {}
        for prec in ("fp32", "bf16x3"):
            u = time_uniform(msft, torch, wl, d, b, prec, args.steps, args.warmup)
            line["uniform_q"][prec] = u
            print(f"[bench] uniform-q {prec}: {u['ms_per_step']:.3f} ms/pattern, "
                  f"{u['contract_tflops']:.1f} TFLOP/s (two stages), error "
                  f"{u['error_vs_fp64_oracle']['rel_l2_intensity']:.2e}", file=sys.stderr, flush=True)
    if not args.only:
        line["render"] = time_render(msft, torch, args.steps)
        print(f"[bench] render l<=8 soft star 128^3: {line['render']['render_ms'] * 1e3:.1f} us, "
              f"gradient {line['render']['gradient_ms'] * 1e3:.1f} us", file=sys.stderr, flush=True)
    if not args.only:
        pk = time_peaks(msft, torch)
        # the headline kernels against what the device sustains (roofline.peak stays the
        # published figure)
        pk["fwd_g3_frac_of_sustained"] = line["roofline"]["achieved"] / pk["fp32_mfma_tflops"]
        v3 = line["variants"].get("bf16x3")
        if v3:
            pk["fwd_pair_bf16x3_frac_of_sustained"] = 3.0 * v3["contract_tflops"] / pk["bf16_mfma_tflops"]
        line["peaks"] = pk
        print(f"[bench] sustained: FP32 MFMA {pk['fp32_mfma_tflops']:.1f} TF/s, BF16 MFMA "
              f"{pk['bf16_mfma_tflops']:.1f} TF/s, HBM copy {pk['hbm_copy_gbs']:.0f} GB/s",
              file=sys.stderr, flush=True)
    if args.fit > 0 and not args.only:
        dets = ["flat", "uniform_q"] if args.fit_detector == "both" else [args.fit_detector]
        line["fit"] = {}
        for det in dets:
            line["fit"][det] = time_fit(torch, args.fit, args.fit_steps, 1 if args.fit_steps else 0,
                                        lambda m: print(f"[bench] {m}", file=sys.stderr, flush=True), det)
    if not args.no_cpu_baseline and not args.only:
        line["cpu_baseline"] = cpu_baseline(wl, args.cpu_seconds)
    print(json.dumps(line))


if __name__ == "__main__":
    main()
