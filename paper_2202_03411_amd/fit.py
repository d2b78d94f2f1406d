"""Differentiable forward model for shape fitting (Sec. 6: forward fitting).

``MSFTFunction`` wraps msft_simulate / msft_backward in torch.autograd: the
forward saves the amplitudes A, the backward hands dL/dI to the library's
adjoint kernels and returns dL/d delta and dL/d beta.  ``SoftStar`` renders a
star-shaped body r(theta, phi) = R0 (1 + sum c_lm Y_lm) (the spherical-harmonic
shapes of Sec. 5.2, real harmonics, theta polar from +z) as a sigmoid-soft voxel
map so torch can carry the gradient on to the coefficients.  Torch only does
the shape rendering and the loss; every step of the scattering model runs in
the library.
"""
from __future__ import annotations

import math

import torch

from . import msft


class MSFTFunction(torch.autograd.Function):
    """I = |A|^2 of (delta, beta) on a plan; differentiable in delta and beta."""

    @staticmethod
    def forward(ctx, delta, beta, plan):
        delta = delta.detach().contiguous()
        beta = beta.detach().contiguous()
        I, A = plan.simulate(delta, beta, amplitude=True)
        ctx.plan = plan
        ctx.save_for_backward(delta, beta, torch.view_as_real(A))
        return I

    @staticmethod
    def backward(ctx, grad_I):
        delta, beta, A = ctx.saved_tensors
        plan = ctx.plan
        gd = torch.empty_like(delta)
        gb = torch.empty_like(beta)
        msft.msft_backward(plan.handle, delta, beta, A, grad_I.detach().float().contiguous(),
                           gd, gb, plan.workspace())
        return gd, gb, None


def simulate(delta, beta, plan):
    return MSFTFunction.apply(delta, beta, plan)


def log_mse_loss(I, target, eps=1e-6):
    """Mean over pixels (and batch) of (log(I + eps) - log(I* + eps))^2."""
    return torch.mean((torch.log(I + eps) - torch.log(target + eps)) ** 2)


def real_sh_torch(lmax, theta, phi):
    """Real orthonormal spherical harmonics, rows ordered l = 0..lmax, m = -l..l."""
    x, s = torch.cos(theta), torch.sin(theta)
    qbar = {(0, 0): torch.full_like(x, 1.0 / math.sqrt(4.0 * math.pi))}
    for m in range(1, lmax + 1):
        qbar[(m, m)] = math.sqrt((2.0 * m + 1.0) / (2.0 * m)) * s * qbar[(m - 1, m - 1)]
    for m in range(0, lmax):
        qbar[(m + 1, m)] = math.sqrt(2.0 * m + 3.0) * x * qbar[(m, m)]
    for m in range(0, lmax + 1):
        for l in range(m + 2, lmax + 1):
            a = math.sqrt((4.0 * l * l - 1.0) / (l * l - m * m))
            b = math.sqrt(((l - 1.0) ** 2 - m * m) / (4.0 * (l - 1.0) ** 2 - 1.0))
            qbar[(l, m)] = a * (x * qbar[(l - 1, m)] - b * qbar[(l - 2, m)])
    rows = []
    for l in range(lmax + 1):
        for m in range(-l, l + 1):
            if m == 0:
                rows.append(qbar[(l, 0)])
            elif m > 0:
                rows.append(math.sqrt(2.0) * qbar[(l, m)] * torch.cos(m * phi))
            else:
                rows.append(math.sqrt(2.0) * qbar[(l, -m)] * torch.sin(-m * phi))
    return torch.stack(rows, dim=0)


class SoftStar:
    """Sigmoid-soft voxelization of R0 (1 + sum c_lm Y_lm) on an n^3 grid of a box."""

    def __init__(self, n, extent, lmax, r0, eps=None, delta0=0.01, beta0=0.02,
                 device="cuda", dtype=torch.float32):
        self.n, self.extent, self.lmax, self.r0 = n, float(extent), lmax, float(r0)
        self.pitch = self.extent / n
        self.eps = float(eps) if eps is not None else self.pitch
        self.delta0, self.beta0 = float(delta0), float(beta0)
        c = (torch.arange(n, dtype=torch.float64, device=device) * 2.0 + 1.0 - n) * self.pitch / 2.0
        X, Y, Z = torch.meshgrid(c, c, c, indexing="ij")
        rr = torch.sqrt(X * X + Y * Y + Z * Z)
        theta = torch.arccos(torch.clamp(Z / torch.where(rr > 0, rr, torch.ones_like(rr)), -1.0, 1.0))
        phi = torch.atan2(Y, X)
        self.radius = rr.to(dtype).reshape(-1)
        self.basis = real_sh_torch(lmax, theta, phi).to(dtype).reshape((lmax + 1) ** 2, -1)
        self.ncoef = (lmax + 1) ** 2

    def occupancy(self, coeffs):
        """coeffs [..., ncoef] -> soft occupancy [..., n, n, n]."""
        r = self.r0 * (1.0 + coeffs.to(self.basis.dtype) @ self.basis)
        o = torch.sigmoid((r - self.radius) / self.eps)
        return o.reshape(*coeffs.shape[:-1], self.n, self.n, self.n)

    def voxelize(self, coeffs):
        o = self.occupancy(coeffs)
        return self.delta0 * o, self.beta0 * o
