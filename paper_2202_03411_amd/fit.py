"""Differentiable forward model for shape fitting (Sec. 6: forward fitting).

``MSFTFunction`` wraps msft_simulate / msft_backward in torch.autograd: the
forward saves the amplitudes A, the backward hands dL/dI to the library's
adjoint kernels and returns dL/d delta and dL/d beta.  ``SoftStar`` renders a
star-shaped body r(theta, phi) = R0 (1 + sum c_lm Y_lm) (the spherical-harmonic
shapes of Sec. 5.2, real harmonics, theta polar from +z) as a sigmoid-soft voxel
map with msft_render_sh, and ``SHRenderFunction`` carries the gradient on to the
coefficients with msft_render_sh_backward.  Torch only holds the tensors and
computes the loss; the rendering, the scattering model and both adjoints run in
the library.
"""
from __future__ import annotations

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


class SHRenderFunction(torch.autograd.Function):
    """(delta, beta) of a SoftStar from its coefficients; differentiable in the coefficients."""

    @staticmethod
    def forward(ctx, coeffs, star):
        coeffs = coeffs.detach().float().contiguous()
        delta = torch.empty(star.shape, dtype=torch.float32, device=coeffs.device)
        beta = torch.empty_like(delta)
        msft.msft_render_sh(star.grid, star.lmax, star.r0, coeffs, delta, beta)
        ctx.star = star
        ctx.save_for_backward(coeffs)
        return delta, beta

    @staticmethod
    def backward(ctx, grad_delta, grad_beta):
        (coeffs,) = ctx.saved_tensors
        star = ctx.star
        gd = torch.zeros(star.shape, device=coeffs.device) if grad_delta is None else grad_delta
        gb = torch.zeros(star.shape, device=coeffs.device) if grad_beta is None else grad_beta
        grad = torch.empty_like(coeffs)
        msft.msft_render_sh_backward(star.grid, star.lmax, star.r0, coeffs,
                                     gd.detach().float().contiguous(), gb.detach().float().contiguous(),
                                     grad, star.workspace())
        return grad, None


class SoftStar:
    """Sigmoid-soft voxelization of R0 (1 + sum c_lm Y_lm) on an n^3 grid of a box centred on
    the origin; edge width eps (default one pitch); coefficients at l*l + l + m."""

    def __init__(self, n, extent, lmax, r0, eps=None, delta0=0.01, beta0=0.02, device="cuda"):
        self.n, self.extent, self.lmax, self.r0 = n, float(extent), lmax, float(r0)
        self.pitch = self.extent / n
        self.eps = float(eps) if eps is not None else self.pitch
        self.delta0, self.beta0 = float(delta0), float(beta0)
        self.device = torch.device(device)
        self.shape = (n, n, n)
        self.ncoef = (lmax + 1) ** 2
        self.grid = msft.make_shape_grid(self.shape, (self.pitch,) * 3, self.eps, self.delta0,
                                         self.beta0)
        self._ws = None

    def workspace(self):
        if self._ws is None:
            self._ws = msft.workspace_tensor(msft.msft_render_sh_query(self.lmax), self.device)
        return self._ws

    def voxelize(self, coeffs):
        """coeffs [ncoef] (device) -> (delta, beta) [n, n, n], differentiable in coeffs."""
        return SHRenderFunction.apply(coeffs, self)
