"""sigma_1 as a differentiable function of (base flow U, nu, omega).

Forward runs Algorithm 1 on the GPU (rr_factor, rr_sketch_solve,
rr_adjoint_solve, rr_gains with the eq. 9 recovery) and returns sigma_1^AV per
shift.  Backward calls rr_grad, the stencil reduction of
    d sigma / dp = sigma^2 Re(v^H (dL/dp) u),   d sigma / d omega = sigma^2 Im(v^H u)
(first-order perturbation of eq. 5 with H v = sigma u), evaluated with the
recovered triplet (sigma_1^AV, u_1^AV, v_1).  The sketch Theta is held fixed.
Values of U on the boundary ring enter L through the central differences
U_x, U_y of their interior neighbours, so they get a gradient too (the
corners, which no difference reads, get zero).
"""
from __future__ import annotations

import numpy as np
import torch

from . import api


class SigmaOne(torch.autograd.Function):
    """sigma_1(U, nu, omega) for every shift.

    U: float64 CUDA tensor of shape (nx+2, ny+2) (ring included); nu: 0-d
    float64 tensor; omega: float64 tensor of shifts (real).  Keyword-only
    arguments fix the grid, sketch and precision.  The sketch weights Phi
    (eq. 10) come from U unless `phi` (a float64 CUDA tensor of nx*ny
    weights) is given: the gradient holds the sketch fixed, so a finite
    difference of sigma_1 that should match it passes the unperturbed
    weights.  Returns (n_omega,) float64.
    """

    @staticmethod
    def forward(ctx, U, nu, omega, nx: int, ny: int, domain, k: int = 12, q: int = 0,
                seed: int = 0, precision: str = "fp64", tile: int = 64, phi=None):
        if not (U.is_cuda and U.dtype == torch.float64 and U.shape == (nx + 2, ny + 2)):
            raise ValueError("U must be a float64 CUDA tensor of shape (nx+2, ny+2)")
        om = omega.detach().cpu().numpy().astype(np.float64).reshape(-1)
        prob = api.BurgersProblem.from_base_flow(U, nx, ny, domain, float(nu), weighted=True)
        if phi is not None:
            if not (phi.is_cuda and phi.dtype == torch.float64 and phi.numel() == nx * ny):
                raise ValueError("phi must be a float64 CUDA tensor of nx*ny weights")
            prob.phi = phi.detach().contiguous().reshape(-1)
        f = api.factor(prob, om, precision, k_max=k, tile=tile)
        Q = f.sketch_solve(k, seed, q)
        Z = f.adjoint_solve(Q)
        out = f.gains(Q, Z, "av")
        f.check()
        s1 = out["sigma_AV"][:, 0].contiguous()
        ctx.save_for_backward(s1)
        ctx.f = f
        ctx.u1 = out["U"]
        ctx.v1 = out["V"]
        ctx.stride = k * prob.n
        ctx.shape = (nx, ny)
        return s1.clone()

    @staticmethod
    def backward(ctx, grad_out):
        (s1,) = ctx.saved_tensors
        f = ctx.f
        dU, dnu, dom = f.grad(s1, ctx.u1, ctx.v1, ctx.stride)
        f.check()
        g = grad_out.to(torch.float64).reshape(-1)
        gU = (g[:, None, None] * dU).sum(0)
        gnu = (g * dnu).sum()
        gom = (g * dom).to(torch.float64)
        f.free()
        return gU, gnu, gom, None, None, None, None, None, None, None, None, None


def sigma_one(U, nu, omega, nx, ny, domain, **kw):
    return SigmaOne.apply(U, nu, omega, nx, ny, domain, kw.get("k", 12), kw.get("q", 0),
                          kw.get("seed", 0), kw.get("precision", "fp64"), kw.get("tile", 64),
                          kw.get("phi"))
