"""Differentiable even-odd staggered solve.

x = A^-1 b with A = m^2 - D_eo D_oe. The backward pass solves the adjoint system A lambda = dl/dx with
the same solver (A is Hermitian), then forms the link gradient dl/dU, the mass gradient
dl/dm = -2 m Re<lambda, x> and dl/db = lambda in the library's kernels. Complex gradients follow the
PyTorch convention (dl/dRe + i dl/dIm).
"""
from __future__ import annotations

import torch

from .api import Gauge, Lattice, cg_force, cg_solve


class StaggeredSolve(torch.autograd.Function):
    @staticmethod
    def forward(ctx, links, mass, b, lattice: Lattice, opts: dict):
        opts = dict(opts or {})
        inner = opts.get("inner", "f32")
        recon = opts.get("recon", 18)
        gauge = Gauge(lattice, links.detach().contiguous(), lo_prec=inner, recon=recon)
        m = float(mass)
        kw = dict(tol=opts.get("tol", 1e-10), inner=inner, max_iter=opts.get("max_iter", 100000))
        x, st = cg_solve(gauge, m, b.detach().contiguous(), raise_on_not_converged=True, **kw)
        ctx.gauge = gauge
        ctx.kw = kw
        ctx.m = m
        ctx.mass_is_tensor = isinstance(mass, torch.Tensor)
        ctx.save_for_backward(x)
        ctx.stats = st
        return x

    @staticmethod
    def backward(ctx, gx):
        (x,) = ctx.saved_tensors
        lam, _ = cg_solve(ctx.gauge, ctx.m, gx.contiguous(), raise_on_not_converged=True, **ctx.kw)
        gamma, _, dmass = cg_force(ctx.gauge, ctx.m, x, lam, want_force=False)
        gm = dmass if ctx.mass_is_tensor else None
        return gamma, gm, lam, None, None


def staggered_solve(links: torch.Tensor, mass, b: torch.Tensor, lattice: Lattice, **opts) -> torch.Tensor:
    """Differentiable x = (m^2 - D_eo D_oe)^-1 b (links [4][V][3][3], b [V/2][3], complex128 on the GPU)."""
    return StaggeredSolve.apply(links, mass, b, lattice, opts)
