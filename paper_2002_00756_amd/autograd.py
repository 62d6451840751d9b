"""Differentiable Helmholtz solve x = H(kh, kv, delta)^-1 b.

Forward: build the operator hierarchy on the GPU and run the MG-preconditioned
CG. Backward: H is symmetric, so the adjoint lam = H^-1 g is another solve with
the same operator and V-cycle; the coefficient gradients come from one fused
kernel over lam and x (summed over the batch), and the gradient with respect
to b is lam itself.
"""
from __future__ import annotations

import torch

from .solver import Operator


class HelmholtzSolve(torch.autograd.Function):
    @staticmethod
    def forward(ctx, b, kh, kv, delta, cfg):
        """``cfg`` holds N, nz, nlevels and optional Operator keywords plus rtol / maxiter."""
        cfg = dict(cfg)
        rtol = cfg.pop("rtol", 1e-10)
        maxiter = cfg.pop("maxiter", 500)
        N, nz, nlevels = cfg.pop("N"), cfg.pop("nz"), cfg.pop("nlevels")
        batch = b.shape[0] if b.dim() == 3 else 1
        op = Operator(N, nz, kh.detach(), kv.detach(), delta.detach(), nlevels,
                      max_batch=max(batch, cfg.pop("max_batch", 1)), device=b.device, **cfg)
        res = op.solve(b.detach(), rtol=rtol, maxiter=maxiter)
        ctx.op, ctx.rtol, ctx.maxiter = op, rtol, maxiter
        ctx.save_for_backward(res.x)
        ctx.fwd_iters, ctx.fwd_relres = res.iters, res.relres
        return res.x

    @staticmethod
    def backward(ctx, g):
        (x,) = ctx.saved_tensors
        op = ctx.op
        lam = op.solve(g.contiguous(), rtol=ctx.rtol, maxiter=ctx.maxiter).x
        gkh, gkv, gdl = op.face_grad(lam, x)
        return lam, gkh, gkv, gdl, None


def helmholtz_solve(b, kh, kv, delta, **cfg):
    """x = H^-1 b, differentiable in b, kh, kv and delta."""
    return HelmholtzSolve.apply(b, kh, kv, delta, cfg)
