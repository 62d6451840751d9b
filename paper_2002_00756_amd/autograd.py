"""Differentiable Helmholtz solve x = H(kh, kv, delta[, kv2][, s])^-1 b.

Forward: set the operator's coefficients on the GPU (the coefficient part of
the hierarchy set-up, on an operator reused from an earlier call with the
same shape and options) and run the preconditioned Krylov solve.

Backward, for L = g . x: the adjoint lam = H^-T g is another solve. For the
symmetric operators (7-point and 9-cell) H^T = H, so it is the same solve
with the same V-cycle; for the row-weighted operator H = delta + diag(s) L it
is the solve with H^T and the transposed V-cycle. The coefficient gradients
come from one fused kernel over lam and x (summed over the batch); the
gradient with respect to b is lam itself. A forward or adjoint solve that
stops at maxiter raises instead of returning an inexact result.
"""
from __future__ import annotations

import threading

import torch

from .solver import Operator

# Idle operators by (shape, options, device): a forward takes one (or builds
# one), and gives it back when the autograd node that holds it is freed.
_pool: dict = {}
_pool_lock = threading.Lock()


class _Lease:
    """An operator checked out of the pool; returned when this object dies
    (with the autograd node that needs it for the backward solve)."""

    def __init__(self, key, op):
        self.key, self.op = key, op

    def __del__(self):
        op, self.op = self.op, None
        if op is not None:
            with _pool_lock:
                _pool.setdefault(self.key, []).append(op)


def _lease(key, make):
    with _pool_lock:
        idle = _pool.get(key)
        op = idle.pop() if idle else None
    return _Lease(key, op if op is not None else make())


def clear_operator_pool():
    """Drop every idle pooled operator (their workspaces go back to torch)."""
    with _pool_lock:
        _pool.clear()


class HelmholtzNotConverged(RuntimeError):
    """A solve inside the differentiable solve stopped at maxiter."""


def _check(res, what, rtol, maxiter):
    if not res.converged:
        raise HelmholtzNotConverged(
            f"{what} solve did not reach rtol {rtol:g} in {maxiter} iterations "
            f"(iterations {res.iters}, relative residuals {res.relres})")


class HelmholtzSolve(torch.autograd.Function):
    @staticmethod
    def forward(ctx, b, kh, kv, delta, kv2, s, cfg):
        """``cfg`` holds N, nz, nlevels and optional Operator keywords plus
        rtol / maxiter. ``kv2`` (9-cell stencil) and ``s`` (row-weighted
        operator; needs cg="bicgstab") may be None."""
        cfg = dict(cfg)
        rtol = cfg.pop("rtol", 1e-10)
        maxiter = cfg.pop("maxiter", 500)
        N, nz, nlevels = cfg.pop("N"), cfg.pop("nz"), cfg.pop("nlevels")
        batch = b.shape[0] if b.dim() == 3 else 1
        max_batch = max(batch, cfg.pop("max_batch", 1))
        opts = tuple(sorted(cfg.items()))
        key = (N, nz, nlevels, max_batch, opts, kv2 is not None, s is not None, b.device)
        det = lambda t: t.detach() if t is not None else None  # noqa: E731

        def make():
            return Operator(N, nz, det(kh), det(kv), det(delta), nlevels, max_batch=max_batch,
                            device=b.device, kv2=det(kv2), s=det(s), **cfg)
        lease = _lease(key, make)
        op = lease.op
        if getattr(op, "_fresh", True):
            op._fresh = False          # built with these coefficients just now
        else:
            op.update(det(kh), det(kv), det(delta), kv2=det(kv2), s=det(s))
        res = op.solve(b.detach(), rtol=rtol, maxiter=maxiter)
        _check(res, "forward", rtol, maxiter)
        ctx.lease, ctx.rtol, ctx.maxiter = lease, rtol, maxiter
        ctx.nine, ctx.weighted = kv2 is not None, s is not None
        ctx.save_for_backward(res.x)
        ctx.fwd_iters, ctx.fwd_relres = res.iters, res.relres
        return res.x

    @staticmethod
    def backward(ctx, g):
        (x,) = ctx.saved_tensors
        op = ctx.lease.op
        solve = op.solve_adjoint if ctx.weighted else op.solve
        res = solve(g.contiguous(), rtol=ctx.rtol, maxiter=ctx.maxiter)
        _check(res, "adjoint", ctx.rtol, ctx.maxiter)
        grads = op.face_grad(res.x, x)
        gkh, gkv, gdl = grads[:3]
        gkv2 = grads[3] if ctx.nine else None
        gs = grads[3] if ctx.weighted else None
        return res.x, gkh, gkv, gdl, gkv2, gs, None


def helmholtz_solve(b, kh, kv, delta, kv2=None, s=None, **cfg):
    """x = H^-1 b, differentiable in b, kh, kv, delta and, when given, kv2 (the
    9-cell stencil's couplings two levels apart) or s (the row weight of the
    non-symmetric operator; pass cg="bicgstab")."""
    return HelmholtzSolve.apply(b, kh, kv, delta, kv2, s, cfg)
