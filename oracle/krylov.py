"""Preconditioned conjugate gradients around the V-cycle (oracle).

TEST INFRASTRUCTURE ONLY (see the package header).

Section 4.1 lists CG(A, P, eps) and BiCGStab(A, P, eps) among the Krylov
solvers that take a linear operator A and a preconditioner P; the
preconditioner here is one V-cycle from a zero guess (Section 3.6), or, with
one level, block-Jacobi sweeps (P_H^(Jac)). The synthetic operator is
symmetric positive definite and so is the V-cycle with equal pre- and
post-smoothing, so CG applies; BiCGStab does not need the symmetry.
Convergence is judged on the recursively updated residual,
||r|| <= rtol ||b||, from x = 0.

The float32 form keeps the outer loop in float64 and runs only the
preconditioner in float32 (its input rounded from float64, its coefficients
built in float64 and rounded once); its output is widened back to float64.
"""
from __future__ import annotations

import dataclasses

import numpy as np

from .multigrid import MGParams, vcycle


@dataclasses.dataclass
class CGResult:
    x: np.ndarray
    iters: int
    relres: float
    converged: bool
    history: list


def pcg(apply_A, apply_M, b, rtol=1e-8, maxiter=200, flexible=False,
        callback=None) -> CGResult:
    """Hestenes-Stiefel PCG; ``flexible`` uses the Polak-Ribiere beta.

    ``iters`` counts applications of A inside the loop. ``callback(it, x,
    rel)``, when given, sees every iterate and its relative residual (it
    only observes: the iteration does not depend on it).
    """
    x = np.zeros_like(b)
    bnorm = float(np.linalg.norm(b))
    if bnorm == 0.0:
        return CGResult(x, 0, 0.0, True, [0.0])
    r = b.copy()
    z = apply_M(r)
    p = z.copy()
    rho = float(np.vdot(r, z))
    hist = [1.0]
    it = 0
    while True:
        q = apply_A(p)
        alpha = rho / float(np.vdot(p, q))
        x = x + alpha * p
        r_old = r
        r = r - alpha * q
        it += 1
        rel = float(np.linalg.norm(r)) / bnorm
        hist.append(rel)
        if callback is not None:
            callback(it, x, rel)
        if rel <= rtol:
            return CGResult(x, it, rel, True, hist)
        if it >= maxiter:
            return CGResult(x, it, rel, False, hist)
        z = apply_M(r)
        rho_new = float(np.vdot(r, z))
        if flexible:
            beta = float(np.vdot(z, r - r_old)) / rho
        else:
            beta = rho_new / rho
        p = z + beta * p
        rho = rho_new


def bicgstab(apply_A, apply_M, b, rtol=1e-8, maxiter=200) -> CGResult:
    """Right-preconditioned BiCGStab from x = 0 (van der Vorst's method).

    Section 4.1 lists BiCGStab(A, P, eps) among the solvers; the paper's cost
    model gives each iteration two products with H and two preconditioner
    applications, and four global sums (Section 3.7): here (r0, v), the pair
    (t, s), (t, t), and (r0, r) with ||r|| for the next step and the
    convergence test. The shadow residual r0 is the initial residual b.
    Convergence: ||r|| <= rtol ||b|| on the recursively updated residual.
    A zero (r0, v), or a zero (r0, r) or omega before convergence, is a
    breakdown: the iteration stops there, not converged. ``iters`` counts
    iterations (two products with A each).
    """
    x = np.zeros_like(b)
    bnorm = float(np.linalg.norm(b))
    if bnorm == 0.0:
        return CGResult(x, 0, 0.0, True, [0.0])
    r = b.copy()
    r0 = b.copy()
    rho = float(np.vdot(r0, r))
    p = r.copy()
    v = np.zeros_like(b)
    hist = [1.0]
    it = 0
    while True:
        ph = apply_M(p)
        v = apply_A(ph)
        rv = float(np.vdot(r0, v))
        if rv == 0.0:
            return CGResult(x, it, hist[-1], False, hist)
        alpha = rho / rv
        s = r - alpha * v
        sh = apply_M(s)
        t = apply_A(sh)
        tt = float(np.vdot(t, t))
        omega = float(np.vdot(t, s)) / tt if tt > 0.0 else 0.0
        x = x + alpha * ph + omega * sh
        r = s - omega * t
        it += 1
        rel = float(np.linalg.norm(r)) / bnorm
        hist.append(rel)
        if rel <= rtol:
            return CGResult(x, it, rel, True, hist)
        if it >= maxiter:
            return CGResult(x, it, rel, False, hist)
        rho_new = float(np.vdot(r0, r))
        if rho_new == 0.0 or omega == 0.0:
            return CGResult(x, it, rel, False, hist)
        beta = (rho_new / rho) * (alpha / omega)
        p = r + beta * (p - omega * v)
        rho = rho_new


def mg_preconditioner(hier, params: MGParams = MGParams()):
    """x = M r: one V-cycle from zero on ``hier`` (float64)."""
    return lambda r: vcycle(hier, r, params)


def mg_preconditioner_f32(hier, params: MGParams = MGParams()):
    """Float32 V-cycle used inside the float64 loop (input rounded, output widened).

    A whole float32 V-cycle has no bit-exact target; its parts are pinned
    (coefficients rounded once from the exact values, the float32 column solve
    within its forward-error bound, the one-level closed form), and the tests
    bound its distance to the float64 V-cycle.
    """
    h32 = hier.astype(np.float32)
    return lambda r: vcycle(h32, r.astype(np.float32), params).astype(np.float64)


def solve(hier, b, rtol=1e-8, maxiter=200, params: MGParams = MGParams(),
          precision="fp64", flexible=False, method="cg", callback=None) -> CGResult:
    """MG-preconditioned CG (or BiCGStab, ``method="bicgstab"``) for H x = b on
    the finest level of ``hier``. With one level the preconditioner is
    P_H^(Jac)(omega, n_coarse). ``callback`` is passed to ``pcg``."""
    M = mg_preconditioner_f32(hier, params) if precision == "fp32" else \
        mg_preconditioner(hier, params)
    A = lambda v: hier.apply(0, v)  # noqa: E731
    if method == "bicgstab":
        return bicgstab(A, M, b, rtol, maxiter)
    return pcg(A, M, b, rtol, maxiter, flexible, callback)
