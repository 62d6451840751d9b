"""Intergrid transfers and the multigrid V-cycle (oracle).

TEST INFRASTRUCTURE ONLY (see the package header).

Section 3.6: the function spaces are nested, so prolongation is the natural
injection (a coarse value is copied into its four children) and restriction is
the map it induces on the dual spaces (the four children's residuals are
added, with no averaging factor). Algorithm 1 then gives the recursive V-cycle:
pre-smooth, restrict the residual, recurse from a zero coarse guess, add the
prolongated correction, post-smooth; on the coarsest level the "coarse solve"
is a few block-Jacobi sweeps rather than a direct or Krylov solve.
"""
from __future__ import annotations

import dataclasses

from .smoother import block_jacobi


@dataclasses.dataclass(frozen=True)
class MGParams:
    """P_H^(MG)(L, omega, n_pre, n_post) of Section 4.1, with n_coarse (Section 5.1)."""

    omega: float = 0.8
    n_pre: int = 2
    n_post: int = 2
    n_coarse: int = 4


def prolongate(xc, parent):
    """Natural injection: fine value = value of the coarse parent column."""
    return xc[..., parent]


def restrict(r, childs):
    """Dual of injection: coarse value = sum of the four fine children."""
    c00, c10, c01, c11 = childs
    return ((r[..., c00] + r[..., c10]) + r[..., c01]) + r[..., c11]


def vcycle(hier, b, params: MGParams = MGParams(), x=None, l: int = 0):
    """One V-cycle on level ``l`` (Algorithm 1); ``x=None`` starts from zero."""
    if l == hier.nlevels - 1:
        return block_jacobi(hier, l, b, None, params.omega, params.n_coarse)
    x = block_jacobi(hier, l, b, x, params.omega, params.n_pre)
    r = b - hier.apply(l, x)
    bc = restrict(r, hier.childs[l])
    xc = vcycle(hier, bc, params, None, l + 1)
    x = x + prolongate(xc, hier.parents[l])
    return block_jacobi(hier, l, b, x, params.omega, params.n_post)
