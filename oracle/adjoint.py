"""Gradients of a linear loss of the Helmholtz solution (oracle).

TEST INFRASTRUCTURE ONLY (see the package header).

Not in the paper. For x = H^-1 b and L = g . x, with H symmetric:
  dL/db = lambda, where H lambda = g (the adjoint solve is the same solve),
  dL/dc = -lambda^T (dH/dc) x for every coefficient c of H.
In flux form a face coupling K between unknowns i and j enters H as
K (e_i - e_j)(e_i - e_j)^T, so dL/dK = -(lambda_i - lambda_j)(x_i - x_j), and
dL/d delta = -lambda * x. With a batch of right-hand sides sharing one
operator the coefficient gradients are summed over the batch.
"""
from __future__ import annotations

import numpy as np

from .mesh import E, N_


def face_gradients(level, lam, x):
    """Return ``(g_kh[2][nz][ncol], g_kv[nz-1][ncol], g_delta[nz][ncol])``.

    ``lam`` and ``x`` are ``[batch][nz][ncol]`` (or ``[nz][ncol]``).
    """
    lam = lam.reshape((-1,) + lam.shape[-2:])
    x = x.reshape((-1,) + x.shape[-2:])
    g_kh = np.stack([
        -((lam - lam[..., level.nbr[d]]) * (x - x[..., level.nbr[d]])).sum(axis=0)
        for d in (E, N_)])
    g_kv = -((lam[:, :-1] - lam[:, 1:]) * (x[:, :-1] - x[:, 1:])).sum(axis=0)
    g_delta = -(lam * x).sum(axis=0)
    return g_kh, g_kv, g_delta


def kv2_gradient(lam, x):
    """``g_kv2[nz-2][ncol]``: gradient of L with respect to the next-to-nearest
    vertical couplings of the 9-cell stencil (faces k | k+2), summed over the
    batch, by the same flux-form rule."""
    lam = lam.reshape((-1,) + lam.shape[-2:])
    x = x.reshape((-1,) + x.shape[-2:])
    return -((lam[:, :-2] - lam[:, 2:]) * (x[:, :-2] - x[:, 2:])).sum(axis=0)


def weighted_gradients(level, kh, kv, s, lam, x):
    """Gradients for the row-weighted operator H = delta + S L (S = diag(s)),
    with lam = H^-T g: since dH/dK = S a a^T for a face vector a = e_i - e_j,
      dL/dK = -(s_i lam_i - s_j lam_j)(x_i - x_j),
      dL/ds = -lam * (L x),   dL/d delta = -lam * x.
    Returns ``(g_kh, g_kv, g_delta, g_s)``, summed over the batch."""
    from .helmholtz import laplacian
    lam = lam.reshape((-1,) + lam.shape[-2:])
    x = x.reshape((-1,) + x.shape[-2:])
    sl = s * lam
    g_kh = np.stack([
        -((sl - sl[..., level.nbr[d]]) * (x - x[..., level.nbr[d]])).sum(axis=0)
        for d in (E, N_)])
    g_kv = -((sl[:, :-1] - sl[:, 1:]) * (x[:, :-1] - x[:, 1:])).sum(axis=0)
    g_delta = -(lam * x).sum(axis=0)
    g_s = -(lam * laplacian(level, kh, kv, x)).sum(axis=0)
    return g_kh, g_kv, g_delta, g_s
