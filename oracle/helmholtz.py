"""The synthetic Helmholtz operator on one level, and its coarse versions (oracle).

TEST INFRASTRUCTURE ONLY (see the package header).

The paper's pressure operator H (Eq. helmholtz_operator, Section 3.4) couples
each cell to its horizontal neighbours and to the cells above and below
(Section 3.5). Its FE form needs the LFRic model, so a synthetic operator with
the same structure stands in: a zero-order term delta (the role of H_0 =
M_3^{Pi*}), one coupling per horizontal face (the role of D_2^h) and one per
vertical face (the role of D_1^z + D_2^z), in flux form

  (H x)[k,c] = delta[k,c] x[k,c]
             + sum_{d in E,W,N,S} K_h(face d of c, k) (x[k,c] - x[k,nbr_d(c)])
             + K_v[k,c]   (x[k,c] - x[k+1,c])   if k < nz-1
             + K_v[k-1,c] (x[k,c] - x[k-1,c])   if k > 0.

With positive couplings and delta > 0 this is symmetric positive definite
(a graph Laplacian plus a positive diagonal).

Section 3.5 notes that the paper's H also couples each cell to the cells two
levels above and below (a 9-cell stencil, H_z pentadiagonal). With the
optional next-to-nearest coupling K_v2[k,c] between levels k and k+2 the
operator gains

             + K_v2[k,c]   (x[k,c] - x[k+2,c])   if k < nz-2
             + K_v2[k-2,c] (x[k,c] - x[k-2,c])   if k > 1,

and the smoother's matrix drops those off-diagonal entries (Section 3.6).

The paper's H is not symmetric (Section 5.1): its horizontal part behaves
like -(1/rho*) div(rho* theta* grad) (Eq. continuum_pressure_operator), a
symmetric face-weighted Laplacian scaled per row by a cell weight. With the
optional row weight s[k,c] (the role of 1/rho*) the operator becomes

  H x = delta x + s * (L x),    L x = the flux terms above,

so the coupling across a face differs on its two sides. Its transpose is
H^T x = delta x + L (s * x).

Coarse levels are built by re-discretisation, not by the Galerkin product
(Section 3.6). Eq. DH_ratios gives how each part scales with the grid: H_0 with
the cell volume (so the four children's delta add up), the vertical part with
dx^2 / dz (so the four children's K_v add up), and D_2^h with dz only, not with
dx (so a coarse horizontal face keeps the average of the two fine faces that
make it up). Then D_2^h : H_0 drops by 4 per level, as the paper states.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from .mesh import E, W, N_, S


def face_coeffs(kh: np.ndarray, ftab: np.ndarray) -> np.ndarray:
    """Coupling across each of the 4 faces of each column: ``K[d][k][c]``."""
    nz, ncol = kh.shape[1], kh.shape[2]
    flat = np.concatenate([kh[0], kh[1]], axis=1)           # [nz][2*ncol]
    return np.stack([flat[:, ftab[d]] for d in range(4)])   # [4][nz][ncol]


def laplacian(level, kh, kv, x, kv2=None, y=None):
    """The flux terms of H (everything but delta x), in flux form, added to
    ``y`` when given (in the order: horizontal faces, vertical, k+-2)."""
    K = face_coeffs(kh, level.ftab)
    if y is None:
        y = np.zeros(np.broadcast_shapes(x.shape, K.shape[1:]), dtype=np.result_type(x, kh))
    for d in range(4):
        y = y + K[d] * (x - x[..., :, level.nbr[d]])
    if x.shape[-2] > 1:
        dz = x[..., :-1, :] - x[..., 1:, :]
        flux = kv * dz
        y[..., :-1, :] += flux
        y[..., 1:, :] -= flux
    if kv2 is not None and x.shape[-2] > 2:
        flux2 = kv2 * (x[..., :-2, :] - x[..., 2:, :])
        y[..., :-2, :] += flux2
        y[..., 2:, :] -= flux2
    return y


def apply(level, kh, kv, delta, x, kv2=None, s=None, transpose=False):
    """y = H x on one level, in flux form. ``x`` is ``[..., nz, ncol]``;
    ``kv2`` (``[nz-2][ncol]``) adds the next-to-nearest vertical couplings;
    ``s`` (``[nz][ncol]``) weights the flux terms row by row; ``transpose``
    gives H^T x."""
    if s is None:
        return laplacian(level, kh, kv, x, kv2, y=delta * x)
    if transpose:
        return delta * x + laplacian(level, kh, kv, s * x, kv2)
    return delta * x + s * laplacian(level, kh, kv, x, kv2)


def assemble(level, kh, kv, delta, kv2=None, s=None) -> sp.csr_matrix:
    """Sparse matrix of H, unknown index k*ncol + c (used by the pins)."""
    nz, ncol = delta.shape
    n = nz * ncol
    rows, cols, vals = [], [], []
    idx = np.arange(n).reshape(nz, ncol)
    rows.append(idx.ravel()); cols.append(idx.ravel()); vals.append(delta.ravel())

    def couple(i, j, w):
        rows.extend([i, j, i, j]); cols.extend([i, j, j, i])
        vals.extend([w, w, -w, -w])

    # each horizontal face once, through the faces a column owns (E and N)
    for slot, d in ((0, E), (1, N_)):
        couple(idx.ravel(), idx[:, level.nbr[d]].ravel(), kh[slot].ravel())
    if nz > 1:
        couple(idx[:-1].ravel(), idx[1:].ravel(), kv.ravel())
    if kv2 is not None and nz > 2:
        couple(idx[:-2].ravel(), idx[2:].ravel(), kv2.ravel())
    if s is None:
        A = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                          shape=(n, n))
        return A.tocsr()
    # flux terms weighted row by row; delta (the first n entries) unweighted
    r = np.concatenate(rows)
    v = np.concatenate(vals)
    v[n:] = v[n:] * s.ravel()[r[n:]]
    A = sp.coo_matrix((v, (r, np.concatenate(cols))), shape=(n, n))
    return A.tocsr()


def column_tridiagonal(level, kh, kv, delta, kv2=None, s=None, transpose=False):
    """The smoother's column matrix (Sections 3.5-3.6) as ``(sub, diag, sup)``,
    each ``[nz][ncol]``.

    H_z keeps every coupling inside a column and the whole diagonal of H; the
    horizontal off-diagonal couplings form the rest, H - H_z. The smoother's
    matrix is H_z with the next-to-nearest vertical couplings (k to k+-2)
    dropped: the tridiagonal part of H_z, whose diagonal still holds their
    contribution. For the 7-point operator that is H_z itself. With a row
    weight ``s`` the flux part of every row is scaled by s; ``transpose``
    returns the transposed column matrix (the smoother of H^T).
    ``sub[k]`` couples k to k-1 (zero at k = 0), ``sup[k]`` couples k to k+1.
    """
    nz, ncol = delta.shape
    K = face_coeffs(kh, level.ftab)
    diag = delta + K.sum(axis=0)
    sub = np.zeros((nz, ncol))
    sup = np.zeros((nz, ncol))
    if nz > 1:
        diag[:-1] += kv
        diag[1:] += kv
        sup[:-1] = -kv
        sub[1:] = -kv
    if kv2 is not None and nz > 2:
        diag[:-2] += kv2
        diag[2:] += kv2
    if s is not None:
        diag = delta + s * (diag - delta)
        sub = s * sub
        sup = s * sup
        if transpose:
            sub_t = np.zeros_like(sub)
            sup_t = np.zeros_like(sup)
            sub_t[1:] = sup[:-1]
            sup_t[:-1] = sub[1:]
            sub, sup = sub_t, sup_t
    return sub, diag, sup


def coarsen_kv2(kv2, childs):
    """Next-to-nearest vertical couplings scale like K_v (Eq. DH_ratios: the
    vertical part scales with dx^2): the coarse one is the sum over the four
    children."""
    c00, c10, c01, c11 = childs
    return ((kv2[:, c00] + kv2[:, c10]) + kv2[:, c01]) + kv2[:, c11]


def coarsen_s(s, childs):
    """Coarse row weight: the mean of the four children's (the weight stands for
    1/rho* of the cell, a pointwise field)."""
    c00, c10, c01, c11 = childs
    return 0.25 * (((s[:, c00] + s[:, c10]) + s[:, c01]) + s[:, c11])


def coarsen(kh, kv, delta, childs):
    """Coefficients on the next coarser level by re-discretisation (Section 3.6).

    ``childs[s][C]`` lists the fine children (di, dj) = (0,0), (1,0), (0,1),
    (1,1) of coarse column C. The coarse E face is made of the E faces of the
    children with di = 1, the coarse N face of the N faces of those with dj = 1.
    """
    c00, c10, c01, c11 = childs
    kh_c = np.stack([0.5 * (kh[0][:, c10] + kh[0][:, c11]),
                     0.5 * (kh[1][:, c01] + kh[1][:, c11])])
    kv_c = ((kv[:, c00] + kv[:, c10]) + kv[:, c01]) + kv[:, c11]
    delta_c = ((delta[:, c00] + delta[:, c10]) + delta[:, c01]) + delta[:, c11]
    return kh_c, kv_c, delta_c


class Hierarchy:
    """All multigrid levels of one operator: tables and coefficients per level."""

    def __init__(self, levels, parents, childs, kh, kv, delta, dtype=np.float64, kv2=None,
                 s=None):
        self.levels, self.parents, self.childs = levels, parents, childs
        self.coeffs = [(kh, kv, delta)]
        self.kv2s = [kv2]
        self.ss = [s]
        self.transposed = False
        for l in range(len(levels) - 1):
            self.coeffs.append(coarsen(*self.coeffs[-1], childs[l]))
            self.kv2s.append(None if kv2 is None else coarsen_kv2(self.kv2s[-1], childs[l]))
            self.ss.append(None if s is None else coarsen_s(self.ss[-1], childs[l]))
        self.dtype = np.dtype(dtype)
        if self.dtype != np.float64:
            # coarse coefficients are made in float64 and rounded once
            self.coeffs = [tuple(a.astype(dtype) for a in c) for c in self.coeffs]
            self.kv2s = [None if a is None else a.astype(dtype) for a in self.kv2s]
            self.ss = [None if a is None else a.astype(dtype) for a in self.ss]

    @property
    def nlevels(self):
        return len(self.levels)

    def apply(self, l, x):
        return apply(self.levels[l], *self.coeffs[l], x, kv2=self.kv2s[l], s=self.ss[l],
                     transpose=self.transposed)

    def column_tridiagonal(self, l):
        return column_tridiagonal(self.levels[l], *self.coeffs[l], kv2=self.kv2s[l],
                                  s=self.ss[l], transpose=self.transposed)

    def assemble(self, l):
        A = assemble(self.levels[l], *self.coeffs[l], kv2=self.kv2s[l], s=self.ss[l])
        return A.T.tocsr() if self.transposed else A

    def _copy(self):
        h = Hierarchy.__new__(Hierarchy)
        h.__dict__.update(self.__dict__)
        return h

    def transpose(self):
        """The hierarchy of H^T: every level's operator and smoother matrix
        transposed (the coarse operators of H^T are the transposes of H's)."""
        h = self._copy()
        h.transposed = not self.transposed
        return h

    def astype(self, dtype):
        h = self._copy()
        h.dtype = np.dtype(dtype)
        h.coeffs = [tuple(a.astype(dtype) for a in c) for c in self.coeffs]
        h.kv2s = [None if a is None else a.astype(dtype) for a in self.kv2s]
        h.ss = [None if a is None else a.astype(dtype) for a in self.ss]
        return h
