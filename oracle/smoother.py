"""Column tridiagonal solve and block-Jacobi smoothing (oracle).

TEST INFRASTRUCTURE ONLY (see the package header).

Section 3.6: one block-Jacobi step is x <- x + omega * Hz^-1 (b - H x)
(Eq. jacobi), where multiplying by Hz^-1 is an independent tridiagonal solve in
every vertical column, done with the Thomas algorithm. Every column reads the
old iterate of its neighbours, so this is Jacobi, not Gauss-Seidel.
"""
from __future__ import annotations

import numpy as np


def thomas(sub, diag, sup, r):
    """Solve tridiag(sub, diag, sup) z = r in every column; arrays ``[nz][ncol]``.

    Textbook Thomas algorithm: forward elimination, then back substitution.
    ``r`` may carry leading batch dimensions. Runs in the dtype of its inputs.
    """
    nz = diag.shape[0]
    cp = np.empty_like(diag)
    rp = np.empty(r.shape, dtype=np.result_type(r, diag))
    cp[0] = sup[0] / diag[0]
    rp[..., 0, :] = r[..., 0, :] / diag[0]
    for k in range(1, nz):
        den = diag[k] - sub[k] * cp[k - 1]
        cp[k] = sup[k] / den
        rp[..., k, :] = (r[..., k, :] - sub[k] * rp[..., k - 1, :]) / den
    z = np.empty_like(rp)
    z[..., nz - 1, :] = rp[..., nz - 1, :]
    for k in range(nz - 2, -1, -1):
        z[..., k, :] = rp[..., k, :] - cp[k] * z[..., k + 1, :]
    return z


def block_jacobi(hier, l, b, x, omega, nsweeps):
    """``nsweeps`` steps of Eq. jacobi on level ``l``; ``x=None`` means x = 0."""
    sub, diag, sup = hier.column_tridiagonal(l)
    if x is None:
        x = np.zeros(b.shape, dtype=hier.dtype)
    for _ in range(nsweeps):
        r = b - hier.apply(l, x)
        x = x + hier.dtype.type(omega) * thomas(sub, diag, sup, r)
    return x
