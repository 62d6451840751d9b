"""Pins of the oracle's float32 preconditioner form (the mixed-precision
V-cycle: coefficients built in float64 and rounded once, vectors and
arithmetic in float32), against what does not depend on it:

* the rounding rule, bit for bit: every float32 coefficient of every level
  equals the exact (rational) re-discretised value rounded to nearest by the
  C library's float conversion, and coarsening in float32 instead would give
  other bits;
* the float32 Thomas solve against scipy's banded float64 solver on the same
  rounded matrices, within the textbook forward-error bound of a tridiagonal
  LU solve (a small multiple of the column's Skeel condition number
  cond(A, z) = || |A^-1| |A| |z| || / ||z|| times the float32 unit roundoff
  2^-24);
* the closed form of Section 3.6's smoother without horizontal couplings
  (w_h = 0, one level): n sweeps of Eq. jacobi from zero give exactly
  (1 - (1 - omega)^n) H^-1 b; the float32 V-cycle reaches it within the same
  kind of bound.
"""
import struct
from fractions import Fraction

import numpy as np
import pytest
from scipy.linalg import solve_banded

import workloads
from oracle import helmholtz, mesh, multigrid, smoother
from oracle.multigrid import MGParams

U32 = 2.0 ** -24   # float32 unit roundoff


def _f32(v: Fraction) -> np.float32:
    """Round an exact rational to the nearest float32 (C library conversion)."""
    return np.frombuffer(struct.pack("<f", float(v)), dtype=np.float32)[0] if \
        abs(v) < 2 ** 100 else np.float32(np.inf)


def _exact_hierarchy(kh, kv, delta, childs):
    """Coarse coefficients of every level as exact rationals (Section 3.6:
    coarse face = mean of its two fine faces, coarse kv and delta = sum of the
    four children), computed with Python fractions from the float64 fine ones."""
    F = np.vectorize(Fraction, otypes=[object])
    levels = [(F(kh), F(kv), F(delta))]
    for ch in childs:
        c00, c10, c01, c11 = ch
        kh_f, kv_f, dl_f = levels[-1]
        half = Fraction(1, 2)
        kh_c = np.stack([(kh_f[0][:, c10] + kh_f[0][:, c11]) * half,
                         (kh_f[1][:, c01] + kh_f[1][:, c11]) * half])
        kv_c = kv_f[:, c00] + kv_f[:, c10] + kv_f[:, c01] + kv_f[:, c11]
        dl_c = dl_f[:, c00] + dl_f[:, c10] + dl_f[:, c01] + dl_f[:, c11]
        levels.append((kh_c, kv_c, dl_c))
    return levels


def test_float32_coefficients_are_the_exact_ones_rounded_once():
    N, nz, L = 8, 4, 4
    kh, kv, delta = workloads.coefficients(N, nz, 1.0, 1000.0, True)
    levels, parents, childs = mesh.hierarchy(N, L)
    hier = helmholtz.Hierarchy(levels, parents, childs, kh, kv, delta)
    h32 = hier.astype(np.float32)
    exact = _exact_hierarchy(kh, kv, delta, childs[:L - 1])
    rounded = np.vectorize(_f32, otypes=[np.float32])
    differ = 0
    for l in range(L):
        for got, ex in zip(h32.coeffs[l], exact[l]):
            assert got.dtype == np.float32
            want = rounded(ex)
            assert np.array_equal(got.view(np.uint32), want.view(np.uint32)), l
        if l > 0:
            # the same coarsening done in float32 from the float32 fine level
            f32 = helmholtz.coarsen(*h32.coeffs[l - 1], childs[l - 1])
            differ += sum(int((a.astype(np.float32) != b).sum())
                          for a, b in zip(f32, h32.coeffs[l]))
    assert differ > 0   # the pin tells the two rules apart


def _skeel(sub, diag, sup, z):
    """Skeel condition number cond(A, z) of every column's tridiagonal matrix A
    at the solution z (infinity norm)."""
    nz, ncol = diag.shape
    out = np.empty(ncol)
    for c in range(ncol):
        A = np.diag(diag[:, c]) + np.diag(sub[1:, c], -1) + np.diag(sup[:-1, c], 1)
        zc = np.abs(z[:, c])
        out[c] = np.abs(np.abs(np.linalg.inv(A)) @ np.abs(A) @ zc).max() / zc.max()
    return out


@pytest.mark.parametrize("w_v,graded", [(100.0, False), (1000.0, True)])
def test_float32_thomas_within_condition_bound(w_v, graded):
    N, nz = 4, 30
    kh, kv, delta = workloads.coefficients(N, nz, 1.0, w_v, graded)
    lev = mesh.Level(N)
    sub, diag, sup = (a.astype(np.float32) for a in
                      helmholtz.column_tridiagonal(lev, kh, kv, delta))
    r = workloads.rhs(N, nz, seed=31)[0].astype(np.float32)
    z32 = smoother.thomas(sub, diag, sup, r)
    assert z32.dtype == np.float32
    z64 = np.empty(r.shape)
    for c in range(diag.shape[1]):
        ab = np.zeros((3, nz))
        ab[0, 1:] = sup[:-1, c]
        ab[1] = diag[:, c]
        ab[2, :-1] = sub[1:, c]
        z64[:, c] = solve_banded((1, 1), ab, r[:, c].astype(np.float64))
    cond = _skeel(sub.astype(np.float64), diag.astype(np.float64), sup.astype(np.float64), z64)
    err = np.abs(z32 - z64).max(axis=0) / np.abs(z64).max(axis=0)
    assert (err <= 2.0 * cond * U32).all(), (err / (cond * U32)).max()


@pytest.mark.parametrize("omega,n", [(0.8, 4), (1.0, 1), (0.7, 3)])
def test_float32_single_level_closed_form(omega, n):
    """w_h = 0, L = 1: x = (1 - (1 - omega)^n) H^-1 b. The float32 result is
    within 2 (n + 1) cond u of it, cond the largest column Skeel condition
    number at H^-1 b (each sweep adds a residual rounded in float32 and a
    Thomas solve with its forward error; the data are rounded once)."""
    N, nz = 4, 20
    kh, kv, delta = workloads.coefficients(N, nz, 0.0, 1000.0, True)
    levels, parents, childs = mesh.hierarchy(N, 1)
    hier = helmholtz.Hierarchy(levels, parents, childs, kh, kv, delta)
    b = workloads.rhs(N, nz, seed=32)[0]
    sub, diag, sup = hier.column_tridiagonal(0)
    exact = (1.0 - (1.0 - omega) ** n) * smoother.thomas(sub, diag, sup, b)
    prm = MGParams(omega=omega, n_pre=0, n_post=0, n_coarse=n)
    x32 = multigrid.vcycle(hier.astype(np.float32), b.astype(np.float32), prm)
    assert x32.dtype == np.float32
    cond = _skeel(sub, diag, sup, exact).max()
    err = np.abs(x32.astype(np.float64) - exact).max() / np.abs(exact).max()
    assert err <= 2.0 * (n + 1) * cond * U32, (err, cond)
    # and the float64 V-cycle hits it to rounding
    x64 = multigrid.vcycle(hier, b, prm)
    assert np.abs(x64 - exact).max() <= 1e-12 * np.abs(exact).max()
