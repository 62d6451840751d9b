"""Pins of the oracle's operator, coarse operators and column solve."""
import numpy as np
import pytest
import scipy.linalg as sla
import scipy.sparse as sp

import workloads
from oracle import helmholtz, mesh, smoother


def _op(N, nz, w_h=1.0, w_v=100.0, graded=False, seed=0):
    lev = mesh.Level(N)
    kh, kv, delta = workloads.coefficients(N, nz, w_h, w_v, graded, seed)
    return lev, kh, kv, delta


def _brute_force_unit_laplacian(N, nz):
    """delta = 0, all couplings 1: graph Laplacian from 3-D geometry, no tables."""
    cen = np.empty((6 * N * N, 3))
    for p in range(6):
        for j in range(N):
            for i in range(N):
                cen[mesh.column_index(N, p, i, j)] = mesh.cell_centre(N, p, i, j)
    d2 = ((cen[:, None] - cen[None]) ** 2).sum(-1)
    A = ((d2 > 0) & (d2 <= 4)).astype(float)
    Lh = np.diag(A.sum(1)) - A
    T = np.zeros((nz, nz))
    for k in range(nz - 1):
        T[k, k] += 1; T[k + 1, k + 1] += 1; T[k, k + 1] -= 1; T[k + 1, k] -= 1
    # unknown index k*ncol + c
    return np.kron(np.eye(nz), Lh) + np.kron(T, np.eye(A.shape[0]))


@pytest.mark.parametrize("N,nz", [(2, 1), (2, 3), (3, 4), (4, 2)])
def test_structure_matches_geometry(N, nz):
    lev = mesh.Level(N)
    ncol = 6 * N * N
    kh = np.ones((2, nz, ncol)); kv = np.ones((nz - 1, ncol)); delta = np.zeros((nz, ncol))
    H = helmholtz.assemble(lev, kh, kv, delta).toarray()
    assert np.array_equal(H, _brute_force_unit_laplacian(N, nz))


@pytest.mark.parametrize("N,nz", [(2, 3), (4, 5), (3, 1)])
def test_apply_matches_assembled_and_is_symmetric(N, nz):
    lev, kh, kv, delta = _op(N, nz)
    H = helmholtz.assemble(lev, kh, kv, delta)
    assert abs(H - H.T).max() == 0.0
    x = np.random.default_rng(5).standard_normal((2, nz, lev.ncol))
    y = helmholtz.apply(lev, kh, kv, delta, x)
    for b in range(2):
        ref = (H @ x[b].ravel()).reshape(nz, lev.ncol)
        assert np.allclose(y[b], ref, rtol=1e-13, atol=1e-11)


def test_constant_vector_gives_delta():
    lev, kh, kv, delta = _op(6, 10, w_v=1000.0)
    y = helmholtz.apply(lev, kh, kv, delta, np.ones((10, lev.ncol)))
    assert np.allclose(y, delta, rtol=0, atol=1e-12)


def test_spectrum_bounds():
    lev, kh, kv, delta = _op(2, 3)
    H = helmholtz.assemble(lev, kh, kv, delta).toarray()
    ev = np.linalg.eigvalsh(H)
    assert ev.min() >= delta.min() - 1e-12          # Laplacian part is PSD
    rows = np.abs(H).sum(1)
    assert ev.max() <= rows.max() + 1e-12           # Gershgorin


@pytest.mark.parametrize("N,nz", [(2, 3), (4, 2), (6, 4)])
def test_coarse_operator_closed_form(N, nz):
    """H_c = P^T (L_h / 2 + L_v + diag(delta)) P with P the injection (Section 3.6)."""
    lev, kh, kv, delta = _op(N, nz, graded=True)
    levc = mesh.Level(N // 2)
    par = mesh.parent(N)
    khc, kvc, dc = helmholtz.coarsen(kh, kv, delta, mesh.children(N // 2))
    Hc = helmholtz.assemble(levc, khc, kvc, dc).toarray()
    ncf, ncc = lev.ncol, levc.ncol
    P1 = sp.csr_matrix((np.ones(ncf), (np.arange(ncf), par)), shape=(ncf, ncc))
    P = sp.kron(sp.eye(nz), P1).toarray()
    Lh = helmholtz.assemble(lev, kh, np.zeros_like(kv), np.zeros_like(delta)).toarray()
    Lv = helmholtz.assemble(lev, np.zeros_like(kh), kv, np.zeros_like(delta)).toarray()
    ref = P.T @ (0.5 * Lh + Lv + np.diag(delta.ravel())) @ P
    assert np.allclose(Hc, ref, rtol=1e-13, atol=1e-10)


def test_thomas_matches_banded_solver():
    rng = np.random.default_rng(3)
    nz, ncol = 9, 7
    off = rng.uniform(0.1, 2.0, (nz - 1, ncol))
    diag = rng.uniform(0.5, 1.0, (nz, ncol))
    diag[:-1] += off; diag[1:] += off
    sub = np.zeros((nz, ncol)); sup = np.zeros((nz, ncol))
    sub[1:] = -off; sup[:-1] = -off
    r = rng.standard_normal((2, nz, ncol))
    z = smoother.thomas(sub, diag, sup, r)
    for b in range(2):
        for c in range(ncol):
            ab = np.zeros((3, nz))
            ab[0, 1:] = sup[:-1, c]; ab[1] = diag[:, c]; ab[2, :-1] = sub[1:, c]
            ref = sla.solve_banded((1, 1), ab, r[b, :, c])
            assert np.allclose(z[b, :, c], ref, rtol=1e-13, atol=1e-13)


def test_thomas_single_level_is_division():
    lev, kh, kv, delta = _op(2, 1)
    sub, diag, sup = helmholtz.column_tridiagonal(lev, kh, kv, delta)
    r = np.random.default_rng(1).standard_normal((1, lev.ncol))
    K = helmholtz.face_coeffs(kh, lev.ftab)
    assert np.allclose(smoother.thomas(sub, diag, sup, r), r / (delta + K.sum(0)), rtol=1e-15)


def test_column_operator_is_H_without_horizontal_couplings():
    lev, kh, kv, delta = _op(2, 4)
    sub, diag, sup = helmholtz.column_tridiagonal(lev, kh, kv, delta)
    H = helmholtz.assemble(lev, kh, kv, delta).toarray()
    nz, ncol = delta.shape
    Hz = np.zeros_like(H)
    idx = np.arange(nz * ncol).reshape(nz, ncol)
    Hz[idx.ravel(), idx.ravel()] = diag.ravel()
    Hz[idx[1:].ravel(), idx[:-1].ravel()] = sub[1:].ravel()
    Hz[idx[:-1].ravel(), idx[1:].ravel()] = sup[:-1].ravel()
    dH = H - Hz
    # what remains only couples different columns at the same level
    rr, cc = np.nonzero(np.abs(dH) > 1e-12 * np.abs(H).max())
    assert np.all(rr // ncol == cc // ncol) and np.all(rr % ncol != cc % ncol)


def test_block_jacobi_exact_without_horizontal_coupling():
    """w_h = 0 makes H = H_z, so one sweep with omega = 1 is an exact solve."""
    lev, kh, kv, delta = _op(3, 6, w_h=0.0, w_v=1000.0)
    levels, parents, childs = mesh.hierarchy(3, 1)
    hier = helmholtz.Hierarchy(levels, parents, childs, kh, kv, delta)
    b = workloads.rhs(3, 6)[0]
    x = smoother.block_jacobi(hier, 0, b, None, 1.0, 1)
    H = helmholtz.assemble(lev, kh, kv, delta)
    assert np.allclose(H @ x.ravel(), b.ravel(), rtol=1e-12, atol=1e-10)


def test_jacobi_iteration_matrix_spectrum():
    """eig(Hz^-1 H) lies in (0, 2), so omega <= 1 contracts."""
    lev, kh, kv, delta = _op(2, 3, w_h=5.0)
    H = helmholtz.assemble(lev, kh, kv, delta).toarray()
    sub, diag, sup = helmholtz.column_tridiagonal(lev, kh, kv, delta)
    n = H.shape[0]
    Hzinv = np.stack([smoother.thomas(sub, diag, sup, e.reshape(delta.shape)).ravel()
                      for e in np.eye(n)], axis=1)
    ev = np.linalg.eigvals(Hzinv @ H).real
    assert ev.min() > 0 and ev.max() < 2
