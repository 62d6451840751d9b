"""Pins of the oracle's 9-cell stencil (Section 3.5: each cell also coupled to
the cells two levels above and below; the smoother drops those couplings,
Section 3.6)."""
import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spla

import workloads
from oracle import adjoint, helmholtz, krylov, mesh, multigrid, smoother
from oracle.multigrid import MGParams


def _op(N, nz, w_h=1.0, w_v=100.0, w_v2=1.0, graded=False):
    lev = mesh.Level(N)
    kh, kv, delta = workloads.coefficients(N, nz, w_h, w_v, graded)
    kv2 = workloads.next_nearest(N, nz, w_v2, graded)
    return lev, kh, kv, delta, kv2


def _hier(N, nz, L, w_h=1.0, w_v=100.0, w_v2=1.0, graded=False):
    levels, parents, childs = mesh.hierarchy(N, L)
    kh, kv, delta = workloads.coefficients(N, nz, w_h, w_v, graded)
    kv2 = workloads.next_nearest(N, nz, w_v2, graded)
    return helmholtz.Hierarchy(levels, parents, childs, kh, kv, delta, kv2=kv2)


def _geometry_laplacian(N, nz):
    """Unit couplings from 3-D cell centres (no tables): horizontal neighbours at
    squared distance <= 4, vertical neighbours one and two levels apart."""
    cen = np.empty((6 * N * N, 3))
    for p in range(6):
        for j in range(N):
            for i in range(N):
                cen[mesh.column_index(N, p, i, j)] = mesh.cell_centre(N, p, i, j)
    d2 = ((cen[:, None] - cen[None]) ** 2).sum(-1)
    A = ((d2 > 0) & (d2 <= 4)).astype(float)
    Lh = np.diag(A.sum(1)) - A
    T = np.zeros((nz, nz))
    for k in range(nz):
        for d in (1, 2):
            if k + d < nz:
                T[k, k] += 1; T[k + d, k + d] += 1; T[k, k + d] -= 1; T[k + d, k] -= 1
    return np.kron(np.eye(nz), Lh) + np.kron(T, np.eye(A.shape[0]))


@pytest.mark.parametrize("N,nz", [(2, 3), (2, 5), (3, 2)])
def test_structure_matches_geometry(N, nz):
    lev = mesh.Level(N)
    ncol = lev.ncol
    H = helmholtz.assemble(lev, np.ones((2, nz, ncol)), np.ones((nz - 1, ncol)),
                           np.zeros((nz, ncol)), kv2=np.ones((max(nz - 2, 0), ncol)))
    assert np.array_equal(H.toarray(), _geometry_laplacian(N, nz))


def test_nine_point_rows_symmetry_spd_and_constants():
    lev, kh, kv, delta, kv2 = _op(2, 7)
    H = helmholtz.assemble(lev, kh, kv, delta, kv2=kv2)
    assert abs(H - H.T).max() == 0.0
    nnz = np.diff(H.indptr).reshape(7, lev.ncol)
    assert np.all(nnz[2:-2] == 9)                         # the 9-cell stencil
    assert np.all(nnz[0] == 7) and np.all(nnz[1] == 8)    # bottom rows
    assert np.linalg.eigvalsh(H.toarray()).min() >= delta.min() - 1e-12
    y = helmholtz.apply(lev, kh, kv, delta, np.ones((7, lev.ncol)), kv2=kv2)
    assert np.allclose(y, delta, rtol=0, atol=1e-12)
    x = np.random.default_rng(2).standard_normal((2, 7, lev.ncol))
    y = helmholtz.apply(lev, kh, kv, delta, x, kv2=kv2)
    for b in range(2):
        assert np.allclose(y[b].ravel(), H @ x[b].ravel(), rtol=1e-13, atol=1e-10)


def test_smoother_matrix_is_tridiagonal_part_of_column_block():
    """Per column: the smoother's matrix equals the column block of H with the
    k+-2 entries set to zero (their value is -kv2); the diagonal is H's."""
    lev, kh, kv, delta, kv2 = _op(2, 6)
    H = helmholtz.assemble(lev, kh, kv, delta, kv2=kv2).toarray()
    sub, diag, sup = helmholtz.column_tridiagonal(lev, kh, kv, delta, kv2=kv2)
    nz, ncol = delta.shape
    for c in range(ncol):
        blk = H[np.ix_(np.arange(nz) * ncol + c, np.arange(nz) * ncol + c)]
        assert np.allclose(np.diag(blk, 2), -kv2[:, c], rtol=1e-15)
        tri = np.diag(diag[:, c]) + np.diag(sub[1:, c], -1) + np.diag(sup[:-1, c], 1)
        ref = blk - np.diag(np.diag(blk, 2), 2) - np.diag(np.diag(blk, -2), -2)
        assert np.allclose(tri, ref, rtol=1e-15, atol=0)


def test_block_jacobi_spectrum_and_energy_decrease():
    """eig(Hz^-1 H) in (0, 2) also with the dropped couplings (2 Hz - H is
    positive definite), so every undamped sweep reduces the error in the
    energy norm. Without horizontal coupling the smoother is no longer an exact
    solve (the k+-2 couplings are dropped), unlike the 7-point case."""
    lev, kh, kv, delta, kv2 = _op(2, 5, w_h=5.0, w_v=100.0, w_v2=40.0)
    H = helmholtz.assemble(lev, kh, kv, delta, kv2=kv2).toarray()
    sub, diag, sup = helmholtz.column_tridiagonal(lev, kh, kv, delta, kv2=kv2)
    n = H.shape[0]
    Hzinv = np.stack([smoother.thomas(sub, diag, sup, e.reshape(delta.shape)).ravel()
                      for e in np.eye(n)], axis=1)
    ev = np.linalg.eigvals(Hzinv @ H).real
    assert ev.min() > 0 and ev.max() < 2
    lev, kh, kv, delta, kv2 = _op(2, 6, w_h=0.0, w_v2=2.0)
    levels, parents, childs = mesh.hierarchy(2, 1)
    hier = helmholtz.Hierarchy(levels, parents, childs, kh, kv, delta, kv2=kv2)
    b = workloads.rhs(2, 6)[0]
    H = hier.assemble(0).toarray()
    xs = np.linalg.solve(H, b.ravel())
    x = None
    energy = []
    for _ in range(40):
        x = smoother.block_jacobi(hier, 0, b, x, 1.0, 1)
        e = x.ravel() - xs
        energy.append(float(e @ H @ e))
    assert energy[0] > 1e-8 * float(xs @ H @ xs)          # not exact in one sweep
    assert all(b_ < a for a, b_ in zip(energy, energy[1:]))
    assert energy[-1] < 1e-6 * energy[0]


@pytest.mark.parametrize("N,nz", [(2, 4), (4, 5)])
def test_coarse_operator_closed_form(N, nz):
    """H_c = P^T (L_h / 2 + L_v + L_v2 + diag(delta)) P, P the injection."""
    lev, kh, kv, delta, kv2 = _op(N, nz, graded=True)
    levc = mesh.Level(N // 2)
    ch = mesh.children(N // 2)
    khc, kvc, dc = helmholtz.coarsen(kh, kv, delta, ch)
    kv2c = helmholtz.coarsen_kv2(kv2, ch)
    Hc = helmholtz.assemble(levc, khc, kvc, dc, kv2=kv2c).toarray()
    par = mesh.parent(N)
    P1 = sp.csr_matrix((np.ones(lev.ncol), (np.arange(lev.ncol), par)),
                       shape=(lev.ncol, levc.ncol))
    P = sp.kron(sp.eye(nz), P1).toarray()
    z = np.zeros_like
    Lh = helmholtz.assemble(lev, kh, z(kv), z(delta)).toarray()
    Lv = helmholtz.assemble(lev, z(kh), kv, z(delta)).toarray()
    Lv2 = helmholtz.assemble(lev, z(kh), z(kv), z(delta), kv2=kv2).toarray()
    ref = P.T @ (0.5 * Lh + Lv + Lv2 + np.diag(delta.ravel())) @ P
    assert np.allclose(Hc, ref, rtol=1e-13, atol=1e-10)


def test_vcycle_dense_closed_form_and_spd():
    """The V-cycle on the 9-cell hierarchy equals (I - E) H^-1 built from dense
    matrices (smoother S = I - omega Hz^-1 H on every level) and is SPD."""
    nz, L = 5, 2
    hier = _hier(4, nz, L, w_h=3.0, w_v2=30.0)
    prm = MGParams()

    def dense_hz_inv(l):
        sub, diag, sup = hier.column_tridiagonal(l)
        return np.stack([smoother.thomas(sub, diag, sup, e.reshape(diag.shape)).ravel()
                         for e in np.eye(diag.size)], axis=1)

    def closed(l):
        H = hier.assemble(l).toarray()
        n = H.shape[0]
        Hzi = dense_hz_inv(l)
        S = np.eye(n) - prm.omega * Hzi @ H
        if l == hier.nlevels - 1:
            B, Sm = np.zeros((n, n)), np.eye(n)
            for _ in range(prm.n_coarse):
                B += Sm @ (prm.omega * Hzi)
                Sm = S @ Sm
            return B
        par = hier.parents[l]
        P1 = np.zeros((par.size, hier.levels[l + 1].ncol))
        P1[np.arange(par.size), par] = 1.0
        P = np.kron(np.eye(nz), P1)
        E = np.linalg.matrix_power(S, prm.n_post) @ (np.eye(n) - P @ closed(l + 1) @ P.T @ H) \
            @ np.linalg.matrix_power(S, prm.n_pre)
        return (np.eye(n) - E) @ np.linalg.inv(H)

    n = nz * hier.levels[0].ncol
    B = np.stack([multigrid.vcycle(hier, e.reshape(nz, -1), prm).ravel() for e in np.eye(n)],
                 axis=1)
    ref = closed(0)
    assert np.allclose(B, ref, rtol=1e-11, atol=1e-12 * np.abs(ref).max())
    assert np.abs(B - B.T).max() <= 1e-12 * np.abs(B).max()
    assert np.linalg.eigvalsh(0.5 * (B + B.T)).min() > 0


def test_cg_and_bicgstab_converge_to_dense_solution():
    w = workloads.C12x10_9
    hier = _hier(w.N, w.nz, w.nlevels, w.w_h, w.w_v, w.w_v2)
    b = workloads.rhs(w.N, w.nz)[0]
    ref = spla.spsolve(hier.assemble(0).tocsc(), b.ravel()).reshape(b.shape)
    for method in ("cg", "bicgstab"):
        res = krylov.solve(hier, b, rtol=1e-11, method=method)
        assert res.converged and res.iters < 20
        assert np.linalg.norm(res.x - ref) <= 1e-9 * np.linalg.norm(ref)


def test_kv2_gradient_dense_fd_and_homogeneity():
    N, nz, B = 2, 5, 2
    lev, kh, kv, delta, kv2 = _op(N, nz, w_v=50.0, w_v2=8.0)
    b = workloads.rhs(N, nz, B)
    g = workloads.loss_weights(N, nz, B)

    def solve(kv2_, v):
        H = helmholtz.assemble(lev, kh, kv, delta, kv2=kv2_).toarray()
        return np.linalg.solve(H, v.reshape(B, -1).T).T.reshape(v.shape)

    x, lam = solve(kv2, b), solve(kv2, g)
    gk2 = adjoint.kv2_gradient(lam, x)
    rng = np.random.default_rng(12)
    fds, ads = [], []
    for idx in rng.integers(kv2.size, size=8):
        unit = np.zeros_like(kv2)
        unit.flat[idx] = 1.0
        dH = helmholtz.assemble(lev, 0 * kh, 0 * kv, 0 * delta, kv2=unit).toarray()
        ref = -sum(lam[i].ravel() @ dH @ x[i].ravel() for i in range(B))
        assert np.isclose(gk2.flat[idx], ref, rtol=1e-10, atol=1e-13)
        h = 1e-4   # kv2 ~ 8: a 1e-5 relative step keeps FD rounding well below the gradient
        kp, km = kv2.copy(), kv2.copy()
        kp.flat[idx] += h
        km.flat[idx] -= h
        fds.append((np.sum(g * solve(kp, b)) - np.sum(g * solve(km, b))) / (2 * h))
        ads.append(gk2.flat[idx])
    fds, ads = np.array(fds), np.array(ads)
    assert np.linalg.norm(ads - fds) <= 1e-6 * np.linalg.norm(fds)
    # H is linear in all coefficients: sum c dL/dc = -L
    gkh, gkv, gd = adjoint.face_gradients(lev, lam, x)
    L = float(np.sum(g * x))
    s = np.sum(kh * gkh) + np.sum(kv * gkv) + np.sum(delta * gd) + np.sum(kv2 * gk2)
    assert abs(s + L) <= 1e-10 * abs(L)
