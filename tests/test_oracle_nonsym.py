"""Pins of the oracle's non-symmetric (row-weighted) operator H = delta + S L
(Section 5.1: the paper's H is not symmetric; its horizontal part weights a
symmetric face Laplacian by a per-cell factor, Eq. continuum_pressure_operator),
its transpose, the transposed V-cycle and the gradients of the adjoint."""
import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spla

import workloads
from oracle import adjoint, helmholtz, krylov, mesh, multigrid, smoother
from oracle.multigrid import MGParams


def _op(N, nz, w_h=1.0, w_v=100.0, graded=False):
    lev = mesh.Level(N)
    kh, kv, delta = workloads.coefficients(N, nz, w_h, w_v, graded)
    return lev, kh, kv, delta, workloads.row_weights(N, nz)


def _hier(N, nz, L, w_h=1.0, w_v=100.0, graded=False):
    levels, parents, childs = mesh.hierarchy(N, L)
    kh, kv, delta = workloads.coefficients(N, nz, w_h, w_v, graded)
    return helmholtz.Hierarchy(levels, parents, childs, kh, kv, delta,
                               s=workloads.row_weights(N, nz))


def test_apply_transpose_and_symmetrisable():
    lev, kh, kv, delta, s = _op(2, 4)
    H = helmholtz.assemble(lev, kh, kv, delta, s=s).toarray()
    assert np.abs(H - H.T).max() > 1e-3 * np.abs(H).max()          # not symmetric
    Hs = H / s.ravel()[:, None]                                     # S^-1 H
    assert np.allclose(Hs, Hs.T, rtol=0, atol=1e-12 * np.abs(Hs).max())
    x = np.random.default_rng(1).standard_normal((2, 4, lev.ncol))
    y = helmholtz.apply(lev, kh, kv, delta, x, s=s)
    yt = helmholtz.apply(lev, kh, kv, delta, x, s=s, transpose=True)
    for b in range(2):
        assert np.allclose(y[b].ravel(), H @ x[b].ravel(), rtol=1e-13, atol=1e-11)
        assert np.allclose(yt[b].ravel(), H.T @ x[b].ravel(), rtol=1e-13, atol=1e-11)
    one = np.ones((4, lev.ncol))
    assert np.allclose(helmholtz.apply(lev, kh, kv, delta, one, s=s), delta, atol=1e-12)


@pytest.mark.parametrize("transpose", [False, True])
def test_column_matrices_are_column_blocks(transpose):
    lev, kh, kv, delta, s = _op(2, 5)
    H = helmholtz.assemble(lev, kh, kv, delta, s=s).toarray()
    if transpose:
        H = H.T
    sub, diag, sup = helmholtz.column_tridiagonal(lev, kh, kv, delta, s=s, transpose=transpose)
    nz, ncol = delta.shape
    for c in range(ncol):
        blk = H[np.ix_(np.arange(nz) * ncol + c, np.arange(nz) * ncol + c)]
        tri = np.diag(diag[:, c]) + np.diag(sub[1:, c], -1) + np.diag(sup[:-1, c], 1)
        assert np.allclose(tri, blk, rtol=1e-15, atol=0)


def test_smoother_spectrum():
    """Hz = S Hz' and H = S H' with Hz', H' symmetric: eig(Hz^-1 H) = eig(Hz'^-1 H')
    is real and in (0, 2)."""
    lev, kh, kv, delta, s = _op(2, 3, w_h=5.0)
    H = helmholtz.assemble(lev, kh, kv, delta, s=s).toarray()
    sub, diag, sup = helmholtz.column_tridiagonal(lev, kh, kv, delta, s=s)
    n = H.shape[0]
    Hzinv = np.stack([smoother.thomas(sub, diag, sup, e.reshape(delta.shape)).ravel()
                      for e in np.eye(n)], axis=1)
    ev = np.linalg.eigvals(Hzinv @ H)
    assert np.abs(ev.imag).max() < 1e-9
    assert ev.real.min() > 0 and ev.real.max() < 2


def test_coarse_operator_closed_form():
    """H_c = diag(delta_c) + S_c P^T (L_h / 2 + L_v) P, s_c the mean of the children."""
    N, nz = 4, 3
    lev, kh, kv, delta, s = _op(N, nz, graded=True)
    levc = mesh.Level(N // 2)
    ch = mesh.children(N // 2)
    khc, kvc, dc = helmholtz.coarsen(kh, kv, delta, ch)
    sc = helmholtz.coarsen_s(s, ch)
    Hc = helmholtz.assemble(levc, khc, kvc, dc, s=sc).toarray()
    par = mesh.parent(N)
    P1 = sp.csr_matrix((np.ones(lev.ncol), (np.arange(lev.ncol), par)),
                       shape=(lev.ncol, levc.ncol))
    P = sp.kron(sp.eye(nz), P1).toarray()
    z = np.zeros_like
    Lh = helmholtz.assemble(lev, kh, z(kv), z(delta)).toarray()
    Lv = helmholtz.assemble(lev, z(kh), kv, z(delta)).toarray()
    ref = np.diag(dc.ravel()) + np.diag(sc.ravel()) @ (P.T @ (0.5 * Lh + Lv) @ P)
    assert np.allclose(Hc, ref, rtol=1e-13, atol=1e-10)
    for C in range(levc.ncol):
        kids = [mesh.children(N // 2)[q][C] for q in range(4)]
        assert np.allclose(sc[:, C], s[:, kids].mean(axis=1), rtol=1e-15)


@pytest.mark.parametrize("prm", [MGParams(), MGParams(omega=0.7, n_pre=1, n_post=1, n_coarse=3)])
def test_transposed_vcycle_is_the_transpose(prm):
    """With n_pre = n_post, and the coarse operators of H^T the transposes of H's,
    the V-cycle of the transposed hierarchy is the transpose of H's V-cycle."""
    nz = 3
    hier = _hier(4, nz, 2, w_h=3.0)
    n = nz * hier.levels[0].ncol
    B = np.stack([multigrid.vcycle(hier, e.reshape(nz, -1), prm).ravel() for e in np.eye(n)],
                 axis=1)
    ht = hier.transpose()
    Bt = np.stack([multigrid.vcycle(ht, e.reshape(nz, -1), prm).ravel() for e in np.eye(n)],
                  axis=1)
    assert np.abs(B - B.T).max() > 1e-6 * np.abs(B).max()            # B itself not symmetric
    assert np.allclose(Bt, B.T, rtol=1e-11, atol=1e-12 * np.abs(B).max())


def test_bicgstab_forward_and_adjoint_solves():
    N, nz, L = 12, 10, 3
    hier = _hier(N, nz, L)
    b = workloads.rhs(N, nz)[0]
    g = workloads.loss_weights(N, nz)[0]
    H = hier.assemble(0).tocsc()
    for h, rhs, A in ((hier, b, H), (hier.transpose(), g, H.T.tocsc())):
        res = krylov.solve(h, rhs, rtol=1e-11, method="bicgstab")
        ref = spla.spsolve(A, rhs.ravel()).reshape(rhs.shape)
        assert res.converged and res.iters < 15
        assert np.linalg.norm(res.x - ref) <= 1e-9 * np.linalg.norm(ref)


def test_weighted_gradients_dense_fd_and_duality():
    N, nz, B = 2, 3, 2
    lev, kh, kv, delta, s = _op(N, nz, w_v=50.0)
    b = workloads.rhs(N, nz, B)
    g = workloads.loss_weights(N, nz, B)

    def H_of(kh_, kv_, dl_, s_):
        return helmholtz.assemble(lev, kh_, kv_, dl_, s=s_).toarray()

    def loss(kh_, kv_, dl_, s_):
        x_ = np.linalg.solve(H_of(kh_, kv_, dl_, s_), b.reshape(B, -1).T).T
        return float(np.sum(g.reshape(B, -1) * x_))

    H = H_of(kh, kv, delta, s)
    x = np.linalg.solve(H, b.reshape(B, -1).T).T.reshape(b.shape)
    lam = np.linalg.solve(H.T, g.reshape(B, -1).T).T.reshape(g.shape)
    grads = dict(zip(("kh", "kv", "delta", "s"),
                     adjoint.weighted_gradients(lev, kh, kv, s, lam, x)))
    arrs = {"kh": kh, "kv": kv, "delta": delta, "s": s}
    rng = np.random.default_rng(3)
    for name in arrs:
        for idx in rng.integers(arrs[name].size, size=6):
            # dense derivative dH/dc by a unit change (H is affine in each coefficient)
            plus = {k: v.copy() for k, v in arrs.items()}
            plus[name].flat[idx] += 1.0
            dH = H_of(plus["kh"], plus["kv"], plus["delta"], plus["s"]) - H
            ref = -sum(lam[i].ravel() @ dH @ x[i].ravel() for i in range(B))
            assert np.isclose(grads[name].flat[idx], ref, rtol=1e-9, atol=1e-12)
            h = 1e-6
            p_, m_ = ({k: v.copy() for k, v in arrs.items()} for _ in range(2))
            p_[name].flat[idx] += h
            m_[name].flat[idx] -= h
            fd = (loss(p_["kh"], p_["kv"], p_["delta"], p_["s"])
                  - loss(m_["kh"], m_["kv"], m_["delta"], m_["s"])) / (2 * h)
            assert abs(fd - grads[name].flat[idx]) <= 1e-6 * max(1.0, abs(fd))
    assert abs(np.sum(lam * b) - np.sum(g * x)) <= 1e-10 * abs(np.sum(g * x))
