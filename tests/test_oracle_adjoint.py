"""Pins of the oracle's gradients: dense reference, finite differences, identities."""
import numpy as np

import workloads
from oracle import adjoint, helmholtz, krylov, mesh


def _problem(N=2, nz=3, batch=2):
    lev = mesh.Level(N)
    kh, kv, delta = workloads.coefficients(N, nz, 1.0, 50.0)
    b = workloads.rhs(N, nz, batch)
    g = workloads.loss_weights(N, nz, batch)
    return lev, kh, kv, delta, b, g


def _loss(lev, kh, kv, delta, b, g):
    H = helmholtz.assemble(lev, kh, kv, delta).toarray()
    x = np.linalg.solve(H, b.reshape(b.shape[0], -1).T).T
    return float(np.sum(g.reshape(g.shape[0], -1) * x))


def _solve_dense(lev, kh, kv, delta, v):
    H = helmholtz.assemble(lev, kh, kv, delta).toarray()
    return np.linalg.solve(H, v.reshape(v.shape[0], -1).T).T.reshape(v.shape)


def test_gradient_matches_dense_derivative():
    """-lambda^T (dH/dc) x with dH/dc assembled from a unit coefficient."""
    lev, kh, kv, delta, b, g = _problem()
    x = _solve_dense(lev, kh, kv, delta, b)
    lam = _solve_dense(lev, kh, kv, delta, g)
    gkh, gkv, gd = adjoint.face_gradients(lev, lam, x)
    rng = np.random.default_rng(4)
    for name, arr, grad in (("kh", kh, gkh), ("kv", kv, gkv), ("delta", delta, gd)):
        for idx in rng.integers(arr.size, size=8):
            unit = [np.zeros_like(kh), np.zeros_like(kv), np.zeros_like(delta)]
            which = {"kh": 0, "kv": 1, "delta": 2}[name]
            unit[which].flat[idx] = 1.0
            dH = helmholtz.assemble(lev, *unit).toarray()
            ref = -sum(lam[i].ravel() @ dH @ x[i].ravel() for i in range(b.shape[0]))
            assert np.isclose(grad.flat[idx], ref, rtol=1e-10, atol=1e-13)


def test_gradient_matches_central_differences():
    lev, kh, kv, delta, b, g = _problem()
    x = _solve_dense(lev, kh, kv, delta, b)
    lam = _solve_dense(lev, kh, kv, delta, g)
    grads = dict(zip(("kh", "kv", "delta"), adjoint.face_gradients(lev, lam, x)))
    h = 1e-6
    sample = workloads.fd_sample(2, 3, count=24)
    fd, ad = [], []
    for name, idx in sample:
        arrs = {"kh": kh, "kv": kv, "delta": delta}
        plus = {k: v.copy() for k, v in arrs.items()}
        minus = {k: v.copy() for k, v in arrs.items()}
        plus[name].flat[idx] += h
        minus[name].flat[idx] -= h
        fd.append((_loss(lev, plus["kh"], plus["kv"], plus["delta"], b, g)
                   - _loss(lev, minus["kh"], minus["kv"], minus["delta"], b, g)) / (2 * h))
        ad.append(grads[name].flat[idx])
    fd, ad = np.array(fd), np.array(ad)
    assert np.linalg.norm(ad - fd) <= 1e-6 * np.linalg.norm(fd)


def test_homogeneity_and_duality():
    """H is linear in its coefficients, so sum c dL/dc = -L; and <lambda, b> = <g, x>."""
    w = workloads.C12x10
    levels, parents, childs = mesh.hierarchy(w.N, w.nlevels)
    kh, kv, delta = workloads.workload_coefficients(w)
    hier = helmholtz.Hierarchy(levels, parents, childs, kh, kv, delta)
    b = workloads.rhs(w.N, w.nz, 2)
    g = workloads.loss_weights(w.N, w.nz, 2)
    x = np.stack([krylov.solve(hier, b[i], rtol=1e-13).x for i in range(2)])
    lam = np.stack([krylov.solve(hier, g[i], rtol=1e-13).x for i in range(2)])
    gkh, gkv, gd = adjoint.face_gradients(levels[0], lam, x)
    L = float(np.sum(g * x))
    s = float(np.sum(kh * gkh) + np.sum(kv * gkv) + np.sum(delta * gd))
    assert abs(s + L) <= 1e-9 * abs(L)
    assert abs(np.sum(lam * b) - L) <= 1e-9 * abs(L)
