"""Pins of the oracle's transfers and V-cycle against dense linear algebra."""
import os

import numpy as np
import pytest

import workloads
from oracle import helmholtz, mesh, multigrid, smoother
from oracle.multigrid import MGParams

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _hier(N, nz, L, w_h=1.0, w_v=100.0, graded=False):
    levels, parents, childs = mesh.hierarchy(N, L)
    kh, kv, delta = workloads.coefficients(N, nz, w_h, w_v, graded)
    return helmholtz.Hierarchy(levels, parents, childs, kh, kv, delta)


def _dense(hier, l):
    return helmholtz.assemble(hier.levels[l], *hier.coeffs[l]).toarray()


def _dense_Hz_inv(hier, l):
    sub, diag, sup = hier.column_tridiagonal(l)
    n = diag.size
    return np.stack([smoother.thomas(sub, diag, sup, e.reshape(diag.shape)).ravel()
                     for e in np.eye(n)], axis=1)


def _dense_P(hier, l, nz):
    par = hier.parents[l]
    P1 = np.zeros((par.size, hier.levels[l + 1].ncol))
    P1[np.arange(par.size), par] = 1.0
    return np.kron(np.eye(nz), P1)


def _closed_form_B(hier, l, nz, prm):
    """Dense V-cycle matrix: B = (I - E) H^-1, E = S^post (I - P B_c P^T H) S^pre."""
    H = _dense(hier, l)
    n = H.shape[0]
    S = np.eye(n) - prm.omega * _dense_Hz_inv(hier, l) @ H
    if l == hier.nlevels - 1:
        Bl = np.zeros((n, n))
        Sm = np.eye(n)
        for _ in range(prm.n_coarse):
            Bl += Sm @ (prm.omega * _dense_Hz_inv(hier, l))
            Sm = S @ Sm
        return Bl
    P = _dense_P(hier, l, nz)
    Bc = _closed_form_B(hier, l + 1, nz, prm)
    E = np.linalg.matrix_power(S, prm.n_post) @ (np.eye(n) - P @ Bc @ P.T @ H) \
        @ np.linalg.matrix_power(S, prm.n_pre)
    return (np.eye(n) - E) @ np.linalg.inv(H)


def test_paper_parameters_are_the_defaults():
    vals = dict(l.split() for l in open(os.path.join(GOLDEN, "mg_parameters.txt"))
                if l.strip() and not l.startswith("#"))
    prm = MGParams()
    assert prm.omega == float(vals["omega"])
    assert (prm.n_pre, prm.n_post, prm.n_coarse) == \
        (int(vals["n_pre"]), int(vals["n_post"]), int(vals["n_coarse"]))


def test_restriction_is_dual_of_prolongation():
    hier = _hier(8, 3, 2)
    rng = np.random.default_rng(9)
    r = rng.standard_normal((3, hier.levels[0].ncol))
    e = rng.standard_normal((3, hier.levels[1].ncol))
    lhs = np.vdot(multigrid.restrict(r, hier.childs[0]), e)
    rhs = np.vdot(r, multigrid.prolongate(e, hier.parents[0]))
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)
    one_c = np.ones((3, hier.levels[1].ncol))
    assert np.array_equal(multigrid.prolongate(one_c, hier.parents[0]),
                          np.ones((3, hier.levels[0].ncol)))
    assert np.array_equal(multigrid.restrict(np.ones((3, hier.levels[0].ncol)), hier.childs[0]),
                          4 * one_c)


@pytest.mark.parametrize("N,nz,L,prm", [
    (4, 3, 3, MGParams()),
    (4, 2, 2, MGParams(omega=0.7, n_pre=1, n_post=3, n_coarse=2)),
    (2, 3, 1, MGParams()),
    (4, 2, 2, MGParams(n_pre=0, n_post=2)),
])
def test_vcycle_equals_dense_closed_form(N, nz, L, prm):
    hier = _hier(N, nz, L, w_h=3.0)
    n = nz * hier.levels[0].ncol
    B = np.stack([multigrid.vcycle(hier, e.reshape(nz, -1), prm).ravel()
                  for e in np.eye(n)], axis=1)
    ref = _closed_form_B(hier, 0, nz, prm)
    assert np.allclose(B, ref, rtol=1e-11, atol=1e-12 * np.abs(ref).max())


def test_vcycle_symmetric_positive_definite():
    hier = _hier(4, 3, 3, w_h=5.0, w_v=1000.0)
    n = 3 * hier.levels[0].ncol
    B = np.stack([multigrid.vcycle(hier, e.reshape(3, -1)).ravel() for e in np.eye(n)], axis=1)
    assert np.abs(B - B.T).max() <= 1e-12 * np.abs(B).max()
    assert np.linalg.eigvalsh(0.5 * (B + B.T)).min() > 0
    H = _dense(hier, 0)
    ev = np.linalg.eigvals(B @ H).real
    assert ev.max() / ev.min() < 2.0        # a strong preconditioner


def test_single_level_without_horizontal_coupling():
    """w_h = 0, L = 1: n sweeps from zero give (1 - (1 - omega)^n) H^-1 b exactly."""
    hier = _hier(2, 5, 1, w_h=0.0, w_v=1000.0)
    b = workloads.rhs(2, 5)[0]
    prm = MGParams()
    x = multigrid.vcycle(hier, b, prm)
    H = _dense(hier, 0)
    xs = np.linalg.solve(H, b.ravel())
    assert np.allclose(x.ravel(), (1 - (1 - prm.omega) ** prm.n_coarse) * xs, rtol=1e-11)


def test_vcycle_batch_is_per_rhs():
    hier = _hier(4, 3, 2)
    b = workloads.rhs(4, 3, batch=3)
    x = multigrid.vcycle(hier, b)
    for i in range(3):
        assert np.allclose(x[i], multigrid.vcycle(hier, b[i]), rtol=0, atol=0)
