"""Pins of the oracle's PCG and its float32-preconditioner form."""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

import workloads
from oracle import helmholtz, krylov, mesh, multigrid
from oracle.multigrid import MGParams


def _hier(w):
    levels, parents, childs = mesh.hierarchy(w.N, w.nlevels)
    kh, kv, delta = workloads.workload_coefficients(w)
    return helmholtz.Hierarchy(levels, parents, childs, kh, kv, delta)


def test_pcg_matches_dense_solve():
    w = workloads.Workload("t", 4, 4, 2.0, 100.0, False, 3)
    hier = _hier(w)
    b = workloads.rhs(w.N, w.nz)[0]
    res = krylov.solve(hier, b, rtol=1e-13)
    H = helmholtz.assemble(hier.levels[0], *hier.coeffs[0]).toarray()
    ref = np.linalg.solve(H, b.ravel())
    assert res.converged
    assert np.linalg.norm(res.x.ravel() - ref) <= 1e-11 * np.linalg.norm(ref)


def test_pcg_manufactured_solution_c12():
    w = workloads.C12x10
    hier = _hier(w)
    xs = np.random.default_rng(11).standard_normal((w.nz, w.ncol))
    b = hier.apply(0, xs)
    res = krylov.solve(hier, b, rtol=1e-13)
    assert res.converged and res.iters < 30
    assert np.linalg.norm(res.x - xs) <= 1e-10 * np.linalg.norm(xs)


def test_pcg_zero_rhs():
    hier = _hier(workloads.C12x10)
    res = krylov.solve(hier, np.zeros((10, 864)))
    assert res.iters == 0 and res.converged and not res.x.any()


def test_pcg_maxiter_reports_not_converged():
    hier = _hier(workloads.C12x10)
    res = krylov.solve(hier, workloads.rhs(12, 10)[0], rtol=1e-14, maxiter=2)
    assert res.iters == 2 and not res.converged


def test_unpreconditioned_cg_agrees_with_scipy():
    """With M = I the loop is plain CG; compare with SciPy's CG on the same matrix."""
    w = workloads.Workload("t", 2, 3, 1.0, 10.0, False, 1)
    hier = _hier(w)
    H = helmholtz.assemble(hier.levels[0], *hier.coeffs[0])
    b = workloads.rhs(2, 3)[0]
    res = krylov.pcg(lambda v: hier.apply(0, v), lambda r: r, b, rtol=1e-12, maxiter=500)
    ref, info = spla.cg(H, b.ravel(), rtol=1e-13, maxiter=1000)
    assert info == 0 and res.converged
    assert res.iters <= b.size
    assert np.allclose(res.x.ravel(), ref, rtol=1e-9, atol=1e-10)


@pytest.mark.parametrize("flexible", [False, True])
def test_config1_converges_fast(flexible):
    w = workloads.C12x10
    hier = _hier(w)
    b = workloads.rhs(w.N, w.nz)[0]
    res = krylov.solve(hier, b, rtol=1e-8, flexible=flexible)
    assert res.converged and res.iters <= 12
    true = np.linalg.norm(b - hier.apply(0, res.x)) / np.linalg.norm(b)
    assert true <= 2e-8


def test_float32_preconditioner_keeps_float64_accuracy():
    w = workloads.C12x10
    hier = _hier(w)
    b = workloads.rhs(w.N, w.nz)[0]
    ref = krylov.solve(hier, b, rtol=1e-12)
    mixed = krylov.solve(hier, b, rtol=1e-8, precision="fp32", flexible=True)
    assert mixed.converged
    err = np.linalg.norm(mixed.x - ref.x) / np.linalg.norm(ref.x)
    assert err <= 1e-7
    # the float32 V-cycle itself is close to the float64 one
    z64 = multigrid.vcycle(hier, b)
    z32 = multigrid.vcycle(hier.astype(np.float32), b.astype(np.float32))
    assert z32.dtype == np.float32
    assert np.linalg.norm(z32 - z64) <= 1e-5 * np.linalg.norm(z64)


def test_block_jacobi_pcg_needs_more_iterations():
    """Single-level P_H^(Jac)(1.0, 1) against the MG preconditioner (Table 1 structure)."""
    w = workloads.Workload("t", 12, 10, 1.0, 1000.0, False, 3)
    hier = _hier(w)
    b = workloads.rhs(w.N, w.nz)[0]
    mg = krylov.solve(hier, b, rtol=1e-6)
    bj = krylov.solve(hier, b, rtol=1e-6, params=MGParams(omega=1.0, n_coarse=1),
                      ) if hier.nlevels == 1 else None
    levels, parents, childs = mesh.hierarchy(w.N, 1)
    h1 = helmholtz.Hierarchy(levels, parents, childs, *hier.coeffs[0])
    bj = krylov.solve(h1, b, rtol=1e-6, params=MGParams(omega=1.0, n_coarse=1))
    assert mg.converged and bj.converged
    assert bj.iters > mg.iters


# ---- BiCGStab (Section 4.1) -------------------------------------------------

def _nonsymmetric(n, seed):
    """Diagonally dominant, clearly non-symmetric test matrix."""
    rng = np.random.default_rng(seed)
    A = rng.uniform(-1.0, 1.0, (n, n))
    A += np.diag(np.abs(A).sum(axis=1) + 1.0)
    return A


def test_bicgstab_iterates_match_scipy():
    """Same algorithm (right preconditioning, shadow residual b, x0 = 0): the
    iterate after k steps agrees with SciPy's to rounding, for k = 1..6, on a
    non-symmetric matrix with a non-trivial preconditioner (Jacobi)."""
    n = 40
    A = _nonsymmetric(n, 5)
    b = np.random.default_rng(6).standard_normal(n)
    d = 1.0 / np.diag(A)
    M = spla.LinearOperator((n, n), matvec=lambda v: d * v)
    for k in range(1, 7):
        ref, _ = spla.bicgstab(A, b, rtol=1e-300, atol=0.0, maxiter=k, M=M)
        res = krylov.bicgstab(lambda v: A @ v, lambda v: d * v, b, rtol=0.0, maxiter=k)
        assert res.iters == k
        assert np.linalg.norm(res.x - ref) <= 1e-12 * np.linalg.norm(ref)


def test_bicgstab_converges_to_dense_solve():
    n = 60
    A = _nonsymmetric(n, 7)
    b = np.random.default_rng(8).standard_normal(n)
    res = krylov.bicgstab(lambda v: A @ v, lambda v: v, b, rtol=1e-13, maxiter=200)
    ref = np.linalg.solve(A, b)
    assert res.converged
    assert np.linalg.norm(A @ res.x - b) <= 1e-13 * np.linalg.norm(b) * 1.0001
    assert np.linalg.norm(res.x - ref) <= 1e-11 * np.linalg.norm(ref)


def test_bicgstab_exact_preconditioner_one_step():
    """With P = A^-1: p_hat = A^-1 b, v = b, alpha = 1, s = 0, t = 0, omega = 0,
    so one step gives x = A^-1 b exactly up to rounding."""
    n = 30
    A = _nonsymmetric(n, 9)
    Ainv = np.linalg.inv(A)
    b = np.random.default_rng(10).standard_normal(n)
    res = krylov.bicgstab(lambda v: A @ v, lambda v: Ainv @ v, b, rtol=1e-10, maxiter=5)
    assert res.converged and res.iters == 1
    assert np.linalg.norm(res.x - np.linalg.solve(A, b)) <= 1e-12 * np.linalg.norm(res.x)


def test_bicgstab_zero_rhs_and_maxiter():
    A = _nonsymmetric(20, 11)
    res = krylov.bicgstab(lambda v: A @ v, lambda v: v, np.zeros(20))
    assert res.converged and res.iters == 0 and not res.x.any()
    b = np.ones(20)
    res = krylov.bicgstab(lambda v: A @ v, lambda v: v, b, rtol=0.0, maxiter=3)
    assert not res.converged and res.iters == 3


@pytest.mark.parametrize("L", [1, 3])
def test_bicgstab_mg_and_jacobi_on_helmholtz(L):
    """BiCGStab + MG(L) (L = 1: P_Jac(1, 1)) on the C12 operator converges to the
    dense solution; the MG-preconditioned one needs far fewer iterations."""
    w = workloads.Workload("t", 12, 10, 1.0, 100.0, False, L)
    hier = _hier(w)
    b = workloads.rhs(w.N, w.nz)[0]
    prm = MGParams() if L > 1 else MGParams(omega=1.0, n_coarse=1)
    res = krylov.solve(hier, b, rtol=1e-11, params=prm, method="bicgstab", maxiter=400)
    H = helmholtz.assemble(hier.levels[0], *hier.coeffs[0]).tocsc()
    ref = spla.spsolve(H, b.ravel()).reshape(b.shape)
    assert res.converged
    assert np.linalg.norm(res.x - ref) <= 1e-9 * np.linalg.norm(ref)
    assert res.iters <= (8 if L > 1 else 400)
