"""GPU parity for the pressure-solver configurations of Section 5.1 (Table 1):
right-preconditioned BiCGStab with the MG or block-Jacobi preconditioner,
the preconditioner-only solvers MG(L) and line relaxation P_Jac(0.8, 10).

Bars as for CG: iteration counts equal to the oracle's +-1, solutions within
1e-8 relative of the oracle's at the same tolerance (both stop on the
recursively updated residual, so the difference is bounded by the tolerance
times the condition of the stopping point; the cases here are tight), float64
V-cycles to 1e-10.
"""
import numpy as np
import pytest
import torch

import workloads
from oracle import helmholtz, krylov, mesh, multigrid
from oracle.multigrid import MGParams

pytestmark = pytest.mark.gpu

JAC1 = MGParams(omega=1.0, n_coarse=1)      # P_H^(Jac)(1.0, 1), one level
LINE = MGParams(omega=0.8, n_coarse=10)     # P_H^(Jac)(0.8, 10), one level


def _setup(N, nz, L, prm=MGParams(), w_h=1.0, w_v=100.0, graded=False, precision="fp64",
           batch=1, cg="bicgstab"):
    from paper_2002_00756_amd import Operator
    kh, kv, delta = workloads.coefficients(N, nz, w_h, w_v, graded)
    levels, parents, childs = mesh.hierarchy(N, L)
    hier = helmholtz.Hierarchy(levels, parents, childs, kh, kv, delta)
    op = Operator(N, nz, kh, kv, delta, L, prm.n_pre, prm.n_post, prm.n_coarse, prm.omega,
                  precision, cg, max_batch=batch)
    return hier, op


def _relnorm(a, ref):
    a = a.detach().cpu().numpy() if isinstance(a, torch.Tensor) else a
    return float(np.linalg.norm(a - ref) / np.linalg.norm(ref))


@pytest.mark.parametrize("L,prm,rtol", [(3, MGParams(), 1e-2), (3, MGParams(), 1e-6),
                                        (3, MGParams(), 1e-10), (1, JAC1, 1e-2),
                                        (1, JAC1, 1e-6), (4, MGParams(), 1e-8)])
def test_bicgstab_matches_oracle(L, prm, rtol):
    print(f"bicgstab L={L} omega={prm.omega} rtol={rtol}", flush=True)
    N, nz = (12, 10) if L < 4 else (24, 30)
    hier, op = _setup(N, nz, L, prm, w_v=100.0 if L < 4 else 1000.0, graded=L == 4)
    b = workloads.rhs(N, nz)[0]
    ref = krylov.solve(hier, b, rtol=rtol, params=prm, method="bicgstab", maxiter=500)
    res = op.solve(torch.from_numpy(b).cuda(), rtol=rtol, maxiter=500)
    assert ref.converged and res.converged
    assert abs(res.iters[0] - ref.iters) <= 1, (res.iters, ref.iters)
    if res.iters[0] == ref.iters:
        assert _relnorm(res.x, ref.x) <= 1e-8
    # true residual of the GPU solution within the tolerance (small slack for
    # the recursive residual's drift)
    true = np.linalg.norm(b - hier.apply(0, res.x.cpu().numpy())) / np.linalg.norm(b)
    assert true <= rtol * 1.05 + 1e-13


@pytest.mark.parametrize("N,cg", [(64, "bicgstab"), (32, "bicgstab"), (64, "standard"),
                                  (64, "flexible")])
def test_patch_staged_apply_matches_oracle(N, cg):
    """Panels whose width is a multiple of 64 (32) take the operator apply
    staged through LDS in 64 x 4 (32 x 8) column patches, with every dot
    product it carries ((r0, v) and (t, s), (t, t) in BiCGStab, p.q in CG)."""
    print(f"patch-staged apply N={N} {cg}", flush=True)
    nz, L, rtol = 6, 3, 1e-8
    hier, op = _setup(N, nz, L, w_v=1000.0, graded=True, cg=cg)
    b = workloads.rhs(N, nz)[0]
    method = "bicgstab" if cg == "bicgstab" else "cg"
    ref = krylov.solve(hier, b, rtol=rtol, method=method, flexible=cg == "flexible")
    res = op.solve(torch.from_numpy(b).cuda(), rtol=rtol)
    print(f"  iterations {res.iters[0]} (oracle {ref.iters}), solution "
          f"{_relnorm(res.x, ref.x):.2e}", flush=True)
    assert ref.converged and res.converged
    assert abs(res.iters[0] - ref.iters) <= 1
    if res.iters[0] == ref.iters:
        assert _relnorm(res.x, ref.x) <= 1e-8
    true = np.linalg.norm(b - hier.apply(0, res.x.cpu().numpy())) / np.linalg.norm(b)
    assert true <= rtol * 1.05 + 1e-13


def test_bicgstab_fp32_preconditioner():
    """Float32 V-cycle inside the float64 BiCGStab: same iterations as the float64
    oracle +-1 and the float64 true residual meets the tolerance."""
    N, nz, L = 24, 30, 4
    hier, op = _setup(N, nz, L, w_v=1000.0, graded=True, precision="fp32")
    b = workloads.rhs(N, nz)[0]
    for rtol in (1e-3, 1e-8):
        ref = krylov.solve(hier, b, rtol=rtol, method="bicgstab")
        res = op.solve(torch.from_numpy(b).cuda(), rtol=rtol)
        assert res.converged and abs(res.iters[0] - ref.iters) <= 1
        true = np.linalg.norm(b - hier.apply(0, res.x.cpu().numpy())) / np.linalg.norm(b)
        assert true <= rtol * 1.05


def test_bicgstab_batch_zero_rhs_and_maxiter():
    N, nz, L = 12, 10, 3
    hier, op = _setup(N, nz, L, batch=3)
    b = workloads.rhs(N, nz, 3)
    b[1] = 0.0
    res = op.solve(torch.from_numpy(b).cuda(), rtol=1e-9)
    assert res.iters[1] == 0 and res.relres[1] == 0.0 and not res.x[1].abs().max()
    for i in (0, 2):
        ref = krylov.solve(hier, b[i], rtol=1e-9, method="bicgstab")
        assert abs(res.iters[i] - ref.iters) <= 1
        assert _relnorm(res.x[i], ref.x) <= 1e-7
    # one iteration only: not converged, the oracle's first iterate
    _, op1 = _setup(N, nz, 1, JAC1)
    hier1, _ = _setup(N, nz, 1, JAC1)
    res = op1.solve(torch.from_numpy(b[0]).cuda(), rtol=1e-12, maxiter=1)
    assert not res.converged and res.iters[0] == 1
    ref = krylov.solve(hier1, b[0], rtol=1e-12, params=JAC1, method="bicgstab", maxiter=1)
    assert _relnorm(res.x, ref.x) <= 1e-10
    assert abs(res.relres[0] - ref.relres) <= 1e-10 * ref.relres


@pytest.mark.parametrize("L", [1, 2, 3, 4])
def test_preonly_mg_levels(L):
    """MG(L) as the whole pressure solver: one V-cycle, L = 1..4 (Table 1)."""
    N, nz = 24, 30
    hier, op = _setup(N, nz, L, w_v=1000.0, graded=True, cg="standard")
    b = workloads.rhs(N, nz, seed=4)[0]
    z = op.vcycle(torch.from_numpy(b).cuda())
    ref = multigrid.vcycle(hier, b)
    assert float(np.abs(z.cpu().numpy() - ref).max() / np.abs(ref).max()) <= 1e-10


def test_preonly_line_relaxation():
    """Line relaxation P_Jac(0.8, 10): ten block-Jacobi sweeps from zero."""
    N, nz = 24, 30
    hier, op = _setup(N, nz, 1, LINE, w_v=1000.0, graded=True, cg="standard")
    b = workloads.rhs(N, nz, seed=4)[0]
    z = op.vcycle(torch.from_numpy(b).cuda())
    ref = multigrid.vcycle(hier, b, LINE)
    assert float(np.abs(z.cpu().numpy() - ref).max() / np.abs(ref).max()) <= 1e-10
