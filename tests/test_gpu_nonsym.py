"""GPU parity for the non-symmetric row-weighted operator H = delta + S L
(Section 5.1; the weight plays the role of 1/rho* in Eq.
continuum_pressure_operator), its transpose, the transposed V-cycle, BiCGStab
forward and adjoint solves and the weighted gradients, against the oracle.

Bars: float64 applies 1e-12 and V-cycles 1e-10 relative (max abs difference
over max abs value), solves within +-1 iteration of the oracle with the true
residual at the tolerance, gradients 1e-12.
"""
import numpy as np
import pytest
import torch

import workloads
from oracle import adjoint, helmholtz, krylov, mesh, multigrid

pytestmark = pytest.mark.gpu


def _setup(N, nz, L, w_h=1.0, w_v=100.0, graded=False, precision="fp64", batch=1):
    from paper_2002_00756_amd import Operator
    kh, kv, delta = workloads.coefficients(N, nz, w_h, w_v, graded)
    s = workloads.row_weights(N, nz)
    levels, parents, childs = mesh.hierarchy(N, L)
    hier = helmholtz.Hierarchy(levels, parents, childs, kh, kv, delta, s=s)
    op = Operator(N, nz, kh, kv, delta, L, precision=precision, cg="bicgstab", max_batch=batch,
                  s=s)
    return hier, op


def _rel(a, ref):
    a = a.detach().cpu().numpy() if isinstance(a, torch.Tensor) else a
    return float(np.abs(a - ref).max() / max(np.abs(ref).max(), 1e-300))


CASES = [
    # N, nz, L, w_h, w_v, graded
    (12, 10, 3, 1.0, 100.0, False),
    (8, 1, 2, 1.0, 100.0, False),
    (4, 3, 3, 5.0, 1000.0, False),
    (24, 30, 4, 1.0, 1000.0, True),
    (6, 70, 2, 1.0, 1000.0, True),
    # the apply and the residual restriction staged through LDS in patches
    # (panel widths 32 and 64), in H and in H^T
    (32, 8, 3, 1.0, 1000.0, True),
    (64, 6, 3, 1.0, 100.0, False),
]


@pytest.mark.parametrize("N,nz,L,w_h,w_v,graded", CASES)
def test_apply_and_vcycles(N, nz, L, w_h, w_v, graded):
    print(f"weighted apply/vcycle N={N} nz={nz} L={L}", flush=True)
    hier, op = _setup(N, nz, L, w_h, w_v, graded, batch=2)
    ht = hier.transpose()
    x = torch.from_numpy(workloads.rhs(N, nz, 2, seed=7)).cuda()
    xn = x.cpu().numpy()
    assert _rel(op.apply(x), hier.apply(0, xn)) <= 1e-12
    assert _rel(op.apply_adjoint(x), ht.apply(0, xn)) <= 1e-12
    assert _rel(op.vcycle(x), multigrid.vcycle(hier, xn)) <= 1e-10
    assert _rel(op.vcycle_adjoint(x), multigrid.vcycle(ht, xn)) <= 1e-10


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("N,nz,L", [(24, 30, 4), (64, 6, 3)])
def test_forward_and_adjoint_solves(precision, N, nz, L):
    print(f"weighted solves N={N} {precision}", flush=True)
    hier, op = _setup(N, nz, L, w_v=1000.0, graded=True, precision=precision)
    ht = hier.transpose()
    b = workloads.rhs(N, nz)[0]
    g = workloads.loss_weights(N, nz)[0]
    for rtol in (1e-6, 1e-10):
        for h, rhs, fn in ((hier, b, op.solve), (ht, g, op.solve_adjoint)):
            ref = krylov.solve(h, rhs, rtol=rtol, method="bicgstab")
            res = fn(torch.from_numpy(rhs).cuda(), rtol=rtol)
            assert res.converged and abs(res.iters[0] - ref.iters) <= 1, (res.iters, ref.iters)
            true = np.linalg.norm(rhs - h.apply(0, res.x.cpu().numpy())) / np.linalg.norm(rhs)
            assert true <= rtol * 1.05 + 1e-13


def test_weighted_gradients_and_duality():
    N, nz, L = 12, 10, 3
    hier, op = _setup(N, nz, L, batch=2)
    lam = workloads.rhs(N, nz, 2, seed=3)
    x = workloads.rhs(N, nz, 2, seed=4)
    got = op.face_grad(torch.from_numpy(lam).cuda(), torch.from_numpy(x).cuda())
    kh, kv, delta = hier.coeffs[0]
    ref = adjoint.weighted_gradients(hier.levels[0], kh, kv, hier.ss[0], lam, x)
    for a, r in zip(got, ref):
        assert _rel(a, r) <= 1e-12
    # <lam, b> = <g, x> for x = H^-1 b, lam = H^-T g
    b = torch.from_numpy(workloads.rhs(N, nz)[0]).cuda()
    g = torch.from_numpy(workloads.loss_weights(N, nz)[0]).cuda()
    xs = op.solve(b, rtol=1e-13).x
    ls = op.solve_adjoint(g, rtol=1e-13).x
    lhs, rhs_ = float(torch.sum(ls * b)), float(torch.sum(g * xs))
    assert abs(lhs - rhs_) <= 1e-10 * abs(rhs_)


def test_weighted_handle_rejects_symmetric_calls():
    from paper_2002_00756_amd import Operator, _lib
    N, nz = 8, 4
    kh, kv, delta = workloads.coefficients(N, nz)
    s = workloads.row_weights(N, nz)
    with pytest.raises(_lib.HelmholtzError):
        Operator(N, nz, kh, kv, delta, 2, cg="standard", s=s)     # CG needs symmetry
    op = Operator(N, nz, kh, kv, delta, 2, cg="bicgstab", s=s)
    z = torch.zeros((1, nz, 6 * N * N), dtype=torch.float64, device="cuda")
    gkh = torch.empty((2, nz, 6 * N * N), dtype=torch.float64, device="cuda")
    code = op.lib.helmholtz_face_grad(op._h, z.data_ptr(), z.data_ptr(), 1, gkh.data_ptr(),
                                      gkh.data_ptr(), gkh.data_ptr(), None)
    assert code == _lib.EINVAL
