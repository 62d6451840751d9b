"""GPU: the Krylov drivers queue work ahead of their read of each published
residual norm. CG queues M r, r.z and beta of the next iteration when the norm
is predicted to stay above the tolerance, and the x update of the right-hand
sides that stop otherwise. BiCGStab queues the next iteration up to its x and
r update. The kernels skip right-hand sides whose device flag the norm
cleared, so the results must not depend on the guess: every solve here equals,
bit for bit, the same solve with the library's timing hook on, which turns the
queueing off. The tolerances sweep across the iterations where each guess is
right and where it is wrong."""
import numpy as np
import pytest
import torch

import workloads

pytestmark = pytest.mark.gpu


def _pair(op, b, rtol, maxiter=200):
    op.profile(True)
    ref = op.solve(b, rtol=rtol, maxiter=maxiter)
    op.profile(False)
    got = op.solve(b, rtol=rtol, maxiter=maxiter)
    return ref, got


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("cg", ["standard", "flexible"])
@pytest.mark.parametrize("N,nz,L", [(24, 30, 4), (64, 6, 3)])
def test_queued_ahead_matches_in_order(precision, cg, N, nz, L):
    from paper_2002_00756_amd import Operator
    print(f"queue ahead {precision} {cg} N={N}", flush=True)
    kh, kv, delta = workloads.coefficients(N, nz, 1.0, 1000.0, True)
    op = Operator(N, nz, kh, kv, delta, L, precision=precision, cg=cg, max_batch=3)
    r = workloads.rhs(N, nz)[0]
    # members that converge at different iterations, and one that never starts
    b = torch.from_numpy(np.stack([r, np.tile(r.mean(axis=0), (nz, 1)),
                                   np.zeros_like(r)])).cuda()
    seen = set()
    for rtol in (0.9, 0.3, 1e-1, 3e-2, 1e-2, 3e-3, 1e-3, 3e-4, 1e-4, 1e-5, 1e-6, 1e-7, 1e-8,
                 1e-9, 1e-10):
        for rhs in (b, b[0], b[1]):
            ref, got = _pair(op, rhs, rtol)
            assert got.iters == ref.iters and got.relres == ref.relres, rtol
            assert got.converged == ref.converged
            assert torch.equal(got.x, ref.x), rtol
            seen.update(got.iters)
    print(f"  iteration counts covered: {sorted(seen)}", flush=True)
    assert {1, 2, 3}.issubset(seen)


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_queued_ahead_at_maxiter(precision):
    """Stopped by maxiter while one member has converged earlier: the owed x
    update of the live members and of the finished one, each exactly once."""
    from paper_2002_00756_amd import Operator
    print(f"queue ahead at maxiter {precision}", flush=True)
    kh, kv, delta = workloads.coefficients(12, 10, 1.0, 100.0, False)
    op = Operator(12, 10, kh, kv, delta, 3, precision=precision, max_batch=2)
    r = workloads.rhs(12, 10)[0]
    b = torch.from_numpy(np.stack([r, np.tile(r.mean(axis=0), (10, 1))])).cuda()
    for maxiter in (1, 2, 3, 4):
        for rtol in (1e-14, 1e-4):
            ref, got = _pair(op, b, rtol, maxiter)
            assert got.iters == ref.iters and got.relres == ref.relres
            assert got.converged == ref.converged
            assert torch.equal(got.x, ref.x)


@pytest.mark.parametrize("weighted", [False, True])
def test_queued_ahead_bicgstab(weighted):
    from paper_2002_00756_amd import Operator
    print(f"queue ahead BiCGStab weighted={weighted}", flush=True)
    kh, kv, delta = workloads.coefficients(24, 30, 1.0, 1000.0, True)
    sw = workloads.row_weights(24, 30) if weighted else None
    op = Operator(24, 30, kh, kv, delta, 4, precision="fp32", cg="bicgstab", max_batch=3, s=sw)
    r = workloads.rhs(24, 30)[0]
    b = torch.from_numpy(np.stack([r, np.tile(r.mean(axis=0), (30, 1)), np.zeros_like(r)])).cuda()
    seen = set()
    for rtol in (0.9, 1e-1, 1e-2, 1e-3, 1e-4, 1e-5, 1e-6, 1e-8, 1e-10):
        for rhs in (b, b[0]):
            for maxiter in (200, 2):
                ref, got = _pair(op, rhs, rtol, maxiter)
                assert got.iters == ref.iters and got.relres == ref.relres, rtol
                assert got.converged == ref.converged
                assert torch.equal(got.x, ref.x), rtol
                seen.update(got.iters)
    print(f"  iteration counts covered: {sorted(seen)}", flush=True)
    assert {1, 2}.issubset(seen)
