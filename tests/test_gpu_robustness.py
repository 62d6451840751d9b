"""GPU: determinism, argument errors through the C ABI, degenerate shapes,
several live handles, the timing hook and larger batches."""
import ctypes

import numpy as np
import pytest
import torch

import workloads
from oracle import adjoint, helmholtz, krylov, mesh
from oracle.multigrid import MGParams

pytestmark = pytest.mark.gpu


def _hier(N, nz, L, w_h=1.0, w_v=100.0, graded=False):
    kh, kv, delta = workloads.coefficients(N, nz, w_h, w_v, graded)
    levels, parents, childs = mesh.hierarchy(N, L)
    return helmholtz.Hierarchy(levels, parents, childs, kh, kv, delta), (kh, kv, delta)


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_solve_is_bitwise_deterministic(precision):
    from paper_2002_00756_amd import Operator
    print(f"determinism {precision}", flush=True)
    _, (kh, kv, delta) = _hier(24, 30, 4, w_v=1000.0, graded=True)
    op = Operator(24, 30, kh, kv, delta, 4, precision=precision)
    b = torch.from_numpy(workloads.rhs(24, 30)[0]).cuda()
    r1 = op.solve(b, rtol=1e-9)
    r2 = op.solve(b, rtol=1e-9)
    assert r1.iters == r2.iters and r1.relres == r2.relres
    assert torch.equal(r1.x, r2.x)


def test_abi_rejects_bad_calls():
    from paper_2002_00756_amd import Operator, _lib
    _, (kh, kv, delta) = _hier(8, 4, 2)
    op = Operator(8, 4, kh, kv, delta, 2, max_batch=2)
    lib = op.lib
    x = torch.zeros((3, 4, 384), dtype=torch.float64, device="cuda")
    y = torch.empty_like(x)
    s = torch.cuda.current_stream().cuda_stream
    assert lib.helmholtz_apply(op._h, x.data_ptr(), y.data_ptr(), 3, s) == _lib.ESHAPE
    assert lib.helmholtz_apply(op._h, x.data_ptr(), y.data_ptr(), 0, s) == _lib.ESHAPE
    assert lib.helmholtz_apply(op._h, None, y.data_ptr(), 1, s) == _lib.EINVAL
    it = (ctypes.c_int32 * 1)()
    rr = (ctypes.c_double * 1)()
    assert lib.helmholtz_solve(op._h, x.data_ptr(), y.data_ptr(), 1, 1e-6, 0, it, rr, s) == \
        _lib.EINVAL
    assert lib.helmholtz_solve(op._h, x.data_ptr(), y.data_ptr(), 1, -1.0, 10, it, rr, s) == \
        _lib.EINVAL
    assert lib.helmholtz_profile_read(op._h, 7, None, None, None) == _lib.EINVAL
    # workspace too small
    h = ctypes.c_void_p()
    ws = torch.empty(1024, dtype=torch.uint8, device="cuda")
    assert lib.helmholtz_create(ctypes.byref(op.cfg), 1, 1, 1, ws.data_ptr() + 0, 1024, s,
                                ctypes.byref(h)) == _lib.EWORKSPACE


def test_single_level_and_single_layer():
    """nz = 1 (the column solve is a division) and L = 1 block-Jacobi PCG."""
    from paper_2002_00756_amd import Operator
    print("nz=1 and L=1", flush=True)
    hier, (kh, kv, delta) = _hier(12, 1, 3)
    op = Operator(12, 1, kh, kv, delta, 3)
    b = workloads.rhs(12, 1)[0]
    res = op.solve(torch.from_numpy(b).cuda(), rtol=1e-10)
    ref = krylov.solve(hier, b, rtol=1e-10)
    assert abs(res.iters[0] - ref.iters) <= 1
    assert np.linalg.norm(res.x.cpu().numpy() - ref.x) <= 1e-8 * np.linalg.norm(ref.x)
    gkh, gkv, gdl = op.face_grad(res.x, res.x)
    assert gkv.numel() == 0 and torch.isfinite(gkh).all() and torch.isfinite(gdl).all()

    prm = MGParams(omega=1.0, n_coarse=1)
    hier1, (kh, kv, delta) = _hier(24, 10, 1, w_v=1000.0)
    op1 = Operator(24, 10, kh, kv, delta, 1, prm.n_pre, prm.n_post, prm.n_coarse, prm.omega)
    b = workloads.rhs(24, 10)[0]
    res = op1.solve(torch.from_numpy(b).cuda(), rtol=1e-8, maxiter=500)
    ref = krylov.solve(hier1, b, rtol=1e-8, params=prm, maxiter=500)
    assert res.converged and abs(res.iters[0] - ref.iters) <= 1
    assert np.linalg.norm(res.x.cpu().numpy() - ref.x) <= 1e-6 * np.linalg.norm(ref.x)


def test_independent_handles():
    """Two operators alive at once keep separate workspaces and state."""
    from paper_2002_00756_amd import Operator
    h1, c1 = _hier(8, 6, 3, w_v=100.0)
    h2, c2 = _hier(8, 6, 3, w_v=1000.0, graded=True)
    op1 = Operator(8, 6, *c1, 3)
    op2 = Operator(8, 6, *c2, 3, precision="fp32")
    b = workloads.rhs(8, 6)[0]
    bd = torch.from_numpy(b).cuda()
    r1, r2 = op1.solve(bd, rtol=1e-10), op2.solve(bd, rtol=1e-10)
    x1 = krylov.solve(h1, b, rtol=1e-12).x
    x2 = krylov.solve(h2, b, rtol=1e-12).x
    assert np.linalg.norm(r1.x.cpu().numpy() - x1) <= 1e-8 * np.linalg.norm(x1)
    assert np.linalg.norm(r2.x.cpu().numpy() - x2) <= 1e-8 * np.linalg.norm(x2)


def test_timing_hook_counts_launches():
    from paper_2002_00756_amd import Operator, _lib
    _, (kh, kv, delta) = _hier(48, 20, 4)
    op = Operator(48, 20, kh, kv, delta, 4, precision="fp32")
    b = torch.from_numpy(workloads.rhs(48, 20)[0]).cuda()
    op.profile(True)
    res = op.solve(b, rtol=1e-8)
    ms, n, by = op.profile_read(_lib.PROF_SWEEP_FINE)
    ams, an, aby = op.profile_read(_lib.PROF_APPLY_FINE)
    op.profile(False)
    # one plain sweep per V-cycle on the finest level (2 pre: zero + plain; the
    # post-smoothing plain sweep), one V-cycle per iteration
    assert n == 2 * res.iters[0] and ms > 0
    assert by == pytest.approx(n * 7 * 4 * 20 * 6 * 48 * 48)
    assert an == res.iters[0] and aby == pytest.approx(an * 6 * 8 * 20 * 6 * 48 * 48)
    op.profile(True)
    assert op.profile_read(_lib.PROF_SWEEP_FINE)[1] == 0


def test_batch_of_eight_matches_single_solves():
    from paper_2002_00756_amd import Operator
    print("batch 8", flush=True)
    _, (kh, kv, delta) = _hier(24, 30, 4, w_v=1000.0, graded=True)
    op = Operator(24, 30, kh, kv, delta, 4, precision="fp32", max_batch=8)
    b = torch.from_numpy(workloads.rhs(24, 30, 8)).cuda()
    res = op.solve(b, rtol=1e-8)
    for i in (0, 5):
        single = op.solve(b[i], rtol=1e-8)
        assert single.iters[0] == res.iters[i]
        assert torch.allclose(single.x, res.x[i], rtol=0, atol=1e-12 * float(single.x.abs().max()))
    lam = op.solve(b.flip(0).contiguous(), rtol=1e-8).x
    gkh, gkv, gdl = op.face_grad(lam, res.x)
    lev = mesh.Level(24)
    rkh, rkv, rdl = adjoint.face_gradients(lev, lam.cpu().numpy(), res.x.cpu().numpy())
    assert np.allclose(gkh.cpu().numpy(), rkh, rtol=1e-12, atol=1e-12 * np.abs(rkh).max())


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("N,nz,L", [(24, 30, 4), (64, 6, 3)])
def test_batch_members_converging_at_different_iterations(precision, N, nz, L):
    """A member that has converged stops while the others go on: every later
    launch must leave it untouched. Each member equals its own solve, bit for
    bit (no kernel mixes right-hand sides). At N = 64 the apply and the
    residual restriction are the patch kernels, whose workgroups leave as a
    whole for a finished member."""
    from paper_2002_00756_amd import Operator
    print(f"batch with staggered convergence {precision} N={N}", flush=True)
    hier, (kh, kv, delta) = _hier(N, nz, L, w_v=1000.0, graded=True)
    op = Operator(N, nz, kh, kv, delta, L, precision=precision, max_batch=3)
    r = workloads.rhs(N, nz)[0]
    # a random right-hand side and a second one that the oracle solves in a
    # different number of iterations at 1e-8 (N = 24: constant along each
    # column, 5 and 6; N = 64: H 1, 6 and 5), and a zero one
    second = np.tile(r.mean(axis=0), (nz, 1)) if N == 24 else hier.apply(0, np.ones_like(r))
    b = np.stack([r, second, np.zeros_like(r)])
    res = op.solve(torch.from_numpy(b).cuda(), rtol=1e-8)
    assert res.converged and res.iters[2] == 0 and not res.x[2].any()
    if precision == "fp64":
        assert res.iters[0] != res.iters[1]
    print(f"  iterations {list(res.iters)}", flush=True)
    for i in (0, 1):
        single = op.solve(torch.from_numpy(b[i]).cuda(), rtol=1e-8)
        assert single.iters[0] == res.iters[i]
        assert torch.equal(single.x, res.x[i])


def test_cg_first_iteration_stop_and_batch_maxiter():
    """The owed x update where the iteration stops: a solve that converges in
    its first iteration (x is written, not added to) against the oracle, and a
    batch stopped by maxiter against the single solves, bit for bit."""
    from paper_2002_00756_amd import Operator
    print("CG stops at iteration 1 and at maxiter", flush=True)
    hier, (kh, kv, delta) = _hier(12, 10, 3)
    for precision in ("fp64", "fp32"):
        op = Operator(12, 10, kh, kv, delta, 3, precision=precision, max_batch=2)
        b = workloads.rhs(12, 10, 2, seed=21)
        bd = torch.from_numpy(b).cuda()
        res = op.solve(bd[0], rtol=0.9)
        ref = krylov.solve(hier, b[0], rtol=0.9)
        assert res.iters[0] == ref.iters == 1
        assert np.linalg.norm(res.x.cpu().numpy() - ref.x) <= 1e-5 * np.linalg.norm(ref.x)
        both = op.solve(bd, rtol=1e-14, maxiter=3)
        assert not both.converged and list(both.iters) == [3, 3]
        for i in range(2):
            single = op.solve(bd[i], rtol=1e-14, maxiter=3)
            assert torch.equal(single.x, both.x[i])
