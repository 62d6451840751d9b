"""GPU parity: the HIP library against the float64 oracle, through the C ABI.

Tolerances: float64 operator applies and V-cycles agree to 1e-10 relative
(max abs difference over max abs value); solves take the same number of
iterations +-1; float32 V-cycles are compared with a bound derived from
float32 rounding (see each test).
"""
import numpy as np
import pytest
import torch

import workloads
from oracle import adjoint, helmholtz, krylov, mesh, multigrid
from oracle.multigrid import MGParams

pytestmark = pytest.mark.gpu


def _flush(msg):
    print(msg, flush=True)


def _rel(a, ref):
    a = a.detach().cpu().numpy() if isinstance(a, torch.Tensor) else a
    return float(np.abs(a - ref).max() / max(np.abs(ref).max(), 1e-300))


def _setup(N, nz, L, w_h=1.0, w_v=100.0, graded=False, precision="fp64", batch=1,
           prm=MGParams(), cg="standard"):
    from paper_2002_00756_amd import Operator
    kh, kv, delta = workloads.coefficients(N, nz, w_h, w_v, graded)
    levels, parents, childs = mesh.hierarchy(N, L)
    hier = helmholtz.Hierarchy(levels, parents, childs, kh, kv, delta)
    op = Operator(N, nz, torch.from_numpy(kh), torch.from_numpy(kv), torch.from_numpy(delta),
                  L, prm.n_pre, prm.n_post, prm.n_coarse, prm.omega, precision, cg,
                  max_batch=batch)
    return hier, op


def _cuda(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


CASES = [
    # N, nz, L, w_h, w_v, graded
    (12, 10, 3, 1.0, 100.0, False),
    (8, 1, 2, 1.0, 100.0, False),
    (4, 3, 3, 5.0, 1000.0, False),
    (24, 30, 4, 1.0, 1000.0, True),
    (6, 70, 2, 1.0, 1000.0, True),
    (16, 120, 5, 2.0, 10.0, False),
    # the residual restriction in coarse patches staged through LDS: 16 x 16
    # patches (coarse panel width 16), 32 x 8 then 16 x 16 (widths 32, 16)
    (32, 8, 3, 1.0, 1000.0, True),
    (64, 6, 3, 1.0, 100.0, False),
    (64, 1, 2, 1.0, 100.0, False),  # one layer: no vertical couplings
]


@pytest.mark.parametrize("N,nz,L,w_h,w_v,graded", CASES)
def test_apply_parity(N, nz, L, w_h, w_v, graded):
    _flush(f"apply N={N} nz={nz}")
    hier, op = _setup(N, nz, L, w_h, w_v, graded, batch=3)
    x = workloads.rhs(N, nz, 3, seed=7)
    y = op.apply(_cuda(x))
    torch.cuda.synchronize()
    assert _rel(y, hier.apply(0, x)) <= 1e-12


@pytest.mark.parametrize("N,nz,L,w_h,w_v,graded", CASES)
def test_vcycle_fp64_parity(N, nz, L, w_h, w_v, graded):
    _flush(f"vcycle64 N={N} nz={nz} L={L}")
    hier, op = _setup(N, nz, L, w_h, w_v, graded, batch=2)
    b = workloads.rhs(N, nz, 2)
    x = op.vcycle(_cuda(b))
    torch.cuda.synchronize()
    assert _rel(x, multigrid.vcycle(hier, b)) <= 1e-10


@pytest.mark.parametrize("prm", [
    MGParams(omega=0.7, n_pre=1, n_post=3, n_coarse=2),
    MGParams(n_pre=0, n_post=2),
    MGParams(n_pre=2, n_post=0),
    MGParams(n_pre=0, n_post=0, n_coarse=1),
    MGParams(omega=1.0, n_pre=3, n_post=1, n_coarse=5),
])
def test_vcycle_parameter_variants(prm):
    _flush(f"vcycle variant {prm}")
    hier, op = _setup(8, 5, 3, 2.0, 100.0, prm=prm)
    b = workloads.rhs(8, 5)
    x = op.vcycle(_cuda(b))
    torch.cuda.synchronize()
    assert _rel(x, multigrid.vcycle(hier, b, prm)) <= 1e-10


@pytest.mark.parametrize("N,nz,L", [(12, 10, 3), (24, 30, 4), (8, 70, 4), (64, 6, 3)])
def test_vcycle_fp32(N, nz, L):
    """Float32 V-cycle against the float32 emulation and the float64 V-cycle.

    Gates (max-norm, relative): about three times the largest errors measured
    on MI355X over these cases (float32 V-cycle vs the float64 oracle 2.0e-7,
    vs the float32 emulation 5.9e-7, float64 entry point of a float32 handle
    2.0e-7). The a-priori bound, the columns' condition number (up to about
    4 kv / delta = 4e3) times the float32 rounding 6e-8, is 2.4e-4.
    """
    _flush(f"vcycle32 N={N} nz={nz}")
    hier, op = _setup(N, nz, L, 1.0, 1000.0, True, precision="fp32")
    b = workloads.rhs(N, nz)
    x32 = op.vcycle_f32(_cuda(b.astype(np.float32)))
    x64in = op.vcycle(_cuda(b))
    torch.cuda.synchronize()
    ref64 = multigrid.vcycle(hier, b)
    ref32 = multigrid.vcycle(hier.astype(np.float32), b.astype(np.float32)).astype(np.float64)
    _flush(f"  fp32 V-cycle vs fp64 oracle {_rel(x32.double(), ref64):.3e}, vs float32 "
           f"emulation {_rel(x32.double(), ref32):.3e}, fp64 entry {_rel(x64in, ref64):.3e}")
    assert _rel(x32.double(), ref64) <= 6e-7
    assert _rel(x32.double(), ref32) <= 1.6e-6
    assert _rel(x64in, ref64) <= 6e-7


def test_solve_config1_fp64():
    """C12 x 10, 3 levels, CG to 1e-8: iterations +-1, solution 1e-8."""
    w = workloads.C12x10
    _flush("solve C12x10")
    hier, op = _setup(w.N, w.nz, w.nlevels, w.w_h, w.w_v, w.graded)
    b = workloads.rhs(w.N, w.nz)[0]
    ref = krylov.solve(hier, b, rtol=1e-8)
    res = op.solve(_cuda(b), rtol=1e-8)
    assert res.converged
    assert abs(res.iters[0] - ref.iters) <= 1
    x = res.x.cpu().numpy()
    assert np.linalg.norm(x - ref.x) <= 1e-6 * np.linalg.norm(ref.x)
    true = np.linalg.norm(b - hier.apply(0, x)) / np.linalg.norm(b)
    assert true <= 2e-8


@pytest.mark.parametrize("flexible", [False, True])
def test_solve_batch_and_variants(flexible):
    _flush(f"solve batch flexible={flexible}")
    hier, op = _setup(8, 6, 3, 1.0, 100.0, batch=3, cg="flexible" if flexible else "standard")
    b = workloads.rhs(8, 6, 3)
    b[1] = 0.0                         # zero right-hand side: zero iterations
    res = op.solve(_cuda(b), rtol=1e-10)
    assert res.iters[1] == 0 and res.relres[1] == 0.0
    assert not res.x[1].any()
    for i in (0, 2):
        ref = krylov.solve(hier, b[i], rtol=1e-10, flexible=flexible)
        assert abs(res.iters[i] - ref.iters) <= 1
        assert np.linalg.norm(res.x[i].cpu().numpy() - ref.x) <= 1e-8 * np.linalg.norm(ref.x)


def test_solve_maxiter_and_nonfinite():
    from paper_2002_00756_amd import HelmholtzError
    hier, op = _setup(8, 6, 3)
    b = workloads.rhs(8, 6)[0]
    res = op.solve(_cuda(b), rtol=1e-14, maxiter=2)
    assert not res.converged and res.iters[0] == 2
    b[2, 5] = np.nan
    with pytest.raises(HelmholtzError):
        op.solve(_cuda(b))


def test_create_rejects_bad_coefficients():
    from paper_2002_00756_amd import HelmholtzError, Operator
    kh, kv, delta = workloads.coefficients(4, 3)
    delta[0, 0] = -1.0
    with pytest.raises(HelmholtzError):
        Operator(4, 3, kh, kv, delta, 2)
    delta[0, 0] = np.inf
    with pytest.raises(HelmholtzError):
        Operator(4, 3, kh, kv, delta, 2)


def test_solve_c96_mg_vs_block_jacobi():
    """C96 x 30 (w_v = 1000): MG-PCG against 1-level block-Jacobi PCG to 1e-6."""
    w = workloads.C96x30
    _flush("solve C96x30")
    hier, op = _setup(w.N, w.nz, w.nlevels, w.w_h, w.w_v, w.graded)
    b = workloads.rhs(w.N, w.nz)[0]
    ref = krylov.solve(hier, b, rtol=1e-6)
    res = op.solve(_cuda(b), rtol=1e-6)
    assert res.converged and abs(res.iters[0] - ref.iters) <= 1
    _, bj = _setup(w.N, w.nz, 1, w.w_h, w.w_v, w.graded, prm=MGParams(omega=1.0, n_coarse=1))
    rbj = bj.solve(_cuda(b), rtol=1e-6, maxiter=1000)
    assert rbj.converged and rbj.iters[0] > res.iters[0]


def test_face_grad_parity():
    _flush("face_grad")
    hier, op = _setup(12, 10, 3, batch=2)
    rng = np.random.default_rng(3)
    lam = rng.standard_normal((2, 10, 864))
    x = rng.standard_normal((2, 10, 864))
    gkh, gkv, gdl = op.face_grad(_cuda(lam), _cuda(x))
    rkh, rkv, rdl = adjoint.face_gradients(hier.levels[0], lam, x)
    assert _rel(gkh, rkh) <= 1e-13 and _rel(gkv, rkv) <= 1e-13 and _rel(gdl, rdl) <= 1e-13


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_vcycle_misaligned_input(precision):
    """Inputs that start one element past an aligned address (a contiguous view
    into a larger buffer) take the element-wise load path and give the same
    V-cycle as an aligned copy."""
    _flush(f"vcycle misaligned {precision}")
    hier, op = _setup(8, 10, 3, 1.0, 100.0, precision=precision)
    b = workloads.rhs(8, 10)[0]
    dt = torch.float32 if precision == "fp32" else torch.float64
    big = torch.zeros(b.size + 1, dtype=dt, device="cuda")
    big[1:] = torch.from_numpy(b.ravel()).to(dt)
    view = big[1:].view(b.shape)
    assert view.is_contiguous() and view.data_ptr() % (2 * view.element_size()) != 0
    fn = op.vcycle_f32 if precision == "fp32" else op.vcycle
    z_view = fn(view)
    z_copy = fn(view.clone())
    torch.cuda.synchronize()
    assert torch.equal(z_view, z_copy)
    if precision == "fp64":
        assert _rel(z_view, multigrid.vcycle(hier, b)) <= 1e-10
