"""GPU: the differentiable solve (forward solve, adjoint solve, fused face gradients)
against a dense reference, the oracle, and central finite differences."""
import numpy as np
import pytest
import torch

import workloads
from oracle import adjoint, helmholtz, krylov, mesh

pytestmark = pytest.mark.gpu


def _flush(msg):
    print(msg, flush=True)


def test_autograd_matches_dense_reference_c6x8():
    """C6 x 8 (1,728 unknowns), 2 levels: every gradient against dense linear algebra."""
    from paper_2002_00756_amd import helmholtz_solve
    w = workloads.C6x8
    _flush("autograd dense C6x8")
    kh, kv, delta = workloads.workload_coefficients(w)
    b = workloads.rhs(w.N, w.nz, 2)
    g = workloads.loss_weights(w.N, w.nz, 2)
    dev = torch.device("cuda")
    tkh = torch.tensor(kh, device=dev, requires_grad=True)
    tkv = torch.tensor(kv, device=dev, requires_grad=True)
    tdl = torch.tensor(delta, device=dev, requires_grad=True)
    tb = torch.tensor(b, device=dev, requires_grad=True)
    x = helmholtz_solve(tb, tkh, tkv, tdl, N=w.N, nz=w.nz, nlevels=w.nlevels, rtol=1e-13)
    loss = (torch.tensor(g, device=dev) * x).sum()
    loss.backward()

    lev = mesh.Level(w.N)
    H = helmholtz.assemble(lev, kh, kv, delta).toarray()
    xs = np.linalg.solve(H, b.reshape(2, -1).T).T.reshape(b.shape)
    lam = np.linalg.solve(H, g.reshape(2, -1).T).T.reshape(g.shape)
    rkh, rkv, rdl = adjoint.face_gradients(lev, lam, xs)

    def rel(a, r):
        return float(np.linalg.norm(a.detach().cpu().numpy() - r) / np.linalg.norm(r))
    assert rel(x, xs) <= 1e-11
    assert rel(tb.grad, lam) <= 1e-11
    assert rel(tkh.grad, rkh) <= 1e-10
    assert rel(tkv.grad, rkv) <= 1e-10
    assert rel(tdl.grad, rdl) <= 1e-10


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_autograd_matches_oracle_c12x10(precision):
    from paper_2002_00756_amd import helmholtz_solve
    w = workloads.C12x10
    _flush(f"autograd oracle C12x10 {precision}")
    kh, kv, delta = workloads.workload_coefficients(w)
    b = workloads.rhs(w.N, w.nz)[0]
    g = workloads.loss_weights(w.N, w.nz)[0]
    dev = torch.device("cuda")
    t = [torch.tensor(a, device=dev, requires_grad=True) for a in (b, kh, kv, delta)]
    x = helmholtz_solve(*t, N=w.N, nz=w.nz, nlevels=w.nlevels, rtol=1e-12, precision=precision,
                        cg="flexible" if precision == "fp32" else "standard")
    (torch.tensor(g, device=dev) * x).sum().backward()
    levels, parents, childs = mesh.hierarchy(w.N, w.nlevels)
    hier = helmholtz.Hierarchy(levels, parents, childs, kh, kv, delta)
    xs = krylov.solve(hier, b, rtol=1e-13).x
    lam = krylov.solve(hier, g, rtol=1e-13).x
    refs = [lam, *adjoint.face_gradients(levels[0], lam, xs)]
    for tt, r in zip(t, refs):
        err = float(np.linalg.norm(tt.grad.cpu().numpy() - r) / np.linalg.norm(r))
        assert err <= 1e-9, err


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_adjoint_gradient_matches_central_differences_c96x30(precision):
    """C96 x 30: 64 sampled coefficients, h = 1e-6, solves converged to 1e-14.

    Agreement ||g_adj - g_fd|| / ||g_fd|| <= 1e-5 over the sample.
    """
    from paper_2002_00756_amd import Operator
    w = workloads.C96x30
    _flush(f"FD C96x30 {precision}")
    kh, kv, delta = workloads.workload_coefficients(w)
    b = workloads.rhs(w.N, w.nz)[0]
    g = workloads.loss_weights(w.N, w.nz)[0]
    dev = torch.device("cuda")
    tb, tg = torch.tensor(b, device=dev), torch.tensor(g, device=dev)
    cg = "flexible" if precision == "fp32" else "standard"
    rtol = 1e-14

    def make(a_kh, a_kv, a_dl):
        return Operator(w.N, w.nz, a_kh, a_kv, a_dl, w.nlevels, precision=precision, cg=cg,
                        device=dev)

    base = {"kh": torch.tensor(kh, device=dev), "kv": torch.tensor(kv, device=dev),
            "delta": torch.tensor(delta, device=dev)}
    op = make(base["kh"], base["kv"], base["delta"])
    x = op.solve(tb, rtol=rtol, maxiter=100).x
    lam = op.solve(tg, rtol=rtol, maxiter=100).x
    grads = dict(zip(("kh", "kv", "delta"), op.face_grad(lam, x)))
    del op

    def loss(arrs):
        o = make(arrs["kh"], arrs["kv"], arrs["delta"])
        xx = o.solve(tb, rtol=rtol, maxiter=100).x
        return float(torch.dot(tg.flatten(), xx.flatten()))

    h = 1e-6
    fd, ad = [], []
    for name, idx in workloads.fd_sample(w.N, w.nz, count=64):
        plus = dict(base)
        minus = dict(base)
        plus[name] = base[name].clone()
        minus[name] = base[name].clone()
        plus[name].view(-1)[idx] += h
        minus[name].view(-1)[idx] -= h
        fd.append((loss(plus) - loss(minus)) / (2 * h))
        ad.append(float(grads[name].reshape(-1)[idx]))
    fd, ad = np.array(fd), np.array(ad)
    err = np.linalg.norm(ad - fd) / np.linalg.norm(fd)
    _flush(f"  FD agreement {err:.2e}")
    assert err <= 1e-5


def test_batched_forward_and_adjoint():
    """Batch of 4 right-hand sides sharing one operator, float32 V-cycle, forward + adjoint."""
    from paper_2002_00756_amd import Operator
    N, nz, L = 24, 30, 4
    _flush("batched forward+adjoint C24x30 B=4")
    kh, kv, delta = workloads.coefficients(N, nz, 1.0, 1000.0, True)
    b = workloads.rhs(N, nz, 4)
    g = workloads.loss_weights(N, nz, 4)
    dev = torch.device("cuda")
    op = Operator(N, nz, kh, kv, delta, L, precision="fp32", cg="flexible", max_batch=4,
                  device=dev)
    res = op.solve(torch.tensor(b, device=dev), rtol=1e-10)
    lam = op.solve(torch.tensor(g, device=dev), rtol=1e-10)
    gkh, gkv, gdl = op.face_grad(lam.x, res.x)
    levels, parents, childs = mesh.hierarchy(N, L)
    hier = helmholtz.Hierarchy(levels, parents, childs, kh, kv, delta)
    xs = np.stack([krylov.solve(hier, b[i], rtol=1e-12).x for i in range(4)])
    ls = np.stack([krylov.solve(hier, g[i], rtol=1e-12).x for i in range(4)])
    assert np.linalg.norm(res.x.cpu().numpy() - xs) <= 1e-8 * np.linalg.norm(xs)
    rkh, rkv, rdl = adjoint.face_gradients(levels[0], ls, xs)
    for a, r in ((gkh, rkh), (gkv, rkv), (gdl, rdl)):
        assert np.linalg.norm(a.cpu().numpy() - r) <= 1e-7 * np.linalg.norm(r)
