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
    """C96 x 30: the gradient from the autograd Function's backward (adjoint
    solve + fused face gradients) against central differences of L = g . x on
    64 sampled coefficients, h = 1e-6, every solve converged to 1e-14 (the
    differences re-solve on one operator whose coefficients are replaced).

    Agreement ||g_adj - g_fd|| / ||g_fd|| <= 1e-5 over the sample.
    """
    from paper_2002_00756_amd import Operator, helmholtz_solve
    w = workloads.C96x30
    _flush(f"FD C96x30 {precision}")
    kh, kv, delta = workloads.workload_coefficients(w)
    b = workloads.rhs(w.N, w.nz)[0]
    g = workloads.loss_weights(w.N, w.nz)[0]
    dev = torch.device("cuda")
    tb, tg = torch.tensor(b, device=dev), torch.tensor(g, device=dev)
    cg = "flexible" if precision == "fp32" else "standard"
    rtol = 1e-14

    base = {"kh": torch.tensor(kh, device=dev), "kv": torch.tensor(kv, device=dev),
            "delta": torch.tensor(delta, device=dev)}
    leaves = {k: v.clone().requires_grad_(True) for k, v in base.items()}
    x = helmholtz_solve(tb, leaves["kh"], leaves["kv"], leaves["delta"], N=w.N, nz=w.nz,
                        nlevels=w.nlevels, precision=precision, cg=cg, rtol=rtol, maxiter=100)
    (tg * x).sum().backward()
    grads = {k: v.grad for k, v in leaves.items()}

    op = Operator(w.N, w.nz, kh, kv, delta, w.nlevels, precision=precision, cg=cg, device=dev)

    def loss(arrs):
        op.update(arrs["kh"], arrs["kv"], arrs["delta"])
        res = op.solve(tb, rtol=rtol, maxiter=100)
        assert res.converged, res.relres
        return float(torch.dot(tg.flatten(), res.x.flatten()))

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


def _dense_weighted(lev, kh, kv, delta, s=None, kv2=None):
    return helmholtz.assemble(lev, kh, kv, delta, kv2=kv2, s=s).toarray()


@pytest.mark.parametrize("form", ["nine_cell", "weighted"])
def test_autograd_nine_cell_and_weighted_dense_c6x8(form):
    """The differentiable solve of the 9-cell operator (CG) and of the
    row-weighted one (BiCGStab; the backward solves with H^T) on C6 x 8, 2
    levels, batch of 2: x, dL/db and every coefficient gradient against dense
    linear algebra."""
    from paper_2002_00756_amd import helmholtz_solve
    w = workloads.C6x8
    _flush(f"autograd dense C6x8 {form}")
    kh, kv, delta = workloads.workload_coefficients(w)
    kv2 = workloads.next_nearest(w.N, w.nz, 10.0) if form == "nine_cell" else None
    sw = workloads.row_weights(w.N, w.nz) if form == "weighted" else None
    b = workloads.rhs(w.N, w.nz, 2)
    g = workloads.loss_weights(w.N, w.nz, 2)
    dev = torch.device("cuda")
    leaf = lambda a: None if a is None else torch.tensor(a, device=dev, requires_grad=True)  # noqa
    tb, tkh, tkv, tdl, tkv2, ts = (leaf(a) for a in (b, kh, kv, delta, kv2, sw))
    kw = dict(cg="bicgstab") if form == "weighted" else {}
    x = helmholtz_solve(tb, tkh, tkv, tdl, kv2=tkv2, s=ts, N=w.N, nz=w.nz, nlevels=w.nlevels,
                        rtol=1e-13, max_batch=2, **kw)
    (torch.tensor(g, device=dev) * x).sum().backward()

    lev = mesh.Level(w.N)
    H = _dense_weighted(lev, kh, kv, delta, s=sw, kv2=kv2)
    xs = np.linalg.solve(H, b.reshape(2, -1).T).T.reshape(b.shape)
    lam = np.linalg.solve(H.T, g.reshape(2, -1).T).T.reshape(g.shape)
    if form == "weighted":
        refs = dict(zip(("kh", "kv", "delta", "s"),
                        adjoint.weighted_gradients(lev, kh, kv, sw, lam, xs)))
    else:
        refs = dict(zip(("kh", "kv", "delta"), adjoint.face_gradients(lev, lam, xs)))
        refs["kv2"] = adjoint.kv2_gradient(lam, xs)

    def rel(a, r):
        return float(np.linalg.norm(a.detach().cpu().numpy() - r) / np.linalg.norm(r))
    assert rel(x, xs) <= 1e-10
    assert rel(tb.grad, lam) <= 1e-10
    got = {"kh": tkh.grad, "kv": tkv.grad, "delta": tdl.grad}
    if tkv2 is not None:
        got["kv2"] = tkv2.grad
    if ts is not None:
        got["s"] = ts.grad
    assert set(got) == set(refs)
    for k in refs:
        assert rel(got[k], refs[k]) <= 1e-9, (k, rel(got[k], refs[k]))


@pytest.mark.parametrize("form", ["nine_cell", "weighted"])
def test_autograd_nine_cell_and_weighted_central_differences(form):
    """C12 x 10, 3 levels: the autograd gradients of the 9-cell operator's
    kv2 (and the other couplings) and of the row weight s against central
    differences (h = 1e-6, 32 sampled coefficients, solves converged)."""
    from paper_2002_00756_amd import Operator, helmholtz_solve
    N, nz, L = 12, 10, 3
    _flush(f"FD C12x10 {form}")
    kh, kv, delta = workloads.coefficients(N, nz, 1.0, 100.0, False)
    arrs = {"kh": kh, "kv": kv, "delta": delta}
    if form == "nine_cell":
        arrs["kv2"] = workloads.next_nearest(N, nz, 1.0)
        kw, rtol = {}, 1e-14
    else:
        arrs["s"] = workloads.row_weights(N, nz)
        kw, rtol = {"cg": "bicgstab"}, 1e-13
    dev = torch.device("cuda")
    b = torch.tensor(workloads.rhs(N, nz)[0], device=dev)
    g = torch.tensor(workloads.loss_weights(N, nz)[0], device=dev)
    base = {k: torch.tensor(v, device=dev) for k, v in arrs.items()}
    leaves = {k: v.clone().requires_grad_(True) for k, v in base.items()}
    x = helmholtz_solve(b, leaves["kh"], leaves["kv"], leaves["delta"], kv2=leaves.get("kv2"),
                        s=leaves.get("s"), N=N, nz=nz, nlevels=L, rtol=rtol, maxiter=200, **kw)
    (g * x).sum().backward()
    op = Operator(N, nz, kh, kv, delta, L, device=dev, kv2=arrs.get("kv2"), s=arrs.get("s"),
                  **kw)

    def loss(a):
        op.update(a["kh"], a["kv"], a["delta"], kv2=a.get("kv2"), s=a.get("s"))
        res = op.solve(b, rtol=rtol, maxiter=200)
        assert res.converged, res.relres
        return float(torch.dot(g.flatten(), res.x.flatten()))

    rng = np.random.default_rng(33)
    names = sorted(base)
    h = 1e-6
    fd, ad = [], []
    for _ in range(32):
        name = names[int(rng.integers(len(names)))]
        idx = int(rng.integers(base[name].numel()))
        plus, minus = dict(base), dict(base)
        plus[name], minus[name] = base[name].clone(), base[name].clone()
        plus[name].view(-1)[idx] += h
        minus[name].view(-1)[idx] -= h
        fd.append((loss(plus) - loss(minus)) / (2 * h))
        ad.append(float(leaves[name].grad.reshape(-1)[idx]))
    fd, ad = np.array(fd), np.array(ad)
    err = np.linalg.norm(ad - fd) / np.linalg.norm(fd)
    _flush(f"  FD agreement {err:.2e}")
    assert err <= 1e-5


def test_autograd_raises_when_a_solve_does_not_converge():
    """maxiter = 1 with a tight rtol: the forward solve raises; with b = 0 the
    forward needs no iteration and the adjoint solve raises in backward."""
    from paper_2002_00756_amd import HelmholtzNotConverged, helmholtz_solve
    N, nz, L = 8, 6, 3
    kh, kv, delta = (torch.tensor(a, device="cuda", requires_grad=True)
                     for a in workloads.coefficients(N, nz))
    b = torch.tensor(workloads.rhs(N, nz)[0], device="cuda")
    with pytest.raises(HelmholtzNotConverged):
        helmholtz_solve(b, kh, kv, delta, N=N, nz=nz, nlevels=L, rtol=1e-14, maxiter=1)
    x = helmholtz_solve(torch.zeros_like(b), kh, kv, delta, N=N, nz=nz, nlevels=L, rtol=1e-14,
                        maxiter=1)
    assert not x.any()
    g = torch.tensor(workloads.loss_weights(N, nz)[0], device="cuda")
    with pytest.raises(HelmholtzNotConverged):
        (g * x).sum().backward()


def test_autograd_reuses_its_operator_with_new_coefficients():
    """A forward keeps its operator while its output's autograd node lives; a
    later forward with the same shape and options takes the operator given
    back (its coefficients replaced by helmholtz_update) and still matches a
    freshly built operator's solve and gradients."""
    import gc

    import paper_2002_00756_amd.autograd as ag
    from paper_2002_00756_amd import Operator, helmholtz_solve
    N, nz, L = 12, 10, 3
    ag.clear_operator_pool()
    dev = torch.device("cuda")
    b = torch.tensor(workloads.rhs(N, nz)[0], device=dev)
    g = torch.tensor(workloads.loss_weights(N, nz)[0], device=dev)
    c1 = [torch.tensor(a, device=dev, requires_grad=True)
          for a in workloads.coefficients(N, nz, 1.0, 100.0)]
    c2 = [torch.tensor(a, device=dev, requires_grad=True)
          for a in workloads.coefficients(N, nz, 2.0, 50.0, seed=7)]
    x1 = helmholtz_solve(b, *c1, N=N, nz=nz, nlevels=L, rtol=1e-12)
    assert not any(ag._pool.values())        # held by x1's node
    del x1
    gc.collect()
    (key, idle), = ag._pool.items()
    op1 = idle[-1]
    x2 = helmholtz_solve(b, *c2, N=N, nz=nz, nlevels=L, rtol=1e-12)
    assert op1 not in ag._pool[key]           # taken again, now held by x2's node
    (g * x2).sum().backward()
    fresh = Operator(N, nz, *(c.detach() for c in c2), L, device=dev)
    xf = fresh.solve(b, rtol=1e-12).x
    lam = fresh.solve(g, rtol=1e-12).x
    rkh, rkv, rdl = fresh.face_grad(lam, xf)
    scale = float(xf.abs().max())
    assert torch.allclose(x2, xf, rtol=0, atol=1e-10 * scale)
    for got, ref in ((c2[0].grad, rkh), (c2[1].grad, rkv), (c2[2].grad, rdl)):
        assert torch.allclose(got, ref, rtol=0, atol=1e-9 * float(ref.abs().max()))
    del x2
    gc.collect()
    assert op1 in ag._pool[key]


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
