"""The allocation-free V-cycle (helmholtz_vcycle_noalloc) through the C ABI:
its level vectors live in the library's static scratch array, and its result
must equal helmholtz_vcycle's bit for bit (same kernels, same arithmetic).
Two calls in a row, the second on a smaller input, so that the second call
reuses the array left as the first one wrote it; then a handle too large for
the array is refused without a launch."""
import numpy as np
import pytest
import torch

import workloads

pytestmark = pytest.mark.gpu


def _op(N, nz, L, precision, batch):
    from paper_2002_00756_amd import Operator
    kh, kv, delta = workloads.coefficients(N, nz, 1.0, 1000.0, True)
    return Operator(N, nz, kh, kv, delta, L, precision=precision, max_batch=batch,
                    device="cuda")


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_noalloc_vcycle_matches_vcycle(precision):
    # first a larger input (C24 x 30, 4 levels, batch 3), then a smaller one
    # (C12 x 10, 3 levels, batch 1) in the same scratch; then C64 x 6, whose
    # residual restriction is the patch-staged kernel on scratch buffers
    for N, nz, L, batch, seed in ((24, 30, 4, 3, 21), (12, 10, 3, 1, 22), (64, 6, 3, 2, 23)):
        print(f"noalloc {precision} C{N}x{nz} L={L} batch={batch}", flush=True)
        op = _op(N, nz, L, precision, batch)
        b = torch.from_numpy(workloads.rhs(N, nz, batch, seed=seed)).cuda()
        ref = op.vcycle(b)
        out = torch.full_like(b, float("nan"))
        got = op.vcycle_noalloc(b, out=out)
        torch.cuda.synchronize()
        assert got.data_ptr() == out.data_ptr()
        assert torch.isfinite(got).all()
        assert torch.equal(got, ref), float((got - ref).abs().max())
        # and again with the scratch holding this call's own values
        again = op.vcycle_noalloc(b)
        assert torch.equal(again, ref)


def test_noalloc_vcycle_batch_members_and_bigger_batch_after_smaller():
    """A batch of 2 after a single right-hand side on the same handle: each
    member equals its own helmholtz_vcycle."""
    op = _op(16, 20, 3, "fp32", 2)
    b = torch.from_numpy(workloads.rhs(16, 20, 2, seed=23)).cuda()
    one = op.vcycle_noalloc(b[:1])
    two = op.vcycle_noalloc(b)
    torch.cuda.synchronize()
    assert torch.equal(one[0], op.vcycle(b[0]))
    assert torch.equal(two, op.vcycle(b))


def test_noalloc_vcycle_refuses_what_does_not_fit():
    from paper_2002_00756_amd import _lib
    # C96 x 30, 5 levels, float64: 50.6 MiB of level vectors at batch 1, 101 at batch 2
    op = _op(96, 30, 5, "fp64", 2)
    b = torch.from_numpy(workloads.rhs(96, 30, 2, seed=24)).cuda()
    x1 = op.vcycle_noalloc(b[:1])
    assert torch.equal(x1[0], op.vcycle(b[0]))
    out = torch.zeros_like(b)
    with pytest.raises(_lib.HelmholtzError) as err:
        op.vcycle_noalloc(b, out=out)
    assert err.value.code == _lib.ESCRATCH
    torch.cuda.synchronize()
    assert not out.any()  # nothing was launched
