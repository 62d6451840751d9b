"""Host-only checks of the C ABI: the library loads, exports what the header
declares, sizes its workspace, rejects bad input before touching the GPU, and
builds mesh tables bit-identical to the oracle's."""
import ctypes
import os
import re

import numpy as np
import pytest

from oracle import mesh as omesh

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def lib():
    from paper_2002_00756_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        from paper_2002_00756_amd import build
        build.build()
    return _lib.load()


def _declared_functions():
    text = open(os.path.join(ROOT, "include", "helmholtz.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(helmholtz_[a-z0-9_]+)\s*\(", text)))


def test_every_declared_symbol_is_exported(lib):
    from paper_2002_00756_amd import _lib
    names = _declared_functions()
    assert len(names) == 22
    for n in names:
        assert hasattr(lib, n), n
        assert n in _lib.SIGNATURES, n


def _cfg(N=12, nz=10, L=3, **kw):
    from paper_2002_00756_amd import _lib
    d = dict(n_pre=2, n_post=2, n_coarse=4, omega=0.8, mg_precision=0, cg_variant=0, max_batch=1,
             stencil=7, weighted=0)
    d.update(kw)
    return _lib.Config(N, nz, L, d["n_pre"], d["n_post"], d["n_coarse"], d["omega"],
                       d["mg_precision"], d["cg_variant"], d["max_batch"], d["stencil"],
                       d["weighted"])


def test_workspace_bytes(lib):
    small = lib.helmholtz_workspace_bytes(ctypes.byref(_cfg()))
    big = lib.helmholtz_workspace_bytes(ctypes.byref(_cfg(max_batch=4)))
    assert 0 < small < big
    # C192 x 70 with 6 levels: per level 6 float64 + 6 float32 coefficient words, ...
    c192 = lib.helmholtz_workspace_bytes(ctypes.byref(_cfg(192, 70, 6)))
    n = 6 * 192 * 192 * 70
    assert 72 * n < c192 < 200 * n
    for bad in (_cfg(12, 10, 4),            # 12 not divisible by 8
                _cfg(12, 0, 1), _cfg(12, 121, 1), _cfg(12, 10, 3, n_coarse=0),
                _cfg(12, 10, 3, omega=0.0), _cfg(12, 10, 3, max_batch=0),
                _cfg(12, 10, 3, mg_precision=2)):
        assert lib.helmholtz_workspace_bytes(ctypes.byref(bad)) == 0


def test_create_rejects_before_touching_the_device(lib):
    from paper_2002_00756_amd import _lib
    h = ctypes.c_void_p()
    dummy = ctypes.c_void_p(256)
    assert lib.helmholtz_create(ctypes.byref(_cfg(12, 10, 4)), dummy, dummy, dummy, dummy,
                                1 << 30, None, ctypes.byref(h)) == _lib.ESHAPE
    assert lib.helmholtz_create(ctypes.byref(_cfg(omega=2.0)), dummy, dummy, dummy, dummy,
                                1 << 30, None, ctypes.byref(h)) == _lib.EINVAL
    assert lib.helmholtz_create(ctypes.byref(_cfg()), dummy, dummy, dummy, None,
                                1 << 30, None, ctypes.byref(h)) == _lib.EWORKSPACE
    assert lib.helmholtz_create(ctypes.byref(_cfg()), dummy, dummy, dummy, ctypes.c_void_p(4096),
                                16, None, ctypes.byref(h)) == _lib.EWORKSPACE
    assert lib.helmholtz_create(ctypes.byref(_cfg()), dummy, dummy, dummy,
                                ctypes.c_void_p(4096 + 8), 1 << 40, None,
                                ctypes.byref(h)) == _lib.EWORKSPACE
    assert lib.helmholtz_create(ctypes.byref(_cfg()), None, dummy, dummy, dummy,
                                1 << 30, None, ctypes.byref(h)) == _lib.EINVAL
    # 9-cell stencil: only through helmholtz_create9, and only with kv2 (nz > 2)
    assert lib.helmholtz_create(ctypes.byref(_cfg(stencil=9)), dummy, dummy, dummy, dummy,
                                1 << 30, None, ctypes.byref(h)) == _lib.EINVAL
    assert lib.helmholtz_create9(ctypes.byref(_cfg(stencil=9)), dummy, dummy, None, dummy,
                                 dummy, 1 << 30, None, ctypes.byref(h)) == _lib.EINVAL
    assert lib.helmholtz_create9(ctypes.byref(_cfg(stencil=7)), dummy, dummy, dummy, dummy,
                                 dummy, 1 << 30, None, ctypes.byref(h)) == _lib.EINVAL
    assert lib.helmholtz_workspace_bytes(ctypes.byref(_cfg(stencil=8))) == 0
    # weighted operator: BiCGStab and the 7-point stencil only, through its own create
    assert lib.helmholtz_workspace_bytes(ctypes.byref(_cfg(weighted=1))) == 0
    assert lib.helmholtz_workspace_bytes(ctypes.byref(_cfg(weighted=1, cg_variant=2,
                                                            stencil=9))) == 0
    assert lib.helmholtz_workspace_bytes(ctypes.byref(_cfg(weighted=1, cg_variant=2))) > 0
    assert lib.helmholtz_create(ctypes.byref(_cfg(weighted=1, cg_variant=2)), dummy, dummy,
                                dummy, dummy, 1 << 30, None, ctypes.byref(h)) == _lib.EINVAL
    assert lib.helmholtz_create_weighted(ctypes.byref(_cfg(weighted=1, cg_variant=2)), dummy,
                                         dummy, dummy, None, dummy, 1 << 30, None,
                                         ctypes.byref(h)) == _lib.EINVAL
    assert lib.helmholtz_workspace_bytes(ctypes.byref(_cfg(stencil=9))) > \
        lib.helmholtz_workspace_bytes(ctypes.byref(_cfg(stencil=7)))
    assert not h.value
    for fn in ("helmholtz_apply", "helmholtz_vcycle", "helmholtz_vcycle_f32",
               "helmholtz_vcycle_noalloc"):
        assert getattr(lib, fn)(None, dummy, dummy, 1, None) == _lib.EINVAL
    assert lib.helmholtz_destroy(None) == _lib.EINVAL


def test_strerror(lib):
    for code in (0, 1, -1, -2, -3, -4, -5, -6, 99):
        assert isinstance(lib.helmholtz_strerror(code), bytes)


@pytest.mark.parametrize("N", [1, 2, 3, 6, 12, 48, 96, 192, 384])
def test_mesh_tables_bit_exact(lib, N):
    from paper_2002_00756_amd.solver import mesh_tables
    nbr, ftab, par = mesh_tables(N)
    ref_nbr = omesh.neighbours(N)
    assert np.array_equal(nbr, ref_nbr)
    assert np.array_equal(ftab, omesh.face_table(N, ref_nbr))
    if N % 2 == 0:
        assert np.array_equal(par, omesh.parent(N))
    else:
        assert par is None


def test_bench_byte_model():
    """The V-cycle byte model of the benchmark, counted by hand for 2/2 sweeps:
    per level 4 (first sweep) + 7 + 6.25 (residual + restriction) + 7.25
    (sweep with prolongation) + 7 = 31.5 words, coarsest 4 + 3 * 7 = 25."""
    import bench
    assert bench.vcycle_words(1, 2, 2, 4) == 25.0
    assert bench.vcycle_words(2, 2, 2, 4) == 31.5 + 25.0 / 4
    L6 = 31.5 * sum(4.0 ** -l for l in range(5)) + 25.0 / 4 ** 5
    assert abs(bench.vcycle_words(6, 2, 2, 4) - L6) < 1e-12
    # one CG iteration: apply+dot 48, residual update 28 (mixed: r, q read; r,
    # r32 written) / 24, dot 12 / 16, p and x update 36 / 40 (z, p, x read;
    # p, x written)
    assert bench.cg_bytes_per_unknown(0.0, True, False) == 48 + 28 + 12 + 36
    assert bench.cg_bytes_per_unknown(0.0, False, False) == 48 + 24 + 16 + 40


def test_bench_bicgstab_byte_model():
    """BiCGStab iteration bytes, counted by hand: per preconditioner application
    a float32 V-cycle of w words (4w bytes) plus its two conversions (12 B
    each way), per apply 48 B plus the 8 B dot partner; updates p 32, s 24,
    x/r 64."""
    import bench
    w = 41.0
    assert bench.bicgstab_bytes_per_unknown(w, True) == 2 * (4 * w + 24 + 56) + 32 + 24 + 64
    assert bench.bicgstab_bytes_per_unknown(w, False) == 2 * (8 * w + 56) + 32 + 24 + 64
