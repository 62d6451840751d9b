"""ctypes binding of ``libhelmholtz.so`` (the C ABI in include/helmholtz.h).

Argument marshalling only: every step of the computation runs in the HIP
library. If the library has not been built this module raises instead of
falling back to anything else.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libhelmholtz.so")

OK, NOT_CONVERGED = 0, 1
EINVAL, ESHAPE, EWORKSPACE, ENONFINITE, EHIP, ESCRATCH = -1, -2, -3, -4, -5, -6
FP64, FP32 = 0, 1
CG_STANDARD, CG_FLEXIBLE, BICGSTAB = 0, 1, 2
NZ_MAX = 120
WORKSPACE_ALIGN = 256
NOALLOC_SCRATCH_BYTES = 64 << 20

# Every function the header declares, with (restype, argtypes).
_c_int, _c_size, _vp, _dp = ctypes.c_int, ctypes.c_size_t, ctypes.c_void_p, ctypes.c_void_p
_i32p = ctypes.POINTER(ctypes.c_int32)
_f64p = ctypes.POINTER(ctypes.c_double)


class Config(ctypes.Structure):
    _fields_ = [("N", ctypes.c_int32), ("nz", ctypes.c_int32), ("nlevels", ctypes.c_int32),
                ("n_pre", ctypes.c_int32), ("n_post", ctypes.c_int32),
                ("n_coarse", ctypes.c_int32), ("omega", ctypes.c_double),
                ("mg_precision", ctypes.c_int32), ("cg_variant", ctypes.c_int32),
                ("max_batch", ctypes.c_int32), ("stencil", ctypes.c_int32),
                ("weighted", ctypes.c_int32)]


SIGNATURES = {
    "helmholtz_workspace_bytes": (_c_size, [ctypes.POINTER(Config)]),
    "helmholtz_create": (_c_int, [ctypes.POINTER(Config), _dp, _dp, _dp, _vp, _c_size, _vp,
                                  ctypes.POINTER(_vp)]),
    "helmholtz_create9": (_c_int, [ctypes.POINTER(Config), _dp, _dp, _dp, _dp, _vp, _c_size,
                                   _vp, ctypes.POINTER(_vp)]),
    "helmholtz_create_weighted": (_c_int, [ctypes.POINTER(Config), _dp, _dp, _dp, _dp, _vp,
                                           _c_size, _vp, ctypes.POINTER(_vp)]),
    "helmholtz_destroy": (_c_int, [_vp]),
    "helmholtz_update": (_c_int, [_vp, _dp, _dp, _dp, _dp, _dp, _vp]),
    "helmholtz_apply_adjoint": (_c_int, [_vp, _dp, _dp, ctypes.c_int32, _vp]),
    "helmholtz_vcycle_adjoint": (_c_int, [_vp, _dp, _dp, ctypes.c_int32, _vp]),
    "helmholtz_face_grad_weighted": (_c_int, [_vp, _dp, _dp, ctypes.c_int32, _dp, _dp, _dp, _dp,
                                              _vp]),
    "helmholtz_apply": (_c_int, [_vp, _dp, _dp, ctypes.c_int32, _vp]),
    "helmholtz_vcycle": (_c_int, [_vp, _dp, _dp, ctypes.c_int32, _vp]),
    "helmholtz_vcycle_f32": (_c_int, [_vp, _dp, _dp, ctypes.c_int32, _vp]),
    "helmholtz_vcycle_noalloc": (_c_int, [_vp, _dp, _dp, ctypes.c_int32, _vp]),
    "helmholtz_solve": (_c_int, [_vp, _dp, _dp, ctypes.c_int32, ctypes.c_double, ctypes.c_int32,
                                 _i32p, _f64p, _vp]),
    "helmholtz_solve_adjoint": (_c_int, [_vp, _dp, _dp, ctypes.c_int32, ctypes.c_double, ctypes.c_int32,
                                 _i32p, _f64p, _vp]),
    "helmholtz_face_grad": (_c_int, [_vp, _dp, _dp, ctypes.c_int32, _dp, _dp, _dp, _vp]),
    "helmholtz_face_grad9": (_c_int, [_vp, _dp, _dp, ctypes.c_int32, _dp, _dp, _dp, _dp, _vp]),
    "helmholtz_mesh_tables": (_c_int, [ctypes.c_int32, _i32p, _i32p, _i32p]),
    "helmholtz_strerror": (ctypes.c_char_p, [_c_int]),
    "helmholtz_profile_enable": (_c_int, [_vp, _c_int]),
    "helmholtz_profile_read": (_c_int, [_vp, ctypes.c_int32, _f64p,
                                        ctypes.POINTER(ctypes.c_int64), _f64p]),
    "helmholtz_bandwidth_kernel": (_c_int, [ctypes.c_int32, _vp, _vp, _vp, ctypes.c_int64,
                                            ctypes.c_float, _vp]),
}
PROF_SWEEP_FINE, PROF_APPLY_FINE, PROF_VCYCLE = 0, 1, 2
BW_READ, BW_WRITE, BW_COPY, BW_TRIAD = 0, 1, 2, 3

_lib = None


class HelmholtzError(RuntimeError):
    def __init__(self, code: int, where: str):
        self.code = code
        super().__init__(f"{where}: {strerror(code)} (code {code})")


def load():
    """Load the HIP library once; raise if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(
            f"{LIB_PATH} is missing: build it with `python -m paper_2002_00756_amd.build` "
            "(there is no fallback implementation)")
    lib = ctypes.CDLL(LIB_PATH)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def strerror(code: int) -> str:
    return load().helmholtz_strerror(code).decode()


def check(code: int, where: str, allow_not_converged: bool = False) -> int:
    if code == OK or (allow_not_converged and code == NOT_CONVERGED):
        return code
    raise HelmholtzError(code, where)
