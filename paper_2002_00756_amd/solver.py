"""Python face of the HIP Helmholtz library: one operator hierarchy per object.

``Operator`` owns a torch workspace on the device and a library handle.
Its methods pass device pointers and the current HIP stream straight to the
C ABI; nothing is computed in Python.
"""
from __future__ import annotations

import ctypes
import dataclasses

import torch

from . import _lib


def mesh_tables(N: int):
    """Library-built mesh tables of C<N>: ``(nbr[4][6N^2], ftab[4][6N^2], parent[6N^2] or None)``."""
    import numpy as np
    lib = _lib.load()
    ncol = 6 * N * N
    nbr = np.empty((4, ncol), dtype=np.int32)
    ftab = np.empty((4, ncol), dtype=np.int32)
    par = np.empty(ncol, dtype=np.int32) if N % 2 == 0 else None
    ptr = lambda a: a.ctypes.data_as(_lib._i32p) if a is not None else None
    _lib.check(lib.helmholtz_mesh_tables(N, ptr(nbr), ptr(ftab), ptr(par)), "mesh_tables")
    return nbr, ftab, par


def _stream_ptr(device) -> int:
    return torch.cuda.current_stream(device).cuda_stream


def _dev(t: torch.Tensor, dtype, device, shape=None) -> torch.Tensor:
    if not isinstance(t, torch.Tensor):
        t = torch.as_tensor(t)
    t = t.to(device=device, dtype=dtype).contiguous()
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"expected shape {tuple(shape)}, got {tuple(t.shape)}")
    return t


@dataclasses.dataclass
class SolveResult:
    x: torch.Tensor
    iters: list
    relres: list
    converged: bool


class Operator:
    """Helmholtz operator hierarchy on one GPU.

    Parameters follow P_H^(MG)(L, omega, n_pre, n_post) with n_coarse sweeps on
    the coarsest level. ``precision`` is the V-cycle arithmetic ("fp64" or
    "fp32"); the Krylov loop is always float64. ``cg`` selects the Krylov
    method of ``solve``: conjugate gradients with the standard or flexible beta
    ("standard", "flexible"), or right-preconditioned BiCGStab ("bicgstab",
    where ``iters`` counts iterations of two products with H each). With
    ``nlevels=1`` the preconditioner is P_H^(Jac)(omega, n_coarse), and
    ``vcycle`` alone is the preconditioner-only solver PreOnly. ``kv2``
    (``[nz-2][ncol]``) selects the 9-cell stencil with couplings two levels
    apart; ``face_grad`` then also returns their gradient. ``s``
    (``[nz][ncol]``, > 0) selects the non-symmetric row-weighted operator
    H = delta + diag(s) L (needs ``cg="bicgstab"``); ``apply_adjoint``,
    ``vcycle_adjoint`` and ``solve_adjoint`` work with H^T, and ``face_grad``
    takes lam = H^-T g and also returns the gradient for ``s``.
    """

    _KRYLOV = {"standard": _lib.CG_STANDARD, "flexible": _lib.CG_FLEXIBLE,
               "bicgstab": _lib.BICGSTAB}

    @classmethod
    def _krylov(cls, cg):
        if cg not in cls._KRYLOV:
            raise ValueError(f"cg must be one of {sorted(cls._KRYLOV)}, not {cg!r}")
        return cls._KRYLOV[cg]

    def __init__(self, N, nz, kh, kv, delta, nlevels, n_pre=2, n_post=2, n_coarse=4,
                 omega=0.8, precision="fp64", cg="standard", max_batch=1, device="cuda",
                 kv2=None, s=None):
        self.lib = _lib.load()
        self.device = torch.device(device)
        if self.device.type == "cuda" and self.device.index is None:
            self.device = torch.device("cuda", torch.cuda.current_device())
        self.N, self.nz, self.nlevels = int(N), int(nz), int(nlevels)
        self.ncol = 6 * self.N * self.N
        self.precision = precision
        self.nine = kv2 is not None
        self.weighted = s is not None
        self.cfg = _lib.Config(self.N, self.nz, self.nlevels, n_pre, n_post, n_coarse,
                               float(omega), _lib.FP32 if precision == "fp32" else _lib.FP64,
                               self._krylov(cg), int(max_batch), 9 if self.nine else 7,
                               1 if self.weighted else 0)
        self.max_batch = int(max_batch)
        self.cg = cg
        nbytes = self.lib.helmholtz_workspace_bytes(ctypes.byref(self.cfg))
        if nbytes == 0:
            raise _lib.HelmholtzError(_lib.EINVAL if self.N % (1 << (self.nlevels - 1)) == 0
                                      else _lib.ESHAPE, "workspace_bytes")
        self.workspace_bytes = nbytes
        raw = torch.empty(nbytes + _lib.WORKSPACE_ALIGN, dtype=torch.uint8, device=self.device)
        off = (-raw.data_ptr()) % _lib.WORKSPACE_ALIGN
        self._raw = raw
        self._ws_ptr = raw.data_ptr() + off
        kh = _dev(kh, torch.float64, self.device, (2, self.nz, self.ncol))
        delta = _dev(delta, torch.float64, self.device, (self.nz, self.ncol))
        kv = _dev(kv, torch.float64, self.device, (self.nz - 1, self.ncol)) if self.nz > 1 else None
        if self.nine and self.nz > 2:
            kv2 = _dev(kv2, torch.float64, self.device, (self.nz - 2, self.ncol))
        else:
            kv2 = None
        handle = ctypes.c_void_p()
        kvp = kv.data_ptr() if kv is not None else None
        with torch.cuda.device(self.device):
            if self.weighted:
                s = _dev(s, torch.float64, self.device, (self.nz, self.ncol))
                code = self.lib.helmholtz_create_weighted(
                    ctypes.byref(self.cfg), kh.data_ptr(), kvp, delta.data_ptr(), s.data_ptr(),
                    self._ws_ptr, nbytes, _stream_ptr(self.device), ctypes.byref(handle))
            else:
                code = self.lib.helmholtz_create9(
                    ctypes.byref(self.cfg), kh.data_ptr(), kvp,
                    kv2.data_ptr() if kv2 is not None else None, delta.data_ptr(), self._ws_ptr,
                    nbytes, _stream_ptr(self.device), ctypes.byref(handle))
        _lib.check(code, "helmholtz_create")
        self._h = handle

    def update(self, kh, kv, delta, kv2=None, s=None):
        """Replace the operator's coefficients (same mesh, levels and options):
        the coefficient part of set-up only. ``kv2`` / ``s`` as at construction."""
        kh = _dev(kh, torch.float64, self.device, (2, self.nz, self.ncol))
        delta = _dev(delta, torch.float64, self.device, (self.nz, self.ncol))
        kv = _dev(kv, torch.float64, self.device, (self.nz - 1, self.ncol)) if self.nz > 1 else None
        if (kv2 is not None) != self.nine or (s is not None) != self.weighted:
            raise ValueError("update must pass kv2 / s exactly as the operator was built")
        kv2 = _dev(kv2, torch.float64, self.device, (self.nz - 2, self.ncol)) \
            if self.nine and self.nz > 2 else None
        s = _dev(s, torch.float64, self.device, (self.nz, self.ncol)) if self.weighted else None
        ptr = lambda t: t.data_ptr() if t is not None else None  # noqa: E731
        with torch.cuda.device(self.device):
            code = self.lib.helmholtz_update(self._h, kh.data_ptr(), ptr(kv), ptr(kv2),
                                             delta.data_ptr(), ptr(s), _stream_ptr(self.device))
        _lib.check(code, "helmholtz_update")

    def close(self):
        if getattr(self, "_h", None):
            self.lib.helmholtz_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- helpers -----------------------------------------------------------
    def _vec(self, v, dtype=torch.float64):
        v = _dev(v, dtype, self.device)
        squeeze = v.dim() == 2
        if squeeze:
            v = v.unsqueeze(0)
        if v.dim() != 3 or tuple(v.shape[1:]) != (self.nz, self.ncol):
            raise ValueError(f"vector must be [batch][{self.nz}][{self.ncol}], got {tuple(v.shape)}")
        if v.shape[0] > self.max_batch:
            raise ValueError(f"batch {v.shape[0]} exceeds max_batch {self.max_batch}")
        return v, squeeze

    # -- operations --------------------------------------------------------
    def apply(self, x, _fn="helmholtz_apply"):
        """y = H x (float64)."""
        x, sq = self._vec(x)
        y = torch.empty_like(x)
        _lib.check(getattr(self.lib, _fn)(self._h, x.data_ptr(), y.data_ptr(), x.shape[0],
                                          _stream_ptr(self.device)), _fn)
        return y[0] if sq else y

    def apply_adjoint(self, x):
        """y = H^T x (float64)."""
        return self.apply(x, "helmholtz_apply_adjoint")

    def vcycle(self, b, _fn="helmholtz_vcycle"):
        """x = M b, one V-cycle from zero in the operator's precision (float64 in and out)."""
        b, sq = self._vec(b)
        x = torch.empty_like(b)
        _lib.check(getattr(self.lib, _fn)(self._h, b.data_ptr(), x.data_ptr(), b.shape[0],
                                          _stream_ptr(self.device)), _fn)
        return x[0] if sq else x

    def vcycle_noalloc(self, b, out=None):
        """``vcycle`` with the level vectors in the library's static scratch array
        instead of the workspace (for callers that cannot allocate; calls on one
        GPU must not overlap). ``out`` receives x when given (then nothing is
        allocated here either)."""
        b, sq = self._vec(b)
        x = torch.empty_like(b) if out is None else out.view(b.shape)
        _lib.check(self.lib.helmholtz_vcycle_noalloc(self._h, b.data_ptr(), x.data_ptr(),
                                                     b.shape[0], _stream_ptr(self.device)),
                   "helmholtz_vcycle_noalloc")
        return x[0] if sq else x

    def vcycle_adjoint(self, b):
        """One V-cycle of the transposed hierarchy (the preconditioner of H^T)."""
        return self.vcycle(b, "helmholtz_vcycle_adjoint")

    def vcycle_f32(self, b):
        """x = M b entirely in float32."""
        b, sq = self._vec(b, torch.float32)
        x = torch.empty_like(b)
        _lib.check(self.lib.helmholtz_vcycle_f32(self._h, b.data_ptr(), x.data_ptr(), b.shape[0],
                                                 _stream_ptr(self.device)),
                   "helmholtz_vcycle_f32")
        return x[0] if sq else x

    def solve_adjoint(self, g, rtol=1e-8, maxiter=200, out=None) -> SolveResult:
        """Solve H^T lam = g (the adjoint solve)."""
        return self.solve(g, rtol, maxiter, out, _fn="helmholtz_solve_adjoint")

    def solve(self, b, rtol=1e-8, maxiter=200, out=None, _fn="helmholtz_solve") -> SolveResult:
        """Preconditioned Krylov solve (the handle's ``cg`` method) from x = 0; returns
        the solution and per-RHS statistics."""
        b, sq = self._vec(b)
        x = torch.empty_like(b) if out is None else out.view(b.shape)
        nb = b.shape[0]
        iters = (ctypes.c_int32 * nb)()
        rel = (ctypes.c_double * nb)()
        code = getattr(self.lib, _fn)(self._h, b.data_ptr(), x.data_ptr(), nb, float(rtol),
                                      int(maxiter), iters, rel, _stream_ptr(self.device))
        _lib.check(code, _fn, allow_not_converged=True)
        return SolveResult(x[0] if sq else x, list(iters), list(rel), code == _lib.OK)

    def profile(self, enable: bool = True):
        """Start (and reset) or stop the library's kernel timing hook."""
        _lib.check(self.lib.helmholtz_profile_enable(self._h, int(enable)), "profile_enable")

    def profile_read(self, kernel: int):
        """``(device ms, launches, algorithmic bytes)`` accumulated for one profiled kernel."""
        ms, n, by = ctypes.c_double(), ctypes.c_int64(), ctypes.c_double()
        _lib.check(self.lib.helmholtz_profile_read(self._h, kernel, ctypes.byref(ms),
                                                   ctypes.byref(n), ctypes.byref(by)),
                   "profile_read")
        return ms.value, n.value, by.value

    def face_grad(self, lam, x):
        """Coefficient gradients of L = g . x given lam = H^-1 g, summed over the batch:
        ``(g_kh, g_kv, g_delta)``, plus ``g_kv2`` last for the 9-cell stencil."""
        lam, _ = self._vec(lam)
        x, _ = self._vec(x)
        gkh = torch.empty((2, self.nz, self.ncol), dtype=torch.float64, device=self.device)
        gkv = torch.empty((max(self.nz - 1, 0), self.ncol), dtype=torch.float64,
                          device=self.device)
        gdl = torch.empty((self.nz, self.ncol), dtype=torch.float64, device=self.device)
        gkv2 = torch.empty((max(self.nz - 2, 0), self.ncol), dtype=torch.float64,
                           device=self.device) if self.nine else None
        if self.weighted:
            gs = torch.empty((self.nz, self.ncol), dtype=torch.float64, device=self.device)
            _lib.check(self.lib.helmholtz_face_grad_weighted(
                self._h, lam.data_ptr(), x.data_ptr(), lam.shape[0], gkh.data_ptr(),
                gkv.data_ptr() if self.nz > 1 else None, gdl.data_ptr(), gs.data_ptr(),
                _stream_ptr(self.device)), "helmholtz_face_grad_weighted")
            return gkh, gkv, gdl, gs
        _lib.check(self.lib.helmholtz_face_grad9(
            self._h, lam.data_ptr(), x.data_ptr(), lam.shape[0], gkh.data_ptr(),
            gkv.data_ptr() if self.nz > 1 else None,
            gkv2.data_ptr() if gkv2 is not None and self.nz > 2 else None, gdl.data_ptr(),
            _stream_ptr(self.device)), "helmholtz_face_grad")
        if self.nine:
            return gkh, gkv, gdl, gkv2
        return gkh, gkv, gdl
