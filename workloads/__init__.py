"""Seeded synthetic inputs for the cubed-sphere Helmholtz workloads.

This module is the only code shared by the oracle and the GPU library's tests
and benchmark. It draws random numbers and scales them; it holds none of the
solver's arithmetic (no mesh, no operator, no smoother, no Krylov step).

Shapes follow the paper's grids: a cubed-sphere mesh C<N> has 6*N*N vertical
columns and ``nz`` levels; the paper's C192 mesh is 6 x 192 x 192 cells
(Section 5.1). Its operators are not available, so a synthetic symmetric
positive definite face-coupling operator stands in for the Helmholtz operator
H of Section 3.4:

* one horizontal coupling per horizontal face, ``kh[2][nz][ncol]`` (slot 0 is
  the face a column owns on its E side, slot 1 the one on its N side), drawn as
  ``w_h * (1 + 0.1 u)`` with ``u ~ U[0, 1]``, one draw per face so the two
  cells that share it see the same value;
* one vertical coupling per interior vertical face, ``kv[nz-1][ncol]`` (face
  between levels k and k+1), ``w_v * g(k) * (1 + 0.1 u)`` with ``g = 1`` or
  the height grading ``g(k) = exp(-k / 20)``;
* a zero-order term ``delta[nz][ncol] ~ U[0.5, 1.5]``;
* for the 9-cell stencil of Section 3.5 (each cell also coupled to the cells
  two levels above and below), a next-to-nearest vertical coupling
  ``kv2[nz-2][ncol]`` (levels k and k+2), ``w_v2 * g(k) * (1 + 0.1 u)``,
  drawn from its own seed so the other draws do not change.

Vectors are ``[batch][nz][ncol]`` with the column index fastest.
"""
from __future__ import annotations

import dataclasses

import numpy as np

SEED_OP = 0
SEED_B = 1
SEED_G = 2
SEED_FD = 3
SEED_K2 = 4
SEED_S = 5


@dataclasses.dataclass(frozen=True)
class Workload:
    """One synthetic problem: mesh size, levels, coupling weights, hierarchy depth."""

    name: str
    N: int
    nz: int
    w_h: float
    w_v: float
    graded: bool
    nlevels: int
    batch: int = 1
    w_v2: float = 0.0   # > 0: 9-cell stencil with next-to-nearest vertical couplings

    @property
    def ncol(self) -> int:
        return 6 * self.N * self.N

    @property
    def n(self) -> int:
        return self.ncol * self.nz


# The configurations the paper's grids suggest (C192 is the paper's mesh,
# Section 5.1; C12, C96 and C384 bracket it; C6 x 8 is small enough for
# dense linear algebra).
C12x10 = Workload("C12x10", 12, 10, 1.0, 100.0, False, 3)
C96x30 = Workload("C96x30", 96, 30, 1.0, 1000.0, False, 5)
C192x70 = Workload("C192x70", 192, 70, 1.0, 1000.0, True, 6)
C384x70 = Workload("C384x70", 384, 70, 1.0, 1000.0, True, 7, batch=4)
C6x8 = Workload("C6x8", 6, 8, 1.0, 1000.0, False, 2)
# 9-cell stencil versions: next-to-nearest vertical couplings 1 % of the
# nearest ones (the paper's scalings put the term they come from, D_1^z, at
# N^2 dz / g ~ 2e-3 of D_2^z on its grid; 1e-2 exercises them a little harder)
C12x10_9 = Workload("C12x10_9", 12, 10, 1.0, 100.0, False, 3, w_v2=1.0)
C192x70_9 = Workload("C192x70_9", 192, 70, 1.0, 1000.0, True, 6, w_v2=10.0)

ALL = {w.name: w for w in (C12x10, C96x30, C192x70, C384x70, C6x8, C12x10_9, C192x70_9)}


def coefficients(N: int, nz: int, w_h: float = 1.0, w_v: float = 100.0,
                 graded: bool = False, seed: int = SEED_OP):
    """Return ``(kh, kv, delta)`` as float64 arrays for a C<N> x nz operator.

    Draw order is fixed: u for kh, then u for kv, then delta.
    """
    ncol = 6 * N * N
    rng = np.random.default_rng(seed)
    u_h = rng.random((2, nz, ncol))
    u_v = rng.random((max(nz - 1, 0), ncol))
    delta = rng.uniform(0.5, 1.5, size=(nz, ncol))
    kh = w_h * (1.0 + 0.1 * u_h)
    grade = np.ones(max(nz - 1, 0))
    if graded:
        grade = np.exp(-np.arange(max(nz - 1, 0), dtype=np.float64) / 20.0)
    kv = w_v * grade[:, None] * (1.0 + 0.1 * u_v)
    return kh, kv, delta


def workload_coefficients(w: Workload, seed: int = SEED_OP):
    return coefficients(w.N, w.nz, w.w_h, w.w_v, w.graded, seed)


def next_nearest(N: int, nz: int, w_v2: float, graded: bool = False, seed: int = SEED_K2):
    """``kv2[nz-2][ncol]``: coupling between levels k and k+2 (9-cell stencil)."""
    ncol = 6 * N * N
    m = max(nz - 2, 0)
    rng = np.random.default_rng(seed)
    u = rng.random((m, ncol))
    grade = np.ones(m)
    if graded:
        grade = np.exp(-np.arange(m, dtype=np.float64) / 20.0)
    return w_v2 * grade[:, None] * (1.0 + 0.1 * u)


def row_weights(N: int, nz: int, seed: int = SEED_S):
    """``s[nz][ncol] ~ U[0.5, 1.5]``: the per-cell row weight of the
    non-symmetric operator H = delta + diag(s) L (the role of 1/rho*)."""
    rng = np.random.default_rng(seed)
    return rng.uniform(0.5, 1.5, size=(nz, 6 * N * N))


def workload_kv2(w: Workload):
    """The workload's next-to-nearest couplings, or None for the 7-point stencil."""
    return next_nearest(w.N, w.nz, w.w_v2, w.graded) if w.w_v2 > 0 else None


def rhs(N: int, nz: int, batch: int = 1, seed: int = SEED_B) -> np.ndarray:
    """Right-hand sides ``b ~ N(0, 1)`` of shape ``[batch][nz][ncol]``."""
    rng = np.random.default_rng(seed)
    return rng.standard_normal((batch, nz, 6 * N * N))


def loss_weights(N: int, nz: int, batch: int = 1, seed: int = SEED_G) -> np.ndarray:
    """Weights ``g ~ N(0, 1)`` of the linear loss ``L = g . x``."""
    return rhs(N, nz, batch, seed)


def fd_sample(N: int, nz: int, count: int = 64, seed: int = SEED_FD):
    """Pick ``count`` coefficient entries for a finite-difference check.

    Returns a list of ``(array_name, flat_index)`` with array_name in
    ``{"kh", "kv", "delta"}``.
    """
    ncol = 6 * N * N
    sizes = {"kh": 2 * nz * ncol, "kv": max(nz - 1, 0) * ncol, "delta": nz * ncol}
    names = [k for k in ("kh", "kv", "delta") if sizes[k] > 0]
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(count):
        name = names[int(rng.integers(len(names)))]
        out.append((name, int(rng.integers(sizes[name]))))
    return out
