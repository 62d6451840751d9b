"""Cubed-sphere column mesh and its horizontal 2x2 hierarchy (oracle).

TEST INFRASTRUCTURE ONLY (see the package header).

The paper runs on cubed-sphere meshes C<N> of 6 x N x N cells (Section 5.1)
and coarsens them horizontally only, each coarse cell being the union of 2x2
fine cells (Section 3.6). It reads both meshes and intergrid maps from files,
so the topology below is a reading: a canonical orientation written out in
integer geometry on the cube [0, 2N]^3.

Panel p has outward normal n, origin O and in-panel axes a ("E", index i) and
b ("N", index j). Cell (p, i, j) has its centre at O + (2i+1) a + (2j+1) b and
column index c = p N^2 + j N + i. Directions are numbered E=0, W=1, N=2, S=3.
A step that leaves the panel goes to the edge and then one unit down the
adjacent face, which is the panel whose normal is the step direction.
"""
from __future__ import annotations

import numpy as np

E, W, N_, S = 0, 1, 2, 3

# (normal, origin in units of M = 2N, axis a, axis b)
_PANELS = (
    ((1, 0, 0), (1, 0, 0), (0, 1, 0), (0, 0, 1)),
    ((0, 1, 0), (1, 1, 0), (-1, 0, 0), (0, 0, 1)),
    ((-1, 0, 0), (0, 1, 1), (0, 0, -1), (0, -1, 0)),
    ((0, -1, 0), (0, 0, 1), (0, 0, -1), (1, 0, 0)),
    ((0, 0, 1), (1, 1, 1), (-1, 0, 0), (0, -1, 0)),
    ((0, 0, -1), (0, 0, 0), (0, 1, 0), (1, 0, 0)),
)


def _panel(p, M):
    n, o, a, b = (np.array(v, dtype=np.int64) for v in _PANELS[p])
    return n, o * M, a, b


def cell_centre(N: int, p: int, i: int, j: int) -> np.ndarray:
    """Integer centre of cell (p, i, j) on the cube [0, 2N]^3."""
    _, o, a, b = _panel(p, 2 * N)
    return o + (2 * i + 1) * a + (2 * j + 1) * b


def column_index(N: int, p: int, i: int, j: int) -> int:
    return p * N * N + j * N + i


def neighbours(N: int) -> np.ndarray:
    """Horizontal neighbour table ``nbr[4][6N^2]`` (int32), directions E, W, N, S."""
    M = 2 * N
    ncol = 6 * N * N
    nbr = np.full((4, ncol), -1, dtype=np.int64)
    normals = [tuple(_PANELS[q][0]) for q in range(6)]
    jj, ii = np.meshgrid(np.arange(N), np.arange(N), indexing="ij")
    ii, jj = ii.ravel(), jj.ravel()          # in-panel order: c = j*N + i
    for p in range(6):
        n, o, a, b = _panel(p, M)
        cols = p * N * N + jj * N + ii
        centre = o[None, :] + (2 * ii + 1)[:, None] * a + (2 * jj + 1)[:, None] * b
        for d, (step, di, dj) in enumerate(((a, 1, 0), (-a, -1, 0),
                                            (b, 0, 1), (-b, 0, -1))):
            i2, j2 = ii + di, jj + dj
            inside = (i2 >= 0) & (i2 < N) & (j2 >= 0) & (j2 < N)
            nbr[d, cols[inside]] = p * N * N + j2[inside] * N + i2[inside]
            # leaving the panel: go to the edge, then one unit down the face
            # whose outward normal is the step direction
            q = normals.index(tuple(int(s) for s in step))
            _, oq, aq, bq = _panel(q, M)
            rel = centre[~inside] + step - n - oq
            ia, jb = rel @ aq, rel @ bq
            assert np.all(ia % 2 == 1) and np.all(jb % 2 == 1)
            nbr[d, cols[~inside]] = q * N * N + ((jb - 1) // 2) * N + (ia - 1) // 2
    assert (nbr >= 0).all()
    return nbr.astype(np.int32)


def face_table(N: int, nbr: np.ndarray | None = None) -> np.ndarray:
    """Face table ``ftab[4][6N^2]`` (int32): flat face index ``slot*ncol + owner``.

    Every horizontal face is stored once, as the E face (slot 0) or the N face
    (slot 1) of the cell that owns it. A cell's E and N faces are its own; its
    W or S face belongs to the neighbour on that side, in slot 0 if the cell
    is that neighbour's E neighbour and in slot 1 if it is its N neighbour.
    """
    if nbr is None:
        nbr = neighbours(N)
    ncol = nbr.shape[1]
    ftab = np.empty((4, ncol), dtype=np.int64)
    cols = np.arange(ncol)
    ftab[E] = cols
    ftab[N_] = ncol + cols
    for d in (W, S):
        other = nbr[d].astype(np.int64)
        is_e = nbr[E][other] == cols
        is_n = nbr[N_][other] == cols
        assert np.all(is_e ^ is_n), "face owned by neither or both"
        ftab[d] = np.where(is_e, other, ncol + other)
    return ftab.astype(np.int32)


def parent(N: int) -> np.ndarray:
    """Coarse column of each fine column: (p, i, j) -> (p, i >> 1, j >> 1) on C<N/2>."""
    assert N % 2 == 0
    Nc = N // 2
    c = np.arange(6 * N * N, dtype=np.int64)
    p, rem = c // (N * N), c % (N * N)
    j, i = rem // N, rem % N
    return (p * Nc * Nc + (j >> 1) * Nc + (i >> 1)).astype(np.int32)


def children(Nc: int) -> np.ndarray:
    """Fine children ``ch[4][6 Nc^2]`` of each coarse column on C<2 Nc>.

    Order: (di, dj) = (0,0), (1,0), (0,1), (1,1), i.e. fine (2I+di, 2J+dj).
    """
    Nf = 2 * Nc
    C = np.arange(6 * Nc * Nc, dtype=np.int64)
    p, rem = C // (Nc * Nc), C % (Nc * Nc)
    J, I = rem // Nc, rem % Nc
    ch = np.empty((4, C.size), dtype=np.int64)
    for s, (di, dj) in enumerate(((0, 0), (1, 0), (0, 1), (1, 1))):
        ch[s] = p * Nf * Nf + (2 * J + dj) * Nf + (2 * I + di)
    return ch.astype(np.int32)


class Level:
    """Tables of one multigrid level: C<N>, its neighbours and faces."""

    def __init__(self, N: int):
        self.N = N
        self.ncol = 6 * N * N
        self.nbr = neighbours(N)
        self.ftab = face_table(N, self.nbr)


def hierarchy(N: int, nlevels: int):
    """Levels l = 1..L with N_l = N / 2^(l-1) (Section 3.6); plus parent/children maps.

    Returns ``(levels, parents, childs)`` where ``parents[l]`` maps level l to
    level l+1 and ``childs[l]`` maps level l+1 back to level l (0-based lists).
    """
    if nlevels < 1 or N % (1 << (nlevels - 1)) != 0:
        raise ValueError("N must be divisible by 2^(L-1)")
    levels = [Level(N >> l) for l in range(nlevels)]
    parents = [parent(levels[l].N) for l in range(nlevels - 1)]
    childs = [children(levels[l + 1].N) for l in range(nlevels - 1)]
    return levels, parents, childs
