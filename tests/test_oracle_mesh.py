"""Pins of the oracle's cubed-sphere mesh and hierarchy against geometry and brute force."""
import os

import numpy as np
import pytest

from oracle import mesh

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _centres(N):
    out = np.empty((6 * N * N, 3), dtype=np.int64)
    for p in range(6):
        for j in range(N):
            for i in range(N):
                out[mesh.column_index(N, p, i, j)] = mesh.cell_centre(N, p, i, j)
    return out


def test_c1_matches_hand_derived_table():
    rows = [l.split() for l in open(os.path.join(GOLDEN, "c1_neighbours.txt"))
            if l.strip() and not l.startswith("#")]
    expect = np.array([[int(v) for v in r[1:]] for r in rows]).T
    assert np.array_equal(mesh.neighbours(1), expect)
    # never the opposite face
    opposite = {0: 2, 2: 0, 1: 3, 3: 1, 4: 5, 5: 4}
    nb = mesh.neighbours(1)
    for c in range(6):
        assert opposite[c] not in nb[:, c]


@pytest.mark.parametrize("N", [2, 3, 4, 5])
def test_neighbours_are_the_four_nearest_cells_brute_force(N):
    """Independent of the stepping rule: the 4 nearest cell centres in 3-D.

    In doubled units a same-panel neighbour is at squared distance 4, one
    across a cube edge at 2, and every other cell at 6 or more (N >= 2; on C1
    the opposite face is also at 4, and the hand-derived table covers it).
    """
    cen = _centres(N)
    d2 = ((cen[:, None, :] - cen[None, :, :]) ** 2).sum(-1)
    nb = mesh.neighbours(N)
    for c in range(cen.shape[0]):
        near = set(np.nonzero((d2[c] > 0) & (d2[c] <= 4))[0].tolist())
        assert near == set(nb[:, c].tolist())
        others = np.delete(d2[c], list(near) + [c])
        assert others.min() >= 6


@pytest.mark.parametrize("N", [1, 2, 3, 6, 8])
def test_neighbour_table_invariants(N):
    nb = mesh.neighbours(N)
    ncol = 6 * N * N
    cols = np.arange(ncol)
    for c in range(ncol):
        assert len(set(nb[:, c].tolist())) == 4 and c not in nb[:, c]
    # symmetric: each neighbour lists c back exactly once
    for d in range(4):
        back = (nb[:, nb[d]] == cols).sum(axis=0)
        assert np.all(back == 1)
    # within a panel the direction is the grid direction
    p, rem = cols // (N * N), cols % (N * N)
    j, i = rem // N, rem % N
    inner = i < N - 1
    assert np.all(nb[mesh.E][inner] == cols[inner] + 1)
    inner = j < N - 1
    assert np.all(nb[mesh.N_][inner] == cols[inner] + N)


@pytest.mark.parametrize("N", [1, 2, 3, 4, 7])
def test_every_face_owned_once(N):
    """Each of the 12 N^2 faces is the E or N face of exactly one of its two cells."""
    nb = mesh.neighbours(N)
    ft = mesh.face_table(N, nb)
    ncol = 6 * N * N
    pairs = {}
    for c in range(ncol):
        for d in range(4):
            key = frozenset((c, int(nb[d, c])))
            pairs.setdefault(key, set()).add(int(ft[d, c]))
    assert len(pairs) == 12 * N * N
    for faces in pairs.values():
        assert len(faces) == 1      # both cells name the same stored face
    stored = sorted(f for faces in pairs.values() for f in faces)
    assert stored == list(range(2 * ncol))


@pytest.mark.parametrize("N", [2, 4, 6, 12])
def test_parent_children_and_nesting(N):
    par = mesh.parent(N)
    ch = mesh.children(N // 2)
    Nc = N // 2
    assert np.all(par[ch] == np.arange(6 * Nc * Nc)[None, :])
    assert sorted(ch.ravel().tolist()) == list(range(6 * N * N))
    nbf, nbc = mesh.neighbours(N), mesh.neighbours(Nc)
    # nesting: fine neighbours have the same parent or neighbouring parents,
    # also across panel edges
    for d in range(4):
        pc, pn = par, par[nbf[d]]
        same = pc == pn
        assert np.all(same | (nbc[:, pc] == pn).any(axis=0))
    # a coarse face is made of exactly two fine faces
    for C in range(6 * Nc * Nc):
        for D in nbc[:, C]:
            kids_c, kids_d = set(ch[:, C].tolist()), set(ch[:, D].tolist())
            crossing = sum(1 for c in kids_c for d in range(4) if nbf[d, c] in kids_d)
            assert crossing == 2


def test_hierarchy_rejects_indivisible():
    with pytest.raises(ValueError):
        mesh.hierarchy(6, 3)     # 6 is not divisible by 4
    levels, parents, childs = mesh.hierarchy(12, 3)
    assert [l.N for l in levels] == [12, 6, 3]
