"""Pins of the oracle's leaf ordering (tree construction, Section 3)."""
import os

import numpy as np
import pytest

from oracle import morton

GOLD = os.path.join(os.path.dirname(__file__), "golden", "morton_keys.txt")


def test_hand_worked_keys():
    rows = [list(map(int, l.split())) for l in open(GOLD) if l.strip() and not l.startswith("#")]
    for bits, bx, by, bz, key in rows:
        assert int(morton.interleave(bx, by, bz, bits)) == key


@pytest.mark.parametrize("n,ell", [(8, 2), (16, 4), (16, 2), (8, 8), (32, 8)])
def test_leaf_order_is_preorder_of_octree(n, ell):
    perm = morton.leaf_order(n, ell)
    assert np.array_equal(np.sort(perm), np.arange(n ** 3))
    i, j, k = np.unravel_index(perm, (n, n, n))
    s = ell ** 3
    # every run of ell^3 entries is one leaf block, in C order inside the leaf
    leaf = np.stack([i // ell, j // ell, k // ell], 1).reshape(-1, s, 3)
    assert np.all(leaf == leaf[:, :1, :])
    loc = ((i % ell) * ell + (j % ell)) * ell + (k % ell)
    assert np.array_equal(loc.reshape(-1, s), np.tile(np.arange(s), (leaf.shape[0], 1)))
    # pre-order: at every coarser level, runs of 8^m leaves form one box
    nb = n // ell
    lb = leaf[:, 0, :]
    level_size = 1
    while level_size < nb:
        level_size *= 2
        m = level_size ** 3
        boxes = (lb // level_size).reshape(-1, m, 3)
        assert np.all(boxes == boxes[:, :1, :])
    # children of a box are visited in octant order (x, y, z) = 000, 001, 010, ...
    if nb >= 2:
        first8 = lb[:8]
        assert [tuple(v) for v in first8] == [(a, b, c) for a in (0, 1) for b in (0, 1) for c in (0, 1)]


def test_column_order_hand_worked():
    # 2 x 2 x 4 cells, leaves of 1 x 1 x 1, so 2 cubes of 2^3 leaves along z: the first 8
    # positions are the cube z in {0, 1} in octant order (x, y, z) = 000, 001, 010, ...,
    # the next 8 the cube z in {2, 3}; grid index = (i * 2 + j) * 4 + k
    perm = morton.column_leaf_order(2, 4, 1, 1)
    first = [(i * 2 + j) * 4 + k for i in (0, 1) for j in (0, 1) for k in (0, 1)]
    second = [(i * 2 + j) * 4 + k + 2 for i in (0, 1) for j in (0, 1) for k in (0, 1)]
    assert perm.tolist() == first + second
    # leaves of 1 x 1 x 2 cells (ellz = 2): each leaf's two cells are consecutive along z
    perm = morton.column_leaf_order(2, 8, 1, 2)
    assert perm[:4].tolist() == [0, 1, 2, 3]          # leaf (0,0,0): cells k = 0, 1; leaf (0,0,1): k = 2, 3


@pytest.mark.parametrize("n,nz,ell,ellz", [(8, 24, 4, 4), (16, 40, 8, 2), (8, 8, 4, 4), (4, 20, 4, 4)])
def test_column_order_invariants(n, nz, ell, ellz):
    perm = morton.column_leaf_order(n, nz, ell, ellz)
    assert np.array_equal(np.sort(perm), np.arange(n * n * nz))
    i, j, k = np.unravel_index(perm, (n, n, nz))
    s = ell * ell * ellz
    leaf = np.stack([i // ell, j // ell, k // ellz], 1).reshape(-1, s, 3)
    assert np.all(leaf == leaf[:, :1, :])            # runs of s cells are one leaf
    lb = leaf[:, 0, :]
    nb = n // ell
    root = lb[:, 2] // nb
    assert np.all(np.diff(root) >= 0)                # cube after cube upwards
    # a cube is the Morton (octree pre-order) leaf order of a cube of side nb
    if nz == n and ellz == ell:
        assert np.array_equal(perm, morton.leaf_order(n, ell))
