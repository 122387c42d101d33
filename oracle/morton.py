"""Morton (Z-order) leaf ordering of a uniform grid (oracle; tests only).

Section 3 builds the octree by splitting a root cube into eight equal sub-cubes
until a box holds at most m points (tree construction step of the algorithm
outline).  On an n^3 grid with n a power of two and leaves of ell^3 cells, every
leaf is an ell^3 block and the pre-order of the complete octree visits leaves in
Morton order: the key of block (bx, by, bz) interleaves their bits as
... x1 y1 z1 x0 y0 z0 (x the most significant of each triple), and the pre-order
visits children in that octant order.

This module writes out that definition with a plain bit loop and a sort.
"""
import numpy as np


def interleave(bx, by, bz, bits):
    """Morton key of integer box coordinates with `bits` bits per axis (bit loop)."""
    bx = np.asarray(bx, dtype=np.int64)
    by = np.asarray(by, dtype=np.int64)
    bz = np.asarray(bz, dtype=np.int64)
    key = np.zeros(np.broadcast(bx, by, bz).shape, dtype=np.int64)
    for bit in range(bits):
        key |= ((bx >> bit) & 1) << (3 * bit + 2)
        key |= ((by >> bit) & 1) << (3 * bit + 1)
        key |= ((bz >> bit) & 1) << (3 * bit + 0)
    return key


def leaf_order(n, ell):
    """Flat grid indices of all cells listed leaf by leaf.

    Returns perm of length n^3: position p of the leaf-ordered array holds the cell
    perm[p] of the C-order grid.  Leaves follow increasing Morton key; inside a
    leaf the ell^3 cells follow C order (x slowest, z fastest).
    """
    nb = n // ell
    bits = int(np.log2(nb)) if nb > 1 else 0
    i, j, k = np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij")
    i, j, k = i.ravel(), j.ravel(), k.ravel()
    leaf_key = interleave(i // ell, j // ell, k // ell, bits)
    local = ((i % ell) * ell + (j % ell)) * ell + (k % ell)
    order = np.lexsort((local, leaf_key))   # sort by leaf key, then local index
    return order.astype(np.int64)


def column_leaf_order(n, nz, ell, ellz):
    """Leaf order of a box of n x n x nz cells cut into leaves of ell x ell x ellz cells,
    the leaves forming a column of R = nz / (ellz * n / ell) cubes of (n / ell)^3 leaves
    stacked along z, each cube a complete octree visited in pre-order (Morton order of the
    leaf coordinates inside the cube), cube after cube from z = 0 upwards; inside a leaf
    the cells follow C order.  Returns perm of length n * n * nz (position p of the
    leaf-ordered array holds the cell perm[p] of the C-order grid)."""
    nb = n // ell
    assert nb * ell == n and nz % (ellz * nb) == 0
    bits = int(np.log2(nb)) if nb > 1 else 0
    i, j, k = np.meshgrid(np.arange(n), np.arange(n), np.arange(nz), indexing="ij")
    i, j, k = i.ravel(), j.ravel(), k.ravel()
    lz = k // ellz                      # leaf z in the column
    root = lz // nb
    key = interleave(i // ell, j // ell, lz % nb, bits)
    local = ((i % ell) * ell + (j % ell)) * ellz + (k % ellz)
    order = np.lexsort((local, key, root))   # by cube, then Morton key, then local index
    return order.astype(np.int64)
