"""Box-shaped grids evaluated inside a cube.

The tree needs an n^3 grid with n a power of two.  A box-shaped grid of isotropic
cells (nx, ny, nz) is evaluated exactly by placing its sources at the corner of the
smallest such cube with the same cell size and zeros elsewhere: zero sources add
nothing to the sum, and the box's own cells are read back.  Evaluated as is, this
costs the cube's work (for 320 x 320 x 160 inside 512^3, 8.2 times the box's cells);
with the padding's sources skipped (Ops.skip_zero_sources) and the targets restricted
to the leaves that meet the box (Ops.restrict_targets with leaf_mask below), most of
the padding's work is not done.
"""
import numpy as np
import torch


def cube_side(shape, min_side=8):
    n = min_side
    while n < max(shape):
        n *= 2
    return n


def embed(I, shape, n=None):
    """[nx*ny*nz] or [nx, ny, nz] tensor -> [n^3] tensor, I at the low corner."""
    n = n or cube_side(shape)
    cube = torch.zeros((n, n, n), dtype=I.dtype, device=I.device)
    cube[:shape[0], :shape[1], :shape[2]] = I.reshape(shape)
    return cube.reshape(-1)


def extract(S, shape, n=None):
    """[n^3] tensor -> [nx, ny, nz] view of the box's cells (contiguous copy)."""
    n = n or cube_side(shape)
    return S.reshape(n, n, n)[:shape[0], :shape[1], :shape[2]].contiguous()


def leaf_mask(shape, n, leaf_side):
    """[nb, nb, nb] uint8 mask (nb = n / leaf_side) of the leaves that hold at least one
    cell of the box [0, nx) x [0, ny) x [0, nz) at the cube's low corner."""
    nb = n // leaf_side
    m = np.zeros((nb, nb, nb), dtype=np.uint8)
    m[:-(-shape[0] // leaf_side), :-(-shape[1] // leaf_side), :-(-shape[2] // leaf_side)] = 1
    return m
