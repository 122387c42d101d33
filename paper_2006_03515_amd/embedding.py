"""Box-shaped grids evaluated inside a cube.

The tree needs an n^3 grid with n a power of two.  A box-shaped grid of isotropic
cells (nx, ny, nz) is evaluated exactly by placing its sources at the corner of the
smallest such cube with the same cell size and zeros elsewhere: zero sources add
nothing to the sum, and the box's own cells are read back.  This costs the cube's
work (for 320 x 320 x 160 inside 512^3, 8.2 times the box's cells).
"""
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
