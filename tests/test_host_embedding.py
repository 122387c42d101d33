"""Host logic of the cube embedding of box-shaped grids (no GPU)."""
import numpy as np
import torch

from paper_2006_03515_amd import embedding


def test_cube_side_is_the_smallest_power_of_two_cover():
    assert embedding.cube_side((320, 320, 160)) == 512
    assert embedding.cube_side((12, 10, 6)) == 16
    assert embedding.cube_side((8, 8, 8)) == 8
    assert embedding.cube_side((3, 2, 1)) == 8          # at least one 8^3 leaf
    assert embedding.cube_side((65, 1, 1)) == 128


def test_embed_then_extract_round_trip_and_zero_padding():
    shape = (5, 3, 7)
    I = torch.arange(5 * 3 * 7, dtype=torch.float64).reshape(shape) + 1.0
    cube = embedding.embed(I, shape)
    n = embedding.cube_side(shape)
    assert cube.numel() == n ** 3
    c = cube.reshape(n, n, n)
    assert torch.equal(c[:5, :3, :7], I)
    assert float(c.abs().sum()) == float(I.sum())        # nothing outside the box
    assert torch.equal(embedding.extract(cube, shape), I)


def test_leaf_mask_covers_exactly_the_leaves_that_meet_the_box():
    shape, n, ell = (12, 10, 6), 16, 4
    m = embedding.leaf_mask(shape, n, ell)
    assert m.shape == (4, 4, 4) and m.dtype == np.uint8
    # brute force: a leaf is wanted iff one of its cells lies in the box
    for a in range(4):
        for b in range(4):
            for c in range(4):
                meets = any(a * ell + i < shape[0] and b * ell + j < shape[1] and c * ell + k < shape[2]
                            for i in range(ell) for j in range(ell) for k in range(ell))
                assert bool(m[a, b, c]) == meets, (a, b, c)
    # the paper's 320 x 320 x 160 box in 512^3 with 8^3 leaves: 40 x 40 x 20 leaves
    m = embedding.leaf_mask((320, 320, 160), 512, 8)
    assert int(m.sum()) == 40 * 40 * 20
