"""Host logic of the cube embedding of box-shaped grids (no GPU)."""
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
