"""Trees over boxes that are columns of cubes along z (nx = ny, nz = R ellz nx / ell), with
cubic or anisotropic cells (Section 3, tree construction; its closing remark on non-uniform
meshes): the leaf order against the oracle's, and the FMM against the oracle's exact sum."""
import numpy as np
import pytest
import torch

from oracle import direct as odirect
from oracle import morton
from tests.gpu_common import rel_l2

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def K():
    from paper_2006_03515_amd import kifmm
    return kifmm


# (n, nz, cell widths, max_leaf) -> (leaf cells x, y, z), root cubes
SHAPES = [
    ((16, 48, (1e-3, 1e-3, 1e-3), 64), ((4, 4, 4), 3)),
    ((32, 40, (1e-3, 1e-3, 4.5e-3), 512), ((8, 8, 2), 5)),
    ((4, 20, (2e-3, 2e-3, 2e-3), 64), ((4, 4, 4), 5)),     # depth 0: one leaf per cube
    ((16, 16, (1e-3, 1e-3, 2e-3), 128), ((4, 4, 2), 2)),
    ((64, 64, (1e-3, 1e-3, 1e-3), 512), ((8, 8, 8), 1)),   # a cube: the octree of before
]


@pytest.mark.parametrize("grid,expect", SHAPES)
def test_column_tree_leaf_order(K, grid, expect):
    n, nz, h, max_leaf = grid
    t = K.build_tree(K.Grid((n, n, nz), h), max_leaf)
    assert (t.leaf_shape, t.roots) == expect
    ell, _, ellz = t.leaf_shape
    got = t.permutation().cpu().numpy()
    assert np.array_equal(got, morton.column_leaf_order(n, nz, ell, ellz))


def _source(shape, h, seed):
    rng = np.random.default_rng(seed)
    I = rng.random(shape) * 1e3
    c = [(np.arange(m) + 0.5) * hh for m, hh in zip(shape, h)]
    x0 = [cc[len(cc) // 3] for cc in c]
    g = [np.exp(-((cc - x) / (4 * hh)) ** 2) for cc, x, hh in zip(c, x0, h)]
    return I + 1e6 * g[0][:, None, None] * g[1][None, :, None] * g[2][None, None, :]


@pytest.mark.parametrize("grid,p_o2", [((16, 48, (1e-3, 1e-3, 1e-3), 64), 150.0),
                                       ((32, 40, (1e-3, 1e-3, 4.5e-3), 512), 150.0),
                                       ((32, 40, (1e-3, 1e-3, 4.5e-3), 512), 1.974),
                                       ((4, 20, (2e-3, 2e-3, 2e-3), 64), 19.74),
                                       ((16, 16, (1e-3, 1e-3, 2e-3), 128), 150.0)])
def test_column_fmm_against_the_exact_sum(K, grid, p_o2, record_property):
    # the FMM over a column of cubes (M2L from level 0, where roots two or more apart
    # interact) in FP64 and FP32 against the oracle's exact sum (its FFT form, any box and
    # cell shape)
    n, nz, h, max_leaf = grid
    shape = (n, n, nz)
    I = _source(shape, h, 300 + n + nz).astype(np.float32).astype(np.float64)
    tree = K.build_tree(K.Grid(shape, h), max_leaf)
    ops = K.precompute_operators(tree, K.Kernel(p_o2), K.Opts(K.LAYOUT_NESTED, 6, 10, 1e-7))
    It = torch.from_numpy(I.ravel()).cuda()
    s64 = K.eval(tree, ops, It, 0.5, precision="fp64").cpu().numpy()
    s32 = K.eval(tree, ops, It.float(), 0.5, precision="fp32").double().cpu().numpy()
    ref = odirect.fft_full(I, h, p_o2, prefactor=0.5).ravel()
    e64, e32, d = rel_l2(s64, ref), rel_l2(s32, ref), rel_l2(s32, s64)
    record_property("rel_l2_fp64", e64)
    print("column %s, %g Torr: fp64 %.3e fp32 %.3e fp32-fp64 %.3e" % (shape, p_o2, e64, e32, d))
    # nested shells m0 = 6, rcond 1e-7 (measured 2.4-4.5e-7 in FP64, FP32 within 1e-7 of it)
    assert e64 < 1e-6 and e32 < 1e-6
    assert d < 1e-6
