"""Tree construction (HIP Morton scatter) against the oracle's leaf order."""
import numpy as np
import pytest
import torch

from oracle import morton

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("n,max_leaf,ell", [(4, 64, 4), (16, 64, 4), (32, 64, 4), (32, 512, 8),
                                            (64, 512, 8), (64, 100, 4), (16, 4096, 16)])
def test_permutation_bit_exact(n, max_leaf, ell):
    from paper_2006_03515_amd import kifmm as K
    t = K.build_tree(K.Grid.cube(n, 0.1), max_leaf)
    assert t.leaf_side == ell
    assert t.depth == int(np.log2(n // ell))
    got = t.permutation().cpu().numpy()
    assert np.array_equal(got, morton.leaf_order(n, ell))
