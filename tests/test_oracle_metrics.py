"""Pins of the error measures of Section 4, eq. (relativefun), on hand-computed cases."""
import numpy as np
import pytest

from oracle import metrics


def test_rel_l2_hand_case():
    # ||(3, 4+1) - (3, 4)|| / ||(3, 4)|| = 1 / 5
    assert metrics.rel_l2([3.0, 5.0], [3.0, 4.0]) == pytest.approx(0.2, rel=1e-15)
    # the reference is the denominator, not the approximation: ||(0, 4)|| / ||(3, 0)||
    assert metrics.rel_l2([3.0, 4.0], [3.0, 0.0]) == pytest.approx(4.0 / 3.0, rel=1e-15)


def _grid3():
    # cell centres of a 3 x 3 x 3 grid of unit cells, x0 = the middle centre
    c = np.arange(3) + 0.5
    X, Y, Z = np.meshgrid(c, c, c, indexing="ij")
    return np.stack([X, Y, Z], -1), (1.5, 1.5, 1.5)


def test_e_delta_hand_case():
    centres, x0 = _grid3()
    ref = np.full((3, 3, 3), 2.0)
    num = ref.copy()
    num[1, 1, 1] = 2.2      # the middle point: relative error 0.1
    num[1, 1, 2] = 1.5      # a face neighbour at distance exactly 1 = delta: 0.25, counted
    num[0, 0, 1] = 100.0    # an edge neighbour at distance sqrt(2) > delta: not counted
    # delta = 1: the middle point and its 6 face neighbours, N_tot = 7
    assert metrics.e_delta(num, ref, centres, x0, 1.0) == pytest.approx((0.1 + 0.25) / 7, rel=1e-14)
    # delta = 1.5 also takes the 12 edge neighbours (sqrt 2), not the 8 corners (sqrt 3):
    # N_tot = 19, and the far point now counts with |100 - 2| / 2 = 49
    assert metrics.e_delta(num, ref, centres, x0, 1.5) == pytest.approx((0.1 + 0.25 + 49.0) / 19, rel=1e-14)
    # the error is relative to the reference at each point, not to its mean
    ref2 = ref.copy()
    ref2[1, 1, 2] = 1.0
    num2 = ref2.copy()
    num2[1, 1, 2] = 1.5     # 0.5 relative
    assert metrics.e_delta(num2, ref2, centres, x0, 1.0) == pytest.approx(0.5 / 7, rel=1e-14)


def test_e_delta_needs_points_in_the_ball():
    centres, _ = _grid3()
    with pytest.raises(ValueError):
        metrics.e_delta(np.ones(27), np.ones(27), centres, (10.0, 10.0, 10.0), 1.0)
