"""Pins of the FP64 reference layers of the surrogate network."""
import numpy as np
import pytest
from scipy.signal import correlate

from oracle import conv3d_ref as C

rng = np.random.default_rng(0)


def test_conv3_matches_scipy_correlate():
    x = rng.standard_normal((3, 6, 6, 6))
    w = rng.standard_normal((2, 3, 3, 3, 3))
    y = C.conv3(x, w)
    for o in range(2):
        ref = sum(correlate(x[i], w[o, i], mode="same", method="direct") for i in range(3))
        np.testing.assert_allclose(y[o], ref, rtol=1e-12, atol=1e-12)


def test_point_is_matrix_product():
    x = rng.standard_normal((4, 3, 3, 3))
    w = rng.standard_normal((5, 4))
    np.testing.assert_allclose(C.point(x, w), (w @ x.reshape(4, -1)).reshape(5, 3, 3, 3), rtol=1e-13)


def test_down2_matches_strided_correlation():
    x = rng.standard_normal((2, 8, 8, 8))
    w = rng.standard_normal((3, 2, 2, 2, 2))
    y = C.down2(x, w)
    for o in range(3):
        full = sum(correlate(x[i], w[o, i], mode="valid", method="direct") for i in range(2))
        np.testing.assert_allclose(y[o], full[::2, ::2, ::2], rtol=1e-12, atol=1e-12)


def test_up2_is_adjoint_of_down2():
    # <down2(x, w), y> = <x, up2(y, w^T)> with w^T swapping the channel axes
    x = rng.standard_normal((2, 8, 8, 8))
    y = rng.standard_normal((3, 4, 4, 4))
    w = rng.standard_normal((3, 2, 2, 2, 2))
    lhs = np.vdot(C.down2(x, w), y)
    rhs = np.vdot(x, C.up2(y, w.transpose(1, 0, 2, 3, 4)))
    assert lhs == pytest.approx(rhs, rel=1e-12)


@pytest.mark.parametrize("layer", ["conv3", "down2", "up2", "point"])
def test_backward_is_adjoint_and_weight_gradient_matches_differences(layer):
    f, b = getattr(C, layer), getattr(C, layer + "_backward")
    shapes = {"conv3": ((2, 5, 5, 5), (3, 2, 3, 3, 3)), "down2": ((2, 6, 6, 6), (3, 2, 2, 2, 2)),
              "up2": ((2, 3, 3, 3), (3, 2, 2, 2, 2)), "point": ((2, 4, 4, 4), (3, 2))}
    xs, ws = shapes[layer]
    x, w = rng.standard_normal(xs), rng.standard_normal(ws)
    gy = rng.standard_normal(f(x, w).shape)
    gx, gw = b(x, w, gy)
    # linear in x: <gy, f(dx)> = <gx, dx>
    dx = rng.standard_normal(xs)
    assert np.vdot(gy, f(dx, w)) == pytest.approx(np.vdot(gx, dx), rel=1e-11)
    # central differences in w (f is linear in w, so they are exact up to rounding)
    dw = rng.standard_normal(ws)
    e = 1e-3
    num = (np.vdot(gy, f(x, w + e * dw)) - np.vdot(gy, f(x, w - e * dw))) / (2 * e)
    assert np.vdot(gw, dw) == pytest.approx(num, rel=1e-9)


def test_leaky_and_loss_gradients_by_differences():
    x = rng.standard_normal(50)
    gy = rng.standard_normal(50)
    gx = C.leaky_backward(x, 0.1, gy)
    d = rng.standard_normal(50)
    e = 1e-7
    num = (np.vdot(gy, C.leaky(x + e * d, 0.1)) - np.vdot(gy, C.leaky(x - e * d, 0.1))) / (2 * e)
    assert np.vdot(gx, d) == pytest.approx(num, rel=1e-6)
    y = [rng.standard_normal((2, 3)), rng.standard_normal((2, 3))]
    t = [rng.standard_normal((2, 3)), rng.standard_normal((2, 3))]
    L, g = C.rel_l2_loss(y, t)
    assert L == pytest.approx(np.mean([np.sum((a - b) ** 2) / np.sum(b * b) for a, b in zip(y, t)]))
    dy = [rng.standard_normal((2, 3)) for _ in y]
    e = 1e-6
    Lp = C.rel_l2_loss([a + e * b for a, b in zip(y, dy)], t)[0]
    Lm = C.rel_l2_loss([a - e * b for a, b in zip(y, dy)], t)[0]
    assert sum(np.vdot(a, b) for a, b in zip(g, dy)) == pytest.approx((Lp - Lm) / (2 * e), rel=1e-7)


def test_adam_first_step_moves_by_learning_rate():
    # with zero moments the bias-corrected first step is lr * g / (|g| + eps)
    w = np.array([1.0, -2.0, 3.0])
    g = np.array([0.5, -4.0, 1e-3])
    w1, m, v = C.adam(w, g, np.zeros(3), np.zeros(3), 1, lr=0.01, eps=1e-12)
    np.testing.assert_allclose(w1, w - 0.01 * np.sign(g), rtol=1e-9)
    np.testing.assert_allclose(m, 0.1 * g)
    np.testing.assert_allclose(v, 0.001 * g * g)
