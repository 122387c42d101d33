"""Pins of the FP64 reference network and its resampling helpers."""
import numpy as np
import pytest
from scipy.ndimage import map_coordinates

from oracle import conv3d_ref as C
from oracle import surrogate_ref as S

TAPS = {"conv3": 27, "down2": 8, "up2": 8, "point": 1}


def _params(rng):
    return {name: (rng.standard_normal((TAPS[k], co, ci)) * np.sqrt(2 / (TAPS[k] * ci)),
                   rng.standard_normal(co) * 0.1) for name, k, ci, co, act, skip in S.LAYERS}


def test_network_gradient_matches_differences():
    rng = np.random.default_rng(0)
    n = 8
    params = _params(rng)
    feat = C.neighbourhood27(rng.standard_normal((n, n, n)))
    t = rng.standard_normal((n, n, n))
    pred, cache = S.forward(feat, params)
    _, g = C.rel_l2_loss([pred], [t])
    grads = S.backward(cache, params, g[0])
    e = 1e-7
    for name in ("in", "e0", "d1", "e2", "d3", "u2", "u0", "head"):
        w, b = params[name]
        for which, base in ((0, w), (1, b)):
            d = np.random.default_rng(hash(name) % 1000 + which).standard_normal(base.shape)
            pp = dict(params)
            pp[name] = (w + e * d, b) if which == 0 else (w, b + e * d)
            Lp = C.rel_l2_loss([S.forward(feat, pp)[0]], [t])[0]
            pp[name] = (w - e * d, b) if which == 0 else (w, b - e * d)
            Lm = C.rel_l2_loss([S.forward(feat, pp)[0]], [t])[0]
            num = (Lp - Lm) / (2 * e)
            ana = np.vdot(grads[name][which], d)
            assert ana == pytest.approx(num, rel=1e-5, abs=1e-9), (name, which)


def test_upsample2_is_scipy_linear_interpolation():
    rng = np.random.default_rng(1)
    c = rng.standard_normal((6, 6, 6))
    x = np.clip((np.arange(12) + 0.5) / 2 - 0.5, 0, 5)
    X, Y, Z = np.meshgrid(x, x, x, indexing="ij")
    ref = map_coordinates(c, [X.ravel(), Y.ravel(), Z.ravel()], order=1, mode="nearest").reshape(12, 12, 12)
    np.testing.assert_allclose(C.upsample2(c), ref, rtol=1e-12, atol=1e-12)


def test_resampling_is_exact_on_affine_fields():
    n = 16
    i = np.arange(n) + 0.5
    X, Y, Z = np.meshgrid(i, i, i, indexing="ij")
    f = 2 * X - 3 * Y + 0.5 * Z + 1
    c = C.coarsen2(f)
    I2 = (np.arange(n // 2) + 0.5) * 2
    Xc, Yc, Zc = np.meshgrid(I2, I2, I2, indexing="ij")
    np.testing.assert_allclose(c, 2 * Xc - 3 * Yc + 0.5 * Zc + 1, rtol=1e-13)
    u = C.upsample2(c)
    np.testing.assert_allclose(u[1:-1, 1:-1, 1:-1], f[1:-1, 1:-1, 1:-1], rtol=1e-12)


def test_neighbourhood27_centre_channel_and_shift():
    f = np.arange(4 ** 3, dtype=float).reshape(4, 4, 4)
    nb = C.neighbourhood27(f)
    np.testing.assert_array_equal(nb[13], f)                   # (0, 0, 0)
    np.testing.assert_array_equal(nb[14][:, :, :3], f[:, :, 1:])  # (0, 0, +1)
    assert np.all(nb[27:] == 0)
