"""Pins of the oracle's exact discrete sum (Section 3, eq. (summation))."""
import numpy as np
import pytest

from oracle import closed_forms, direct

L = 0.1


def _grid(n, L=L):
    h = L / n
    c = (np.arange(n) + 0.5) * h
    return h, np.meshgrid(c, c, c, indexing="ij")


def _gauss(n, sigma=0.01, centre=None):
    h, (X, Y, Z) = _grid(n)
    c = L / 2 if centre is None else centre
    return h, np.exp(-((X - c) ** 2 + (Y - c) ** 2 + (Z - c) ** 2) / sigma ** 2)


def test_three_forms_agree():
    # direct loop (numpy), direct loop (C/OpenMP) and the FFT convolution are three
    # different algorithms for the same sum
    rng = np.random.default_rng(3)
    n = 12
    h = L / n
    I = rng.random((n, n, n))
    full = direct.fft_full(I, (h, h, h), 150.0)
    tg = rng.choice(n ** 3, 40, replace=False)
    a = direct.direct_numpy(I, (h, h, h), 150.0, tg)
    b = direct.direct_targets(I, (h, h, h), 150.0, tg)
    np.testing.assert_allclose(b, a, rtol=1e-13)
    np.testing.assert_allclose(full.ravel()[tg], a, rtol=1e-12)


def test_anisotropic_cells_direct_forms_agree():
    rng = np.random.default_rng(4)
    I = rng.random((6, 5, 7))
    h = (2e-3, 1e-3, 1.5e-3)
    tg = np.arange(I.size)
    np.testing.assert_allclose(direct.direct_targets(I, h, 19.74, tg),
                               direct.direct_numpy(I, h, 19.74, tg), rtol=1e-13)


def test_fft_form_on_box_shaped_grids():
    # box-shaped grids (nx != ny != nz), isotropic and anisotropic cells: the FFT
    # convolution equals the direct loop at every cell
    rng = np.random.default_rng(5)
    for shape, h in (((6, 5, 7), (2e-3, 1e-3, 1.5e-3)), ((8, 8, 4), (1.25e-3,) * 3)):
        I = rng.random(shape)
        full = direct.fft_full(I, h, 19.74, prefactor=0.3)
        ref = direct.direct_numpy(I, h, 19.74, None, prefactor=0.3).reshape(shape)
        np.testing.assert_allclose(full, ref, rtol=1e-12)


def test_linearity_symmetry_positivity():
    rng = np.random.default_rng(5)
    n = 10
    h = (L / n,) * 3
    u, v = rng.random((n, n, n)), rng.random((n, n, n))
    Su, Sv = direct.fft_full(u, h, 150.0), direct.fft_full(v, h, 150.0)
    Suv = direct.fft_full(2.0 * u - 3.0 * v, h, 150.0)
    np.testing.assert_allclose(Suv, 2.0 * Su - 3.0 * Sv, rtol=1e-10, atol=1e-12 * np.abs(Su).max())
    # G is symmetric, so <u, S v> = <S u, v>
    assert np.vdot(u, Sv) == pytest.approx(np.vdot(Su, v), rel=1e-12)
    assert np.all(Su > 0)


def test_translation_by_whole_cells():
    # a compactly supported source shifted by (2,-1,3) cells gives the shifted field
    n = 16
    h = (L / n,) * 3
    rng = np.random.default_rng(6)
    I = np.zeros((n, n, n))
    I[5:10, 5:10, 4:9] = rng.random((5, 5, 5))
    J = np.roll(I, (2, -1, 3), axis=(0, 1, 2))
    SI = direct.fft_full(I, h, 19.74)
    SJ = direct.fft_full(J, h, 19.74)
    np.testing.assert_allclose(SJ[2:, :-1, 3:], SI[:-2, 1:, :-3], rtol=1e-11)


@pytest.mark.parametrize("p_o2", [150.0, 19.74, 1.974])
def test_first_order_convergence_to_closed_forms(p_o2):
    # The discrete sum at the centre of a uniform ball (radius 0.4 mm) and of a
    # Gaussian (sigma 0.1 mm) tends to the continuum value at first order in h:
    # the error ratio at h -> h/2 is near 2, and the Richardson value 2 v(h/2) - v(h)
    # lands on the closed form.
    ex_b = closed_forms.ball_centre(0.04, p_o2)
    ex_g = closed_forms.gaussian_centre(0.01, p_o2)
    vb, vg = [], []
    for n in (64, 128, 256):
        h, (X, Y, Z) = _grid(n)
        c = (n // 2 + 0.5) * h
        R2 = (X - c) ** 2 + (Y - c) ** 2 + (Z - c) ** 2
        t = [(n // 2 * n + n // 2) * n + n // 2]
        vb.append(direct.direct_targets((R2 <= 0.04 ** 2).astype(float), (h,) * 3, p_o2, t)[0])
        vg.append(direct.direct_targets(np.exp(-R2 / 0.01 ** 2), (h,) * 3, p_o2, t)[0])
    for v, ex, tol in ((vb, ex_b, 2e-3), (vg, ex_g, 2e-3)):
        e = [x / ex - 1 for x in v]
        assert all(x < 0 for x in e)
        assert 1.8 < e[1] / e[2] < 2.2
        assert abs((2 * v[2] - v[1]) / ex - 1) < tol


def test_uniform_cube_bracketed_by_balls():
    # K > 0, so a full uniform cube at its centre lies between the closed forms of the
    # inscribed and the circumscribed balls (checked on the Richardson value)
    p_o2 = 150.0
    vals = []
    for n in (64, 128):
        h = L / n
        I = np.ones((n, n, n))
        # centre cell of the cube (offset h/2 from the true centre)
        t = [(n // 2 * n + n // 2) * n + n // 2]
        vals.append(direct.direct_targets(I, (h,) * 3, p_o2, t)[0])
    rich = 2 * vals[1] - vals[0]
    lo = closed_forms.ball_centre(L / 2 - L / 128, p_o2)
    hi = closed_forms.ball_centre(np.sqrt(3) * (L / 2 + L / 128), p_o2)
    assert lo < rich < hi


def test_gaussian_closed_form_two_derivations():
    for p_o2 in (150.0, 19.74, 1.974):
        assert closed_forms.gaussian_centre(0.01, p_o2) == pytest.approx(
            closed_forms.gaussian_centre_radial(0.01, p_o2), rel=1e-11)


def test_ball_tends_to_photon_conservation():
    # Rb -> infinity: S(0) -> c I0
    assert closed_forms.ball_centre(1e4, 150.0, I0=2.0, prefactor=0.5) == pytest.approx(1.0, rel=1e-12)
