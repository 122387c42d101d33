"""Pins of the oracle's kernel (Section 2.1 eq. (gfun), Section 3 self-cell rule)."""
import numpy as np
import pytest
from scipy.integrate import quad

from oracle import kernel as K


@pytest.mark.parametrize("h", [(1e-3, 1e-3, 1e-3), (2e-3, 1e-3, 5e-4), (3.125e-3,) * 3])
@pytest.mark.parametrize("p_o2", [150.0, 19.74, 0.1])
def test_self_value_is_2x2x2_gauss_legendre(h, p_o2):
    # The self value of Section 3 equals the second-order (2-point per axis)
    # Gauss-Legendre rule applied to the kernel over the cell, divided by the
    # cell volume.  Nodes from numpy's leggauss, not from the formula.
    x, w = np.polynomial.legendre.leggauss(2)
    hx, hy, hz = h
    total = 0.0
    for xi, wi in zip(x, w):
        for yj, wj in zip(x, w):
            for zk, wk in zip(x, w):
                R = np.sqrt((xi * hx / 2) ** 2 + (yj * hy / 2) ** 2 + (zk * hz / 2) ** 2)
                total += wi * wj * wk / 8 * K.K(R, p_o2)
    assert K.self_value(hx, hy, hz, p_o2) == pytest.approx(total, rel=1e-14)


@pytest.mark.parametrize("p_o2", [150.0, 19.74, 1.974, 0.1])
def test_photon_conservation(p_o2):
    # int_0^inf g(r) dr = ln(chi_max/chi_min)/ln(chi_max/chi_min) = 1: every photon
    # emitted is absorbed somewhere (Frullani integral).  Catches a wrong
    # normalisation, sign or exponent in g.
    a, b, _ = K.coefficients(p_o2)
    pts = [0, 1 / b, 10 / b, 1 / a, 10 / a, 60 / a]
    tot = sum(quad(lambda r: K.g(r, p_o2), lo, hi, limit=400, epsrel=1e-13, epsabs=0)[0]
              for lo, hi in zip(pts[:-1], pts[1:]))
    assert tot == pytest.approx(1.0, rel=1e-9)


def test_g_small_r_limit():
    # g(r) -> (b - a)/ln(chi_max/chi_min) as r -> 0 (first-order Taylor of the exponentials)
    for p_o2 in (150.0, 1.0):
        a, b, ln = K.coefficients(p_o2)
        r = 1e-9 / b
        assert K.g(r, p_o2) == pytest.approx((b - a) / ln, rel=1e-7)


def test_kernel_positive_decreasing():
    R = np.geomspace(1e-5, 10.0, 2000)
    for p_o2 in (150.0, 19.74, 1.974):
        k = K.K(R, p_o2)
        assert np.all(k > 0)
        assert np.all(np.diff(k) < 0)


def test_expm1_form_matches_difference_without_cancellation():
    # where b r is large the plain difference has no cancellation; both forms agree
    r = np.linspace(0.05, 2.0, 100)
    p_o2 = 150.0
    a, b, ln = K.coefficients(p_o2)
    plain = (np.exp(-a * r) - np.exp(-b * r)) / (r * ln)
    np.testing.assert_allclose(K.g(r, p_o2), plain, rtol=1e-14)


def test_offset_table_symmetry_and_centre():
    T = K.offset_table(5, (1e-3, 1e-3, 1e-3), 150.0)
    np.testing.assert_array_equal(T, T[::-1, :, :])
    np.testing.assert_array_equal(T, T.transpose(1, 0, 2))
    assert T[4, 4, 4] == K.self_value(1e-3, 1e-3, 1e-3, 150.0)
