"""Continuum closed forms of the photoionization integral (oracle; tests only).

These are values of eq. (integral) of Section 2.1 itself, not of its discretisation,
at the centre of two sources with spherical symmetry.  In spherical coordinates
around the evaluation point the solid angle cancels the 4 pi R^2 of the kernel:

    S(0) = c * int_0^inf I(R) g(R) dR,  g(R) = (e^{-aR} - e^{-bR}) / (R ln(chi_max/chi_min))

Ball of radius Rb and constant value I0:
    int_0^Rb (e^{-aR} - e^{-bR})/R dR = ln(b/a) + E1(b Rb) - E1(a Rb)
  (differentiate in a: d/da gives -(1 - e^{-a Rb})/a; integrate back, using that
   the expression vanishes at a = b).  As Rb -> inf it tends to ln(b/a) =
   ln(chi_max/chi_min), so S(0) -> c I0: every emitted photon is absorbed somewhere.

Gaussian I0 exp(-R^2/sigma^2):
    int_0^inf e^{-R^2/sigma^2 - tR} dR = (sigma sqrt(pi)/2) erfcx(t sigma/2)
  and (e^{-aR} - e^{-bR})/R = int_a^b e^{-tR} dt, so
    S(0) = c I0 sqrt(pi) / ln(chi_max/chi_min) * int_{a sigma/2}^{b sigma/2} erfcx(u) du.
"""
import numpy as np
from scipy.integrate import quad
from scipy.special import erfcx, exp1

from . import kernel as _k


def ball_centre(Rb, p_o2, I0=1.0, prefactor=1.0):
    a, b, ln = _k.coefficients(p_o2)
    return prefactor * I0 * (np.log(b / a) + exp1(b * Rb) - exp1(a * Rb)) / ln


def gaussian_centre(sigma, p_o2, I0=1.0, prefactor=1.0):
    a, b, ln = _k.coefficients(p_o2)
    val, _ = quad(erfcx, a * sigma / 2, b * sigma / 2, limit=400, epsabs=0, epsrel=1e-13)
    return prefactor * I0 * np.sqrt(np.pi) * val / ln


def gaussian_centre_radial(sigma, p_o2, I0=1.0, prefactor=1.0):
    """Same value by direct radial quadrature of int_0^inf I(R) g(R) dR."""
    def f(R):
        return np.exp(-(R / sigma) ** 2) * _k.g(R, p_o2)
    val = 0.0
    edges = np.concatenate([[0.0], sigma * np.array([0.25, 0.5, 1, 2, 3, 4, 6, 8])])
    for lo, hi in zip(edges[:-1], edges[1:]):
        v, _ = quad(f, lo, hi, limit=400, epsabs=0, epsrel=1e-13)
        val += v
    return prefactor * I0 * val
