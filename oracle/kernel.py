"""FP64 photoionization kernel (oracle; test infrastructure only).

Definitions followed:
  * Section 2.1, eq. (gfun): g(r)/pO2 = (exp(-chi_min pO2 r) - exp(-chi_max pO2 r))
    / (pO2 r ln(chi_max/chi_min)).  pO2 cancels, so with a = chi_min pO2 and
    b = chi_max pO2:  g(r) = (e^{-a r} - e^{-b r}) / (r ln(chi_max/chi_min)).
  * Section 2.1, eq. (integral): the integrand is I(y) g(|x-y|) / (4 pi |x-y|^2),
    so the point kernel is K(R) = g(R) / (4 pi R^2).
  * Section 3, eq. (summation) and the discrete kernel G that follows it: the
    midpoint rule for i != j, and for the self cell
    G_ii = 3 g(rho) / (pi (hx^2 + hy^2 + hz^2)),  rho = sqrt((hx^2+hy^2+hz^2)/12).
    Cell volumes are applied to the source values, not to G.

The difference of exponentials is written as -e^{-a r} * expm1(-(b-a) r), which is
the same number without the cancellation of the plain difference when b r is small.
"""
import numpy as np

CHI_MIN = 0.035   # 1/(cm Torr), Section 2.1
CHI_MAX = 2.0     # 1/(cm Torr), Section 2.1


def coefficients(p_o2, chi_min=CHI_MIN, chi_max=CHI_MAX):
    """Return (a, b, ln(chi_max/chi_min)) for partial pressure p_o2 [Torr]."""
    return chi_min * p_o2, chi_max * p_o2, np.log(chi_max / chi_min)


def g(r, p_o2, chi_min=CHI_MIN, chi_max=CHI_MAX):
    """Absorption function g(r) of eq. (gfun), r in cm, result in 1/cm."""
    a, b, ln = coefficients(p_o2, chi_min, chi_max)
    r = np.asarray(r, dtype=np.float64)
    return -np.exp(-a * r) * np.expm1(-(b - a) * r) / (r * ln)


def K(R, p_o2, chi_min=CHI_MIN, chi_max=CHI_MAX):
    """Point kernel g(R) / (4 pi R^2) of eq. (integral), in 1/cm^3 (R > 0)."""
    R = np.asarray(R, dtype=np.float64)
    return g(R, p_o2, chi_min, chi_max) / (4.0 * np.pi * R * R)


def self_value(hx, hy, hz, p_o2, chi_min=CHI_MIN, chi_max=CHI_MAX):
    """Self-cell value G_ii of the discrete kernel (Section 3, after eq. (summation))."""
    s2 = hx * hx + hy * hy + hz * hz
    rho = np.sqrt(s2 / 12.0)
    return 3.0 * g(rho, p_o2, chi_min, chi_max) / (np.pi * s2)


def offset_table(n, h, p_o2, chi_min=CHI_MIN, chi_max=CHI_MAX):
    """G over all integer cell offsets of an n[0] x n[1] x n[2] grid (n an int for a
    cube) with spacing h = (hx, hy, hz).

    Returns an array T of shape (2n[a]-1 per axis) with T[d + n-1] = G(offset d),
    where the offset d = (di, dj, dk) is in cells; the centre entry is the self value.
    """
    ns = (n, n, n) if np.isscalar(n) else tuple(int(v) for v in n)
    hx, hy, hz = h
    ox, oy, oz = (np.arange(-(m - 1), m, dtype=np.float64) for m in ns)
    X, Y, Z = np.meshgrid(ox * hx, oy * hy, oz * hz, indexing="ij", sparse=True)
    R = np.sqrt(X * X + Y * Y + Z * Z)
    c = tuple(m - 1 for m in ns)
    R[c] = 1.0  # placeholder, overwritten below
    T = K(R, p_o2, chi_min, chi_max)
    T[c] = self_value(hx, hy, hz, p_o2, chi_min, chi_max)
    return T
