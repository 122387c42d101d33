"""The oracle's three forms of the exact discrete sum (Section 3, eq. (summation))
against a 30-digit brute force on tiny grids.

The brute force is written from the paper's definitions, not from the oracle's
formulas: g in the form of eq. (gfun) with pO2 factored as printed (the plain
difference of exponentials, exact at 30 digits), the point kernel g / (4 pi R^2) of
eq. (integral), and the self cell as the explicit 2 x 2 x 2 Gauss-Legendre product
rule over the cell (nodes +-1/sqrt(3) of the half widths, equal weights), which is
the rule the self-cell formula after eq. (summation) closes.  A dropped term, a
wrong sign, a swapped axis or a lost digit to cancellation (the expm1 rewrite) in
any of the three forms shows up above 5e-15 (the plain difference of the two
exponentials alone costs 1.3e-14 at 10 Torr and R = 1e-3 cm).
"""
import mpmath
import numpy as np
import pytest

from oracle import direct

CHI_MIN, CHI_MAX = mpmath.mpf("0.035"), mpmath.mpf(2)


def _g(r, p_o2):
    # eq. (gfun): g / pO2 = (exp(-chi_min pO2 r) - exp(-chi_max pO2 r)) / (pO2 r ln(chi_max / chi_min))
    return p_o2 * (mpmath.exp(-CHI_MIN * p_o2 * r) - mpmath.exp(-CHI_MAX * p_o2 * r)) / (
        p_o2 * r * mpmath.log(CHI_MAX / CHI_MIN))


def _point(r, p_o2):
    # eq. (integral): the integrand's kernel g(R) / (4 pi R^2)
    return _g(r, p_o2) / (4 * mpmath.pi * r * r)


def _self_cell(h, p_o2):
    # mean of the point kernel over the 8 nodes of the 2-point Gauss-Legendre product rule
    # on the cell [-hx/2, hx/2] x [-hy/2, hy/2] x [-hz/2, hz/2] (weights V/8 each, so the
    # cell integral divided by V)
    t = 1 / mpmath.sqrt(3)
    acc = mpmath.mpf(0)
    for sx in (-1, 1):
        for sy in (-1, 1):
            for sz in (-1, 1):
                x, y, z = sx * t * h[0] / 2, sy * t * h[1] / 2, sz * t * h[2] / 2
                acc += _point(mpmath.sqrt(x * x + y * y + z * z), p_o2)
    return acc / 8


def brute_force(I, h, p_o2, prefactor):
    """S_i = c sum_j G(x_i, y_j) I_j hx hy hz at every cell, 30 significant digits."""
    mpmath.mp.dps = 30
    nx, ny, nz = I.shape
    hm = [mpmath.mpf(float(v)) for v in h]
    pm = mpmath.mpf(float(p_o2))
    # kernel values by integer offset (the same for every pair with that offset)
    table = {}
    for dx in range(nx):
        for dy in range(ny):
            for dz in range(nz):
                if dx == dy == dz == 0:
                    table[(0, 0, 0)] = _self_cell(hm, pm)
                else:
                    table[(dx, dy, dz)] = _point(mpmath.sqrt((dx * hm[0]) ** 2 + (dy * hm[1]) ** 2
                                                             + (dz * hm[2]) ** 2), pm)
    w = mpmath.mpf(float(prefactor)) * hm[0] * hm[1] * hm[2]
    q = [mpmath.mpf(float(v)) for v in I.ravel()]
    out = np.empty(I.size)
    cells = [(i, j, k) for i in range(nx) for j in range(ny) for k in range(nz)]
    for t, (i, j, k) in enumerate(cells):
        acc = mpmath.mpf(0)
        for s, (a, b, c) in enumerate(cells):
            acc += table[(abs(i - a), abs(j - b), abs(k - c))] * q[s]
        out[t] = float(acc * w)
    return out.reshape(I.shape)


CASES = [
    # (shape, cell widths [cm], pO2 [Torr], prefactor)
    ((4, 4, 4), (2.5e-3,) * 3, 150.0, 1.0),
    ((5, 5, 5), (3.125e-3,) * 3, 1.974, 0.0366),   # 10 Torr air: b R ~ 1e-2, the expm1 regime
    ((6, 5, 4), (1e-3, 1.5e-3, 4.5e-3), 19.74, 0.2),  # box-shaped grid, anisotropic cells
    ((6, 6, 6), (1.5625e-3,) * 3, 150.0, 1.0),
]


@pytest.mark.parametrize("shape,h,p_o2,c", CASES)
def test_three_forms_equal_the_30_digit_sum(shape, h, p_o2, c):
    rng = np.random.default_rng(91 + sum(shape))
    I = rng.uniform(0.0, 1e20, shape)
    I[rng.random(shape) < 0.2] = 0.0    # some zero sources, as in the streamer's empty regions
    ref = brute_force(I, h, p_o2, c)
    tg = np.arange(I.size)
    forms = {
        "direct_numpy": direct.direct_numpy(I, h, p_o2, tg, prefactor=c).reshape(shape),
        "direct_targets": direct.direct_targets(I, h, p_o2, tg, prefactor=c).reshape(shape),
        "fft_full": direct.fft_full(I, h, p_o2, prefactor=c),
    }
    for name, got in forms.items():
        err = float(np.max(np.abs(got / ref - 1)))
        assert err <= 5e-15, (name, err)   # measured <= 7e-16 for every form
