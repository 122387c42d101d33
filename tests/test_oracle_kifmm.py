"""Pins of the oracle FMM (Section 3) against the exact discrete sum."""
import numpy as np
import pytest

from oracle import direct, kifmm_ref, metrics

L = 0.1


def _gauss(n, sigma=0.01):
    h = L / n
    c = (np.arange(n) + 0.5) * h
    X, Y, Z = np.meshgrid(c, c, c, indexing="ij")
    return h, 1e20 * np.exp(-((X - L / 2) ** 2 + (Y - L / 2) ** 2 + (Z - L / 2) ** 2) / sigma ** 2)


def test_depth_one_tree_is_all_near_field():
    # with at most 2 leaves per axis every leaf is in every other's near range, so the
    # method must reproduce the exact sum
    h, I = _gauss(16)
    ref = direct.fft_full(I, (h,) * 3, 150.0)
    S = kifmm_ref.evaluate(I, L, 150.0, ell=8)
    assert metrics.rel_l2(S, ref) < 1e-13


@pytest.mark.parametrize("p_o2", [150.0, 1.974])
def test_nested_layout_truncation(p_o2):
    h, I = _gauss(32)
    ref = direct.fft_full(I, (h,) * 3, p_o2)
    S = kifmm_ref.evaluate(I, L, p_o2, ell=8, layout="nested", rcond=1e-10)
    assert metrics.rel_l2(S, ref) < 1e-6


def test_paper_layout_within_paper_error_envelope():
    # m0 = 6 single surfaces: the paper reports E_V of 0.15 % to 0.69 % for its runs
    # (Tables 3-7); the oracle's paper layout stays inside 1 % on the 32^3 case
    h, I = _gauss(32)
    ref = direct.fft_full(I, (h,) * 3, 150.0)
    S = kifmm_ref.evaluate(I, L, 150.0, ell=4, layout="paper", rcond=1e-7)
    e = metrics.rel_l2(S, ref)
    assert 1e-4 < e < 1e-2


def test_linearity():
    rng = np.random.default_rng(2)
    n = 32
    u, v = rng.random((n, n, n)), rng.random((n, n, n))
    f = lambda x: kifmm_ref.evaluate(x, L, 19.74, ell=8, layout="single", rcond=1e-7)
    np.testing.assert_allclose(f(u + 2 * v), f(u) + 2 * f(v), rtol=1e-9)


@pytest.mark.parametrize("p_o2", [150.0, 1.974])
def test_lattice_layout_truncation(p_o2):
    # the 125-point lattices bound the accuracy at a few 1e-5 (measured against the exact
    # sum at 32^3 to 256^3, pressures 2 to 150 Torr O2, lattice radii 1.0 r to 1.4 r)
    h, I = _gauss(32)
    ref = direct.fft_full(I, (h,) * 3, p_o2)
    for R in (1.0, 1.2, 1.4):
        S = kifmm_ref.evaluate(I, L, p_o2, ell=4, layout="lattice", m0=5, rcond=1e-7, lattice_radius=R)
        e = metrics.rel_l2(S, ref)
        assert 1e-6 < e < 1e-4, (R, e)


def test_lattice_m2l_matrix_is_a_convolution():
    # with y^u and x^d on lattices of one spacing t, G(x^d_i, y^u_j + 2 r o) depends on
    # i - j only, so applying it is a cyclic convolution of length 2 m0 - 1 per axis; the
    # product computed with numpy's FFT must equal the matrix product
    r, m0, p_o2 = 0.003, 5, 150.0
    R = 1.2 * r
    yu, _, _, xd = kifmm_ref.point_sets("lattice", m0, 10, r, lattice_radius=1.2)
    t = 2 * R / (m0 - 1)
    idx = np.rint((yu + R) / t).astype(int)          # lattice indices 0..m0-1
    assert np.allclose(idx * t - R, yu) and np.allclose(xd, yu)
    N = 2 * m0 - 1
    rng = np.random.default_rng(8)
    e = rng.standard_normal(len(yu))
    for o in ((2, 0, 0), (-3, 1, 2), (3, 3, -3), (0, -2, 1)):
        sh = 2 * r * np.array(o)
        want = kifmm_ref.gmat(xd, yu + sh, p_o2) @ e
        d = np.stack(np.meshgrid(*(np.arange(-(m0 - 1), m0),) * 3, indexing="ij"), -1).reshape(-1, 3)
        g = np.zeros((N, N, N))
        g[tuple((d % N).T)] = kifmm_ref.gmat(np.zeros((1, 3)), -(d * t) + sh, p_o2)[0]
        E = np.zeros((N, N, N))
        E[tuple(idx.T)] = e
        conv = np.fft.irfftn(np.fft.rfftn(g) * np.fft.rfftn(E), s=(N, N, N))
        got = conv[tuple(idx.T)]
        np.testing.assert_allclose(got, want, rtol=1e-11, atol=1e-11 * np.abs(want).max())
