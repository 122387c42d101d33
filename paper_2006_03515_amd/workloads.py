"""Seeded synthetic inputs (source fields, pressures, target samples).

This module only draws inputs: it holds none of the method's arithmetic, and both
the GPU path and the CPU oracle take their inputs from it.  All randomness is
numpy Generator(PCG64(seed)).

Physical units: cm, Torr.  A source field is I(y) of eq. (Ifun) sampled at the
cell centres x0 + (i + 1/2) h of an n^3 grid spanning [0, L]^3.
"""
from dataclasses import dataclass
from functools import lru_cache

import numpy as np

P_Q = 30.0                # quenching pressure [Torr] (Section 4.1)
O2_FRACTION = 150.0 / 760.0


def p_o2_of(p):
    """Partial pressure of O2 at air pressure p, keeping 150 Torr at 760 Torr."""
    return p * O2_FRACTION


def quench(p):
    """p_q / (p + p_q): the quenching factor of eq. (Ifun)."""
    return P_Q / (p + P_Q)


@dataclass
class Workload:
    name: str
    n: int
    L: float           # cube side [cm]
    p: float           # air pressure [Torr]
    I: np.ndarray      # (n, n, n) float64 source

    @property
    def h(self):
        return self.L / self.n

    @property
    def p_o2(self):
        return p_o2_of(self.p)

    @property
    def prefactor(self):
        return quench(self.p)


def centres(n, L):
    return (np.arange(n) + 0.5) * (L / n)


def _mesh(n, L):
    c = centres(n, L)
    return np.meshgrid(c, c, c, indexing="ij")


@lru_cache(maxsize=4)
def _points(n, L):
    """(n^3, 3) cell centres in C order (cached, read-only)."""
    P = np.stack(_mesh(n, L), -1).reshape(-1, 3)
    P.setflags(write=False)
    return P


def _gauss_separable(n, L, c, sigma):
    """exp(-|r - c|^2 / sigma^2) on the grid as an outer product of three 1D factors."""
    x = centres(n, L)
    ex, ey, ez = (np.exp(-((x - c[a]) / sigma) ** 2) for a in range(3))
    return ex[:, None, None] * ey[None, :, None] * ez[None, None, :]


def gaussian_peak(n=32, L=0.1, amp=1e20, sigma=0.01, p=760.0):
    """One Gaussian 1e20 exp(-|r-c|^2/sigma^2) at the cube centre (1 mm cube, 32^3)."""
    I = amp * _gauss_separable(n, L, (L / 2,) * 3, sigma)
    return Workload("gaussian_peak_%d" % n, n, L, p, I)


def two_heads_random(n=128, L=0.4, p=760.0, seed=8):
    """Mixture of 2 Gaussian heads: centres U[L/4, 3L/4]^3, sigma U[0.005, 0.02] cm,
    amplitude log-uniform in [1e18, 1e21]."""
    rng = np.random.default_rng(seed)
    I = np.zeros((n, n, n))
    for _ in range(2):
        c = rng.uniform(L / 4, 3 * L / 4, 3)
        s = rng.uniform(0.005, 0.02)
        a = 10.0 ** rng.uniform(18, 21)
        I += a * _gauss_separable(n, L, c, s)
    return Workload("two_heads_%d" % n, n, L, p, I)


def streamer_channel(n=256, L=0.4, p=760.0, dtype=np.float32):
    """Elongated streamer channel: a cylinder of radius 0.01 cm along z through
    (L/2, L/2) for z in [L/8, 7L/8] (length 3 mm at L = 4 mm) with value 1e19, a
    Gaussian head sigma = 0.008 cm and peak 1e21 at its upper end, and a background
    of 1e15 (1e-6 of the peak)."""
    c = centres(n, L).astype(np.float64)
    X = c[:, None, None]
    Y = c[None, :, None]
    Z = c[None, None, :]
    I = np.full((n, n, n), 1e15, dtype=dtype)
    r2 = (X - L / 2) ** 2 + (Y - L / 2) ** 2           # (n, n, 1)
    zin = (Z >= L / 8) & (Z <= 7 * L / 8)              # (1, 1, n)
    cyl = (r2 <= 0.01 ** 2) & zin
    I[np.broadcast_to(cyl, I.shape)] += dtype(1e19)
    zh = 7 * L / 8
    for i in range(n):   # slab by slab to bound memory at 256^3
        d2 = (c[i] - L / 2) ** 2 + (Y[0] - L / 2) ** 2 + (Z[0] - zh) ** 2
        I[i] += (1e21 * np.exp(-d2 / 0.008 ** 2)).astype(dtype)
    return Workload("streamer_channel_%d" % n, n, L, p, I)


def anisotropic_heads(n=64, L=0.4, seed=40000, p=760.0):
    """1-4 anisotropic Gaussian heads: per-axis sigma U[0.003, 0.03] cm, a random
    rotation (QR of a normal 3x3 matrix, signs fixed so det = +1), log-uniform
    amplitude in [1e18, 1e21], centres U[L/4, 3L/4]^3."""
    rng = np.random.default_rng(seed)
    P = _points(n, L)
    I = np.zeros(n ** 3)
    for _ in range(int(rng.integers(1, 5))):
        s = rng.uniform(0.003, 0.03, 3)
        Q, R = np.linalg.qr(rng.standard_normal((3, 3)))
        Q = Q * np.sign(np.diag(R))
        if np.linalg.det(Q) < 0:
            Q[:, 0] = -Q[:, 0]
        a = 10.0 ** rng.uniform(18, 21)
        c = rng.uniform(L / 4, 3 * L / 4, 3)
        d = (P - c) @ (Q / s)
        d *= d
        I += a * np.exp(-d.sum(-1))
    return Workload("anisotropic_heads_%d_%d" % (n, seed), n, L, p, I.reshape(n, n, n))


def interacting_heads(k, n=128, L=0.4, steps=200, p=760.0):
    """Step k of two sigma = 0.01 cm Gaussian heads (peak 1e20 each) at
    (L/2, L/2, L/2 +- d_k/2), d_k shrinking linearly from 0.2 cm to 0.03 cm."""
    d = 0.2 - 0.17 * k / (steps - 1)
    c = L / 2
    I = np.zeros((n, n, n))
    for s in (-1, 1):
        I += 1e20 * _gauss_separable(n, L, (c, c, c + s * d / 2), 0.01)
    return Workload("interacting_heads_%d_%d" % (n, k), n, L, p, I)


def sample_targets(n_cells, count, seed):
    """`count` distinct flat cell indices drawn without replacement."""
    rng = np.random.default_rng(seed)
    return np.sort(rng.choice(n_cells, size=min(count, n_cells), replace=False)).astype(np.int64)


# ------------------------------------------------- the paper's Section 4 sources ----
XI = 0.1                  # xi of eq. (Ifun), Section 4.1
OMEGA_OVER_ALPHA = 0.6    # omega / alpha of eq. (Ifun), Section 4.1


@dataclass
class BoxWorkload:
    """A source on a box-shaped grid of isotropic cells (cell centres (i + 1/2) h)."""
    name: str
    shape: tuple
    h: float
    p: float
    p_o2: float
    prefactor: float      # I of eq. (Ifun) = prefactor * S_i
    S_i: np.ndarray       # ionization source on the grid
    x0: tuple             # centre of the local error ball [cm]
    delta: float          # its radius [cm]


def _box_centres(shape, h):
    return [(np.arange(m) + 0.5) * h for m in shape]


def paper_gaussian(case=1, dtype=np.float32):
    """Section 4.1: S_i = 1.53e25 exp(-|x - x0|^2 / sigma^2) on 320 x 320 x 160 cells,
    case 1: 0.4 x 0.4 x 0.2 cm, sigma = 0.01 cm; case 2: 0.04 x 0.04 x 0.02 cm,
    sigma = 0.001 cm; x0 the domain centre; 760 Torr, pO2 = 150 Torr, p_q = 30 Torr,
    xi = 0.1, omega/alpha = 0.6; error ball radius 5 sigma."""
    xd, zd, sigma = (0.4, 0.2, 0.01) if case == 1 else (0.04, 0.02, 0.001)
    shape = (320, 320, 160)
    h = xd / 320
    cx, cy, cz = _box_centres(shape, h)
    x0 = (xd / 2, xd / 2, zd / 2)
    ex, ey, ez = (np.exp(-((c - x0[a]) / sigma) ** 2) for a, c in enumerate((cx, cy, cz)))
    S = (1.53e25 * ex[:, None, None] * ey[None, :, None] * ez[None, None, :]).astype(dtype)
    return BoxWorkload("paper_gaussian_%d" % case, shape, h, 760.0, 150.0,
                       XI * OMEGA_OVER_ALPHA * quench(760.0), S, x0, 5 * sigma)


def paper_multipeak(dtype=np.float32):
    """Section 4.3: S_i = 1.53e25 sin^2(50 pi x) sin^2(50 pi y) sin^2(50 pi z) inside
    [x_d/4, 3x_d/4] x [y_d/4, 3y_d/4] x [z_d/4, 3z_d/4], zero outside, on the grid of
    Section 4.1 case 1; error ball radius 0.05 cm around the domain centre."""
    xd, zd = 0.4, 0.2
    shape = (320, 320, 160)
    h = xd / 320
    f = []
    for c, d in zip(_box_centres(shape, h), (xd, xd, zd)):
        v = np.sin(50 * np.pi * c) ** 2
        v[(c < d / 4) | (c > 3 * d / 4)] = 0.0
        f.append(v)
    S = (1.53e25 * f[0][:, None, None] * f[1][None, :, None] * f[2][None, None, :]).astype(dtype)
    return BoxWorkload("paper_multipeak", shape, h, 760.0, 150.0, XI * OMEGA_OVER_ALPHA * quench(760.0), S,
                       (xd / 2, xd / 2, zd / 2), 0.05)


@dataclass
class ColumnWorkload:
    """A source on a box of n x n x nz cells of hx = hy != hz (cell centres (i + 1/2) h)."""
    name: str
    shape: tuple
    h: tuple              # (hx, hy, hz) [cm]
    p: float
    p_o2: float
    prefactor: float
    I: np.ndarray
    x0: tuple             # centre of the local error ball [cm]
    delta: float


SPEED_OF_LIGHT = 2.99792458e10   # cm / s


def paper_pressure(p_o2, dtype=np.float32):
    """Section 4.2: I = 4 pi xi c exp(-|x - x_s|^2 / sigma^2) (I of eq. (Ifun) itself, so the
    prefactor is 1), xi = 0.1, sigma = 0.01 cm, on V = [0, 0.25] x [0, 0.25] x [0, 1.4] cm cut
    into 256 x 256 x 320 cells (hz = 4.48 hx); pO2 / p = 0.2; the source centre x_s and the
    error ball's centre x0 at the centre of V, delta = 0.05 cm."""
    shape = (256, 256, 320)
    ext = (0.25, 0.25, 1.4)
    h = tuple(e / m for e, m in zip(ext, shape))
    xc = tuple(e / 2 for e in ext)
    sigma = 0.01
    f = [np.exp(-(((np.arange(m) + 0.5) * hh - c) / sigma) ** 2) for m, hh, c in zip(shape, h, xc)]
    I = (4 * np.pi * XI * SPEED_OF_LIGHT * f[0][:, None, None] * f[1][None, :, None] * f[2][None, None, :]).astype(dtype)
    return ColumnWorkload("paper_pressure_%g" % p_o2, shape, h, p_o2 / 0.2, p_o2, 1.0, I, xc, 0.05)
