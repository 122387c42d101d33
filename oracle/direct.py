"""Exact discrete photoionization sum in FP64 (oracle; test infrastructure only).

The quantity is Section 3, eq. (summation), on a uniform grid of cell centres
(Section 4: V = V' = a box cut into nx*ny*nz equal cells):

    S_i = c * sum_j G(x_i, y_j) * I_j * (hx hy hz)

with G the discrete kernel of Section 3 (midpoint value off the diagonal, the
2x2x2 Gauss-Legendre self value on it) and c a caller prefactor (for example
xi p_q/(p+p_q) omega/alpha of eq. (Ifun)).

Three forms of the same sum:
  direct_numpy   plain loop over targets, vectorised over all sources (small grids)
  direct_targets the same loop in C with OpenMP (oracle/direct_sum.c)
  fft_full       the sum is a linear convolution of q = c I h^3 with the offset
                 table of G; a zero-padded FFT of size 2n per axis computes it for
                 every cell at once
"""
import ctypes
import os

import numpy as np
import scipy.fft

from . import kernel as _k

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle_direct.so")
_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            from . import build_oracle
            build_oracle.build()
        lib = ctypes.CDLL(_LIB_PATH)
        lib.oracle_direct_targets.argtypes = [
            ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
            ctypes.c_double, ctypes.c_double, ctypes.c_double,
            ctypes.c_void_p, ctypes.c_double, ctypes.c_double, ctypes.c_double,
            ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p]
        lib.oracle_direct_targets.restype = None
        lib.oracle_num_threads.restype = ctypes.c_int
        _lib = lib
    return _lib


def num_threads():
    """OpenMP threads the C direct sum runs with."""
    return int(_load().oracle_num_threads())


def weights(I, h, prefactor=1.0):
    """q = c * I * hx hy hz (Section 3: the cell volume multiplies I)."""
    return np.asarray(I, dtype=np.float64) * (prefactor * h[0] * h[1] * h[2])


def direct_numpy(I, h, p_o2, targets=None, prefactor=1.0):
    """Direct sum at flat target indices (all cells if None); numpy, small grids."""
    I = np.asarray(I, dtype=np.float64)
    nx, ny, nz = I.shape
    q = weights(I, h, prefactor).ravel()
    ii, jj, kk = np.meshgrid(np.arange(nx), np.arange(ny), np.arange(nz), indexing="ij")
    ii, jj, kk = ii.ravel(), jj.ravel(), kk.ravel()
    if targets is None:
        targets = np.arange(I.size)
    targets = np.asarray(targets, dtype=np.int64)
    G0 = _k.self_value(h[0], h[1], h[2], p_o2)
    out = np.empty(targets.size)
    for n_t, t in enumerate(targets):
        dx = (ii - ii[t]) * h[0]
        dy = (jj - jj[t]) * h[1]
        dz = (kk - kk[t]) * h[2]
        R = np.sqrt(dx * dx + dy * dy + dz * dz)
        R[t] = 1.0
        G = _k.K(R, p_o2)
        G[t] = G0
        out[n_t] = G @ q
    return out


def direct_targets(I, h, p_o2, targets, prefactor=1.0):
    """Direct sum at flat target indices, FP64 C/OpenMP (oracle/direct_sum.c)."""
    lib = _load()
    I = np.asarray(I, dtype=np.float64)
    nx, ny, nz = I.shape
    q = np.ascontiguousarray(weights(I, h, prefactor))
    tg = np.ascontiguousarray(np.asarray(targets, dtype=np.int64))
    out = np.empty(tg.size)
    a, b, ln = _k.coefficients(p_o2)
    lib.oracle_direct_targets(nx, ny, nz, h[0], h[1], h[2], q.ctypes.data, a, b, ln,
                              tg.ctypes.data, tg.size, out.ctypes.data)
    return out


def fft_full(I, h, p_o2, prefactor=1.0, workers=None):
    """The full field of the same sum by zero-padded FFT convolution.

    Per axis a of length n: S[i] = sum_j T[i - j + n - 1] q[j] with T the offset
    table of G (length 2n-1).  Placing T and q in arrays of length 2n per axis, the
    circular convolution at positions n-1 .. 2n-2 never wraps, so it equals the
    linear one.  Any box shape (nx, ny, nz).
    """
    I = np.asarray(I, dtype=np.float64)
    n = I.shape
    T = _k.offset_table(n, h, p_o2)
    M = tuple(2 * m for m in n)
    q = weights(I, h, prefactor)
    axes = (0, 1, 2)
    Fq = scipy.fft.rfftn(q, s=M, axes=axes, workers=workers)
    del q
    FT = scipy.fft.rfftn(T, s=M, axes=axes, workers=workers)
    del T
    Fq *= FT
    del FT
    full = scipy.fft.irfftn(Fq, s=M, axes=axes, workers=workers)
    del Fq
    return np.ascontiguousarray(full[n[0] - 1:2 * n[0] - 1, n[1] - 1:2 * n[1] - 1, n[2] - 1:2 * n[2] - 1])
