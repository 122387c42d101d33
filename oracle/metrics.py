"""Error measures of Section 4, eq. (relativefun) (oracle; tests only).

E_V is returned as a fraction (the paper prints it times 100 %).
E_delta averages the pointwise relative error over the grid points within
distance delta of x0.
"""
import numpy as np


def rel_l2(num, ref):
    num = np.asarray(num, dtype=np.float64).ravel()
    ref = np.asarray(ref, dtype=np.float64).ravel()
    return float(np.linalg.norm(num - ref) / np.linalg.norm(ref))


def e_delta(num, ref, centres, x0, delta):
    """centres: (..., 3) array of the grid points matching num/ref."""
    num = np.asarray(num, dtype=np.float64).ravel()
    ref = np.asarray(ref, dtype=np.float64).ravel()
    c = np.asarray(centres, dtype=np.float64).reshape(-1, 3)
    inside = np.linalg.norm(c - np.asarray(x0), axis=1) <= delta
    if not inside.any():
        raise ValueError("no grid point within delta of x0")
    return float(np.mean(np.abs(num[inside] - ref[inside]) / ref[inside]))
