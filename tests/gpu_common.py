"""Shared helpers of the GPU tests (inputs from the workload generators; the
oracle is called only from the tests themselves)."""
import numpy as np

from paper_2006_03515_amd import workloads


def gauss(n, L, sigma=0.01, amp=1e20):
    return workloads.gaussian_peak(n=n, L=L, amp=amp, sigma=sigma).I


def rel_l2(a, b):
    a = np.asarray(a, dtype=np.float64).ravel()
    b = np.asarray(b, dtype=np.float64).ravel()
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))
