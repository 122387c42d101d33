"""CPU FP64 oracle for the photoionization integral and its KIFMM evaluation.

This package is TEST INFRASTRUCTURE. It exists to check the GPU library, and
only the test suite, the smoke check and the CPU-baseline leg of the benchmark
may import it. The product path (the HIP library and its Python binding) never
imports, links or calls anything here, and this package imports nothing from
the product.

Modules:
  kernel        absorption function g, kernel K = g/(4 pi R^2), self-cell value
  direct        the exact discrete sum (direct and FFT-convolution forms)
  closed_forms  continuum values at the centre of ball and Gaussian sources
  morton        Morton (Z-order) leaf ordering of a uniform grid
  kifmm_ref     a plain FP64 kernel-independent FMM following the paper's steps
  metrics       the relative errors E_V and E_delta
  conv3d_ref    FP64 3D convolution forward/backward for the surrogate network
"""
