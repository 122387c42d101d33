"""Thin Python binding of libkifmm (ctypes).  Argument marshalling only: every
step of the computation runs in the HIP library.

Functions keep the C names: build_tree, precompute_operators, eval (kifmm_eval),
direct_eval.  Device arrays are torch CUDA tensors; the work is enqueued on
torch's current stream.  If the library is missing this module raises at import.
"""
import ctypes
import os
from dataclasses import dataclass

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("KIFMM_LIB") or os.path.join(_HERE, "libkifmm.so")   # KIFMM_LIB: another build

OK, EINVAL, EUNSUPPORTED, EMISMATCH, ENOMEM, EHIP = 0, -1, -2, -3, -4, -5
LAYOUT_PAPER, LAYOUT_SINGLE, LAYOUT_NESTED, LAYOUT_LATTICE = 0, 1, 2, 3
FP64, FP32, M2L_BF16, M2L_FP16, M2L_BF16X3, BF16X3, BF16, FP16 = 0, 1, 2, 3, 4, 5, 6, 7
PRECISIONS = {"fp64": FP64, "fp32": FP32, "m2l_bf16": M2L_BF16, "m2l_fp16": M2L_FP16,
              "m2l_bf16x3": M2L_BF16X3, "bf16x3": BF16X3, "bf16": BF16, "fp16": FP16}
CHI_MIN, CHI_MAX = 0.035, 2.0

EXPORTS = ("kifmm_build_tree", "kifmm_precompute_operators", "kifmm_ops_rank", "kifmm_tree_info",
           "kifmm_eval", "direct_eval", "kifmm_tree_permutation", "kifmm_tree_destroy",
           "kifmm_ops_destroy", "kifmm_last_error", "kifmm_profile_enable", "kifmm_profile_read",
           "kifmm_ops_skip_zero_sources", "kifmm_ops_restrict_targets", "kifmm_ops_m2l_fft",
           "kifmm_ops_p2p_fft", "kifmm_ops_serial", "kifmm_tree_shape",
           "kifmm_nn_layer_forward", "kifmm_nn_layer_backward_data", "kifmm_nn_layer_backward_weight",
           "kifmm_nn_prepare_weights", "kifmm_nn_bias_act", "kifmm_nn_bias_act_backward",
           "kifmm_nn_rel_l2_loss", "kifmm_nn_adam", "kifmm_nn_pack_input", "kifmm_nn_unpack_output",
           "kifmm_nn_max_abs", "kifmm_nn_coarsen2", "kifmm_nn_upsample2", "kifmm_nn_sampled_rel_err",
           "kifmm_nn_sampled_rel_diff", "kifmm_nn_scale",
           "kifmm_nn_max_abs_noalloc")
NN_CONV3, NN_DOWN2, NN_UP2, NN_POINT = 0, 1, 2, 3
NN_TAPS = {NN_CONV3: 27, NN_DOWN2: 8, NN_UP2: 8, NN_POINT: 1}
PASSES = ("permute_in", "p2m", "m2m", "m2l", "l2l", "l2p", "p2p", "permute_out", "near_products")


class KifmmError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("libkifmm error %d: %s" % (code, msg))
        self.code = code


class _Grid(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
                ("x0", ctypes.c_double), ("y0", ctypes.c_double), ("z0", ctypes.c_double),
                ("hx", ctypes.c_double), ("hy", ctypes.c_double), ("hz", ctypes.c_double)]


class _Kernel(ctypes.Structure):
    _fields_ = [("chi_min", ctypes.c_double), ("chi_max", ctypes.c_double), ("p_o2", ctypes.c_double)]


class _Opts(ctypes.Structure):
    _fields_ = [("layout", ctypes.c_int32), ("m0", ctypes.c_int32), ("check_edge", ctypes.c_int32),
                ("rcond", ctypes.c_double), ("lattice_radius", ctypes.c_double)]


def load_library(path=LIB_PATH):
    if not os.path.exists(path):
        raise ImportError("libkifmm.so not built: run `python -m paper_2006_03515_amd.build_lib` "
                          "(looked for %s)" % path)
    lib = ctypes.CDLL(path)
    P = ctypes.c_void_p
    lib.kifmm_build_tree.argtypes = [ctypes.POINTER(_Grid), ctypes.c_int32, P, ctypes.POINTER(P)]
    lib.kifmm_precompute_operators.argtypes = [P, ctypes.POINTER(_Kernel), ctypes.POINTER(_Opts), P,
                                               ctypes.POINTER(P)]
    lib.kifmm_ops_rank.argtypes = [P, ctypes.c_int32, ctypes.POINTER(ctypes.c_int32),
                                   ctypes.POINTER(ctypes.c_int32)]
    lib.kifmm_tree_info.argtypes = [P, ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32)]
    lib.kifmm_tree_shape.argtypes = [P, ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32),
                                     ctypes.POINTER(ctypes.c_int32)]
    lib.kifmm_eval.argtypes = [P, P, P, ctypes.c_double, P, ctypes.c_int32, P]
    lib.direct_eval.argtypes = [ctypes.POINTER(_Grid), ctypes.POINTER(_Kernel), P, ctypes.c_double, P,
                                ctypes.c_int64, P, ctypes.c_int32, P]
    lib.kifmm_tree_permutation.argtypes = [P, P, P]
    lib.kifmm_tree_destroy.argtypes = [P]
    lib.kifmm_ops_destroy.argtypes = [P]
    lib.kifmm_last_error.restype = ctypes.c_char_p
    lib.kifmm_profile_enable.argtypes = [P, ctypes.c_int32]
    lib.kifmm_profile_read.argtypes = [P, P, P, ctypes.c_int32]
    lib.kifmm_ops_skip_zero_sources.argtypes = [P, ctypes.c_int32]
    lib.kifmm_ops_restrict_targets.argtypes = [P, P]
    lib.kifmm_ops_m2l_fft.argtypes = [P, ctypes.c_int32]
    lib.kifmm_ops_p2p_fft.argtypes = [P, ctypes.c_int32]
    lib.kifmm_ops_serial.argtypes = [P, ctypes.c_int32]
    I32, I64, F32, F64 = ctypes.c_int32, ctypes.c_int64, ctypes.c_float, ctypes.c_double
    nn = {
        "kifmm_nn_layer_forward": [I32, I32, I32, P, I32, P, I32, P, I32, I32, P, I64, P],
        "kifmm_nn_layer_backward_data": [I32, I32, I32, P, I32, P, I32, P, I32, I32, P, I64, P],
        "kifmm_nn_layer_backward_weight": [I32, I32, I32, P, I32, P, I32, P, I32, P, I64, P],
        "kifmm_nn_prepare_weights": [I32, I32, I32, P, P, P, I32, P],
        "kifmm_nn_bias_act": [I64, I32, P, P, F32, P],
        "kifmm_nn_bias_act_backward": [I64, I32, P, P, P, F32, P, I64, P],
        "kifmm_nn_rel_l2_loss": [I32, I32, P, I32, P, P, P, P, I64, P],
        "kifmm_nn_adam": [I64, P, P, P, P, I32, F32, F32, F32, F32, P],
        "kifmm_nn_pack_input": [I32, I32, P, P, P, P],
        "kifmm_nn_unpack_output": [I32, I32, P, I32, P, P, P],
        "kifmm_nn_max_abs": [I32, I64, P, P, I32, P, I64, P],
        "kifmm_nn_coarsen2": [I32, I32, P, P, P],
        "kifmm_nn_upsample2": [I32, I32, P, P, P],
        "kifmm_nn_sampled_rel_err": [I64, P, P, P, F64, P, P],
        "kifmm_nn_sampled_rel_diff": [I64, P, P, P, P, P],
        "kifmm_nn_scale": [I64, P, F32, P],
        "kifmm_nn_add": [I64, P, P, P],
        "kifmm_nn_max_abs_noalloc": [I32, I64, P, P, I32, P],
    }
    for f, a in nn.items():
        getattr(lib, f).argtypes = a
    for f in ("kifmm_build_tree", "kifmm_precompute_operators", "kifmm_ops_rank", "kifmm_tree_info",
              "kifmm_eval", "direct_eval", "kifmm_tree_permutation", "kifmm_profile_enable",
              "kifmm_profile_read") + tuple(nn):
        getattr(lib, f).restype = ctypes.c_int
    lib.kifmm_tree_destroy.restype = None
    lib.kifmm_ops_destroy.restype = None
    return lib


_lib = load_library()


def _check(rc):
    if rc != OK:
        raise KifmmError(rc, _lib.kifmm_last_error().decode())


def _stream(stream):
    if stream is not None:
        return ctypes.c_void_p(stream)
    if torch.cuda.is_available():
        return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    return ctypes.c_void_p(None)


@dataclass
class Grid:
    n: tuple          # (nx, ny, nz)
    h: tuple          # (hx, hy, hz) [cm]
    x0: tuple = (0.0, 0.0, 0.0)

    @staticmethod
    def cube(n, L):
        return Grid((n, n, n), (L / n,) * 3)

    def c(self):
        return _Grid(self.n[0], self.n[1], self.n[2], self.x0[0], self.x0[1], self.x0[2],
                     self.h[0], self.h[1], self.h[2])

    @property
    def N(self):
        return self.n[0] * self.n[1] * self.n[2]


@dataclass
class Kernel:
    p_o2: float
    chi_min: float = CHI_MIN
    chi_max: float = CHI_MAX

    def c(self):
        return _Kernel(self.chi_min, self.chi_max, self.p_o2)


@dataclass
class Opts:
    layout: int = LAYOUT_SINGLE
    m0: int = 6
    check_edge: int = 10
    rcond: float = 1e-7
    lattice_radius: float = 0.0     # layout LATTICE only; 0 = the library default (1.2)

    def c(self):
        return _Opts(self.layout, self.m0, self.check_edge, self.rcond, self.lattice_radius)


class Tree:
    def __init__(self, handle, grid):
        self.handle, self.grid = handle, grid
        d, e = ctypes.c_int32(), ctypes.c_int32()
        _check(_lib.kifmm_tree_info(handle, ctypes.byref(d), ctypes.byref(e)))
        self.depth, self.leaf_side = d.value, e.value
        ez, r = ctypes.c_int32(), ctypes.c_int32()
        _check(_lib.kifmm_tree_shape(handle, None, ctypes.byref(ez), ctypes.byref(r)))
        # leaf cells (x, y, z) and root cubes stacked along z (1 for a cubic grid)
        self.leaf_shape, self.roots = (e.value, e.value, ez.value), r.value
        nb = self.grid.n[0] // e.value
        self.leaves = (nb, nb, self.roots * nb)   # leaves per axis (the restriction mask's shape)

    def permutation(self, stream=None):
        out = torch.empty(self.grid.N, dtype=torch.int64, device="cuda")
        _check(_lib.kifmm_tree_permutation(self.handle, ctypes.c_void_p(out.data_ptr()), _stream(stream)))
        return out

    def __del__(self):
        h = getattr(self, "handle", None)
        if h and _lib is not None:
            _lib.kifmm_tree_destroy(h)
            self.handle = None


class Ops:
    def __init__(self, handle, tree):
        self.handle, self.tree = handle, tree

    def rank(self, level):
        ku, kd = ctypes.c_int32(), ctypes.c_int32()
        _check(_lib.kifmm_ops_rank(self.handle, level, ctypes.byref(ku), ctypes.byref(kd)))
        return ku.value, kd.value

    def skip_zero_sources(self, enable=True):
        """Skip taps whose source boxes hold only zeros in later eval() calls (same sum)."""
        _check(_lib.kifmm_ops_skip_zero_sources(self.handle, 1 if enable else 0))

    def m2l_fft(self, enable=True):
        """FFT form of M2L (lattice layout only; on by default there) or the dense M2L."""
        _check(_lib.kifmm_ops_m2l_fft(self.handle, 1 if enable else 0))

    def p2p_fft(self, enable=True):
        """Near field in Fourier space (leaves of 8^3) or the dense near field."""
        _check(_lib.kifmm_ops_p2p_fft(self.handle, 1 if enable else 0))

    def serial(self, enable=True):
        """Run every pass of eval() on the calling stream in order (per-kernel timings
        without overlap; the same results bit for bit)."""
        _check(_lib.kifmm_ops_serial(self.handle, 1 if enable else 0))

    def restrict_targets(self, leaf_mask=None):
        """Evaluate only at the leaves marked in leaf_mask (array of the tree's leaves per
        axis, tree.leaves, C order over leaf coordinates, nonzero = wanted); later eval()
        calls return 0 elsewhere.  None evaluates every target again."""
        if leaf_mask is None:
            _check(_lib.kifmm_ops_restrict_targets(self.handle, None))
            return
        nl = int(np.prod(self.tree.leaves))
        m = np.ascontiguousarray(np.asarray(leaf_mask).reshape(-1) != 0, dtype=np.uint8)
        if m.size != nl:
            raise ValueError("leaf_mask has %d values, the tree has %d leaves" % (m.size, nl))
        _check(_lib.kifmm_ops_restrict_targets(self.handle, ctypes.c_void_p(m.ctypes.data)))

    def profile(self, on=True):
        """Start (clearing old sums) or stop per-pass event timing of eval()."""
        _check(_lib.kifmm_profile_enable(self.handle, 1 if on else 0))

    def profile_read(self):
        """{pass: (total ms, launches)} since profile(True)."""
        n = len(PASSES)
        ms = (ctypes.c_double * n)()
        calls = (ctypes.c_int64 * n)()
        _check(_lib.kifmm_profile_read(self.handle, ctypes.cast(ms, ctypes.c_void_p),
                                       ctypes.cast(calls, ctypes.c_void_p), n))
        return {p: (ms[i], calls[i]) for i, p in enumerate(PASSES)}

    def __del__(self):
        h = getattr(self, "handle", None)
        if h and _lib is not None:
            _lib.kifmm_ops_destroy(h)
            self.handle = None


def build_tree(grid, max_leaf=64, stream=None):
    h = ctypes.c_void_p()
    _check(_lib.kifmm_build_tree(ctypes.byref(grid.c()), int(max_leaf), _stream(stream), ctypes.byref(h)))
    return Tree(h, grid)


def precompute_operators(tree, kernel, opts=None, stream=None):
    h = ctypes.c_void_p()
    o = ctypes.byref(opts.c()) if opts is not None else None
    _check(_lib.kifmm_precompute_operators(tree.handle, ctypes.byref(kernel.c()), o, _stream(stream),
                                           ctypes.byref(h)))
    return Ops(h, tree)


def eval(tree, ops, I, prefactor=1.0, out=None, precision=FP32, stream=None):
    """S = prefactor * sum_j G I_j h^3 by the FMM.  I: CUDA tensor (float32, or
    float64 for precision FP64) in grid order; returns S of the same dtype/shape."""
    precision = PRECISIONS.get(precision, precision)
    want = torch.float64 if precision == FP64 else torch.float32
    if I.dtype != want or not I.is_cuda or not I.is_contiguous():
        raise ValueError("I must be a contiguous CUDA tensor of dtype %s" % want)
    if I.numel() != tree.grid.N:
        raise ValueError("I has %d values, grid has %d" % (I.numel(), tree.grid.N))
    if out is None:
        out = torch.empty_like(I)
    _check(_lib.kifmm_eval(tree.handle, ops.handle, ctypes.c_void_p(I.data_ptr()), float(prefactor),
                           ctypes.c_void_p(out.data_ptr()), int(precision), _stream(stream)))
    return out


def direct_eval(grid, kernel, I, prefactor=1.0, tgt_idx=None, out=None, fp64=True, stream=None):
    """Exact sum at flat target indices (CUDA int64 tensor) or at every cell."""
    if I.dtype != torch.float32 or not I.is_cuda or not I.is_contiguous():
        raise ValueError("I must be a contiguous CUDA float32 tensor")
    n_tgt = grid.N if tgt_idx is None else tgt_idx.numel()
    if tgt_idx is not None and (tgt_idx.dtype != torch.int64 or not tgt_idx.is_cuda):
        raise ValueError("tgt_idx must be a CUDA int64 tensor")
    if out is None:
        out = torch.empty(n_tgt, dtype=torch.float64, device=I.device)
    tp = ctypes.c_void_p(tgt_idx.data_ptr()) if tgt_idx is not None else ctypes.c_void_p(None)
    _check(_lib.direct_eval(ctypes.byref(grid.c()), ctypes.byref(kernel.c()), ctypes.c_void_p(I.data_ptr()),
                            float(prefactor), tp, int(n_tgt), ctypes.c_void_p(out.data_ptr()),
                            1 if fp64 else 0, _stream(stream)))
    return out


# ------------------------------------------------------------- surrogate layers
def _p(t):
    return ctypes.c_void_p(t.data_ptr() if t is not None else None)


def nn_call(name, *args):
    """Call a kifmm_nn_* entry point: tensors become device pointers, the last
    argument is torch's current stream."""
    conv = []
    for a in args:
        if isinstance(a, torch.Tensor):
            conv.append(_p(a))
        elif a is None:
            conv.append(ctypes.c_void_p(None))
        else:
            conv.append(a)
    _check(getattr(_lib, name)(*conv, _stream(None)))
