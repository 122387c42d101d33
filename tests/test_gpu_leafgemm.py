"""P2M fused with the way into leaf order and L2P fused with the sum and the way out (FP32,
and split BF16 under KIFMM_BF16X3; leaves of 8^3 cells) against the same evaluation through
the separate permutes and tap GEMMs, which the library takes when the fields are not 16-byte
aligned."""
import numpy as np
import pytest
import torch

from oracle import direct as odirect
from tests.gpu_common import rel_l2

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def K():
    from paper_2006_03515_amd import kifmm
    return kifmm


def _offset_view(x, off=1):
    """The same values at a 4-byte offset from a 256-byte aligned allocation."""
    buf = torch.zeros(x.numel() + 4, dtype=x.dtype, device=x.device)
    v = buf[off:off + x.numel()]
    v.copy_(x)
    assert v.data_ptr() % 16 != 0
    return v


@pytest.mark.parametrize("n,layout,near_fft", [(32, "lattice", True), (64, "lattice", True), (64, "nested", False),
                                               (128, "lattice", True)])
def test_fused_leaf_passes_equal_the_separate_passes(K, n, layout, near_fft):
    L, p_o2 = 0.1 * n / 64, 150.0
    rng = np.random.default_rng(80 + n)
    I = (rng.random((n, n, n)) * np.exp(-8 * rng.random((n, n, n)))).astype(np.float32)
    tree = K.build_tree(K.Grid.cube(n, L), 512)
    lay = K.LAYOUT_LATTICE if layout == "lattice" else K.LAYOUT_NESTED
    ops = K.precompute_operators(tree, K.Kernel(p_o2), K.Opts(lay, 5, 10, 1e-5))
    ops.p2p_fft(near_fft)
    It = torch.from_numpy(I.ravel()).cuda()
    fused = K.eval(tree, ops, It, 0.7)                                   # both fused
    Im = _offset_view(It)
    sep_in = K.eval(tree, ops, Im, 0.7)                                  # separate way in and P2M
    Sm = _offset_view(torch.zeros_like(It))
    sep_out = K.eval(tree, ops, It, 0.7, out=Sm)                         # separate L2P and way out
    both = K.eval(tree, ops, Im, 0.7, out=_offset_view(torch.zeros_like(It)))
    f64 = K.eval(tree, ops, It.double(), 0.7, precision="fp64")          # tap GEMMs in FP64
    torch.cuda.synchronize()
    a = fused.double().cpu().numpy()
    for name, x in (("separate in", sep_in), ("separate out", sep_out), ("separate both", both)):
        e = rel_l2(a, x.double().cpu().numpy())
        print("%d^3 %s: fused vs %s %.2e" % (n, layout, name, e))
        assert e < 1e-6, name
    assert rel_l2(a, f64.cpu().numpy()) < 1e-6
    exact = odirect.fft_full(I.astype(np.float64), (L / n,) * 3, p_o2, prefactor=0.7).ravel()
    assert rel_l2(a, exact) < 1e-4


@pytest.mark.parametrize("precision", ["fp32", "bf16x3"])
def test_fused_way_out_honours_target_restriction(K, precision):
    # unwanted leaves are written as zeros by the fused way out too (FP32 and split-BF16
    # kernels); wanted ones keep the unrestricted values bit for bit
    n, L, p_o2 = 64, 0.1, 150.0
    I = np.random.default_rng(85).random((n, n, n)).astype(np.float32)
    tree = K.build_tree(K.Grid.cube(n, L), 512)
    ops = K.precompute_operators(tree, K.Kernel(p_o2), K.Opts(K.LAYOUT_LATTICE, 5, 10, 1e-5))
    ops.p2p_fft(True)
    It = torch.from_numpy(I.ravel()).cuda()
    a = K.eval(tree, ops, It, 1.0, precision=precision).reshape(n, n, n)
    nb = n // 8
    m = (np.random.default_rng(86).random((nb, nb, nb)) < 0.3).astype(np.uint8)
    ops.restrict_targets(m)
    b = K.eval(tree, ops, It, 1.0, precision=precision).reshape(n, n, n)
    ops.restrict_targets(None)
    cells = torch.from_numpy(np.kron(m, np.ones((8, 8, 8), dtype=np.uint8)) != 0).cuda()
    assert torch.equal(b[cells], a[cells])
    assert int(torch.count_nonzero(b[~cells])) == 0


@pytest.mark.parametrize("n,layout", [(32, "lattice"), (128, "lattice"), (64, "nested")])
def test_split_bf16_leaf_passes(K, n, layout, record_property):
    # KIFMM_BF16X3 runs the fused P2M and L2P in split BF16: each operand is its BF16 high part
    # plus the BF16 of the remainder (about 16 mantissa bits), and the dropped product of the
    # two remainders is below 2^-16 of each term.  Through the separate passes (fields not
    # 16-byte aligned) the same precision takes FP32 tap GEMMs for them, and KIFMM_M2L_BF16X3
    # takes the FP32 fused kernels: with the near field in Fourier space (FP32) in all three,
    # the fused split-BF16 field differs from the other two by the leaf passes' rounding only.
    L, p_o2 = 0.1 * n / 64, 150.0
    rng = np.random.default_rng(90 + n)
    I = (rng.random((n, n, n)) * np.exp(-8 * rng.random((n, n, n)))).astype(np.float32)
    tree = K.build_tree(K.Grid.cube(n, L), 512)
    lay = K.LAYOUT_LATTICE if layout == "lattice" else K.LAYOUT_NESTED   # nested: other KU, KD
    ops = K.precompute_operators(tree, K.Kernel(p_o2), K.Opts(lay, 5, 10, 1e-5))
    ops.m2l_fft(layout == "lattice")
    ops.p2p_fft(True)
    It = torch.from_numpy(I.ravel()).cuda()
    fused = K.eval(tree, ops, It, 0.7, precision="bf16x3")
    sep = K.eval(tree, ops, _offset_view(It), 0.7, out=_offset_view(torch.zeros_like(It)), precision="bf16x3")
    m2l_only = K.eval(tree, ops, It, 0.7, precision="m2l_bf16x3")
    fp32 = K.eval(tree, ops, It, 0.7)
    torch.cuda.synchronize()
    a = fused.double().cpu().numpy()
    e_sep, e_m2l = rel_l2(a, sep.double().cpu().numpy()), rel_l2(a, m2l_only.double().cpu().numpy())
    e_fp32 = rel_l2(a, fp32.double().cpu().numpy())
    record_property("rel_l2", {"vs_separate": e_sep, "vs_m2l_bf16x3": e_m2l, "vs_fp32": e_fp32})
    print("%d^3 %s split-BF16 leaf passes: vs FP32 leaf passes %.2e (separate) %.2e (fused), vs FP32 %.2e"
          % (n, layout, e_sep, e_m2l, e_fp32))
    assert 0 < e_sep < 2e-6 and 0 < e_m2l < 2e-6
    # against FP32 the M2L's split-BF16 products count too: the FFT form's parent-pair
    # products (lattice) or the dense translations (nested: 316 offsets per level)
    assert e_fp32 < (2e-6 if layout == "lattice" else 1e-5)
    exact = odirect.fft_full(I.astype(np.float64), (L / n,) * 3, p_o2, prefactor=0.7).ravel()
    assert rel_l2(a, exact) < 1e-4
