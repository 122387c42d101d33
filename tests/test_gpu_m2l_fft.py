"""FFT form of M2L on the lattice layout (HIP) against the oracle's dense FMM of the same
layout (Section 3, density form) and the exact sum."""
import numpy as np
import pytest
import torch

from oracle import direct as odirect
from oracle import kifmm_ref
from paper_2006_03515_amd import embedding
from tests.gpu_common import gauss, rel_l2

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def K():
    from paper_2006_03515_amd import kifmm
    return kifmm


def setup(K, n, L, p_o2, max_leaf, rcond=1e-7):
    tree = K.build_tree(K.Grid.cube(n, L), max_leaf)
    ops = K.precompute_operators(tree, K.Kernel(p_o2), K.Opts(K.LAYOUT_LATTICE, 5, 10, rcond))
    return tree, ops


def run(K, tree, ops, I, precision, fft):
    ops.m2l_fft(fft)
    dt = torch.float64 if precision == "fp64" else torch.float32
    It = torch.tensor(np.ascontiguousarray(I), dtype=dt, device="cuda").reshape(-1)
    S = K.eval(tree, ops, It, 1.0, precision=precision)
    return S.double().cpu().numpy().reshape(I.shape)


@pytest.fixture(scope="module")
def g32():
    n, L = 32, 0.1
    I = gauss(n, L).astype(np.float32).astype(np.float64)
    return I, L, {p: odirect.fft_full(I, (L / n,) * 3, p) for p in (150.0, 1.974)}


@pytest.mark.parametrize("p_o2", [150.0, 1.974])
def test_lattice_layout_fp64_is_the_oracle(K, g32, p_o2):
    # dense M2L in FP64 against the oracle's density-form FMM of the same layout
    I, L, refs = g32
    tree, ops = setup(K, 32, L, p_o2, 64)
    got = run(K, tree, ops, I, "fp64", False)
    ora = kifmm_ref.evaluate(I, L, p_o2, ell=4, layout="lattice", m0=5, rcond=1e-7)
    assert rel_l2(got, ora) < max(1e-8, 0.05 * rel_l2(ora, refs[p_o2]))
    assert rel_l2(got, refs[p_o2]) < 1e-4


@pytest.mark.parametrize("p_o2", [150.0, 1.974])
def test_fft_m2l_is_the_dense_m2l(K, g32, p_o2):
    I, L, refs = g32
    tree, ops = setup(K, 32, L, p_o2, 64)
    ora = kifmm_ref.evaluate(I, L, p_o2, ell=4, layout="lattice", m0=5, rcond=1e-7)
    a = run(K, tree, ops, I, "fp32", True)
    b = run(K, tree, ops, I, "fp32", False)
    # FP32 FFT form against the oracle's FMM of the same layout: the benchmark spec's 1e-6
    # (measured 1.0e-7 at 150 Torr, 1.7e-7 at 1.974 Torr; the dense form 1.0-1.1e-7)
    assert rel_l2(a, b) < 1e-6
    assert rel_l2(a, ora) < 1e-6
    assert rel_l2(b, ora) < 1e-6
    # split BF16 products (about 16 mantissa bits per operand): measured 0.9-1.1e-6
    c = run(K, tree, ops, I, "bf16x3", True)
    assert rel_l2(c, ora) < 5e-6


@pytest.mark.parametrize("m0", [3, 4, 6, 7, 8])
def test_fft_m2l_other_lattice_sizes(K, g32, m0):
    # the separable lattice transforms for every supported lattice (N = 2 m0 - 1 = 5 .. 15):
    # the FFT form is the dense form of the same operators up to FP32 rounding
    I, L, refs = g32
    tree = K.build_tree(K.Grid.cube(32, L), 64)
    ops = K.precompute_operators(tree, K.Kernel(150.0), K.Opts(K.LAYOUT_LATTICE, m0, 10, 1e-7))
    a = run(K, tree, ops, I, "fp32", True)
    b = run(K, tree, ops, I, "fp32", False)
    assert rel_l2(a, b) < 2e-6
    assert rel_l2(a, refs[150.0]) < 1e-2


def test_fft_m2l_deep_tree_random_sources(K):
    # 128^3 with leaves of 8^3: M2L on levels 2..4 (up to 4096 boxes), random sources
    n, L, p_o2 = 128, 0.2, 150.0
    I = np.random.default_rng(41).random((n, n, n)).astype(np.float32).astype(np.float64)
    tree, ops = setup(K, n, L, p_o2, 512, rcond=1e-5)
    ora = kifmm_ref.evaluate(I, L, p_o2, ell=8, layout="lattice", m0=5, rcond=1e-5)
    a = run(K, tree, ops, I, "fp32", True)
    assert rel_l2(a, ora) < 1e-6          # measured 1.3e-7
    ref = odirect.fft_full(I, (L / n,) * 3, p_o2)
    assert rel_l2(a, ref) < 1e-4
    # split-BF16 parent-pair products (levels 3 and 4): about 16 mantissa bits per operand
    # (measured 3.6e-7 from the oracle's FMM)
    c = run(K, tree, ops, I, "bf16x3", True)
    assert rel_l2(c, ora) < 2e-6
    assert rel_l2(c, a) < 2e-6
    # single-part FP16 and BF16 parent-pair products: the formats' rounding (2^-11, 2^-8) on
    # the M2L part of the field (measured 2.8e-5 and 8.5e-5 from the oracle's FMM)
    h = run(K, tree, ops, I, "m2l_fp16", True)
    bb = run(K, tree, ops, I, "m2l_bf16", True)
    print("128^3 random sources, single-part pair products vs the oracle FMM: FP16 %.3e, BF16 %.3e"
          % (rel_l2(h, ora), rel_l2(bb, ora)))
    assert rel_l2(h, ora) < 1e-4
    assert rel_l2(bb, ora) < 4e-4


def test_fft_m2l_with_skipping_and_restriction(K):
    # zero-source skipping and target restriction keep the FFT form's values at the
    # wanted leaves bit for bit
    n, L, p_o2 = 64, 0.08, 150.0
    shape = (40, 24, 36)
    I = np.zeros((n, n, n), dtype=np.float32)
    I[:shape[0], :shape[1], :shape[2]] = np.random.default_rng(42).random(shape).astype(np.float32)
    tree, ops = setup(K, n, L, p_o2, 64, rcond=1e-5)
    It = torch.from_numpy(I.ravel()).cuda()
    a = K.eval(tree, ops, It, 1.0).reshape(n, n, n)
    ops.skip_zero_sources(True)
    b = K.eval(tree, ops, It, 1.0).reshape(n, n, n)
    assert float(torch.linalg.vector_norm(b - a) / torch.linalg.vector_norm(a)) < 2e-6
    m = embedding.leaf_mask(shape, n, tree.leaf_side)
    ops.restrict_targets(m)
    c = K.eval(tree, ops, It, 1.0).reshape(n, n, n)
    cells = torch.from_numpy(np.kron(m, np.ones((tree.leaf_side,) * 3, dtype=np.uint8)) != 0).cuda()
    assert torch.equal(c[cells], b[cells])
    assert int(torch.count_nonzero(c[~cells])) == 0


def test_fft_m2l_needs_the_lattice_layout(K):
    tree = K.build_tree(K.Grid.cube(32, 0.1), 64)
    ops = K.precompute_operators(tree, K.Kernel(150.0), K.Opts(K.LAYOUT_NESTED, 5, 10, 1e-5))
    ops.m2l_fft(False)
    with pytest.raises(K.KifmmError) as e:
        ops.m2l_fft(True)
    assert e.value.code == K.EUNSUPPORTED


@pytest.mark.parametrize("p,R,bar", [(760.0, 1.0, 3e-5), (760.0, 1.2, 6e-5), (100.0, 1.2, 6e-5), (10.0, 1.2, 6e-5)])
def test_streamer_256_full_size(K, p, R, bar, record_property):
    # the benchmark channel, 256^3 with leaves of 8^3, against the exact full field; the
    # FFT form and the dense form of the same layout agree to FP32 rounding
    from paper_2006_03515_amd import workloads
    w = workloads.streamer_channel(n=256, L=0.4, p=p)
    I = np.ascontiguousarray(w.I.astype(np.float32).ravel())
    tree = K.build_tree(K.Grid.cube(256, w.L), 512)
    ops = K.precompute_operators(tree, K.Kernel(w.p_o2), K.Opts(K.LAYOUT_LATTICE, 5, 10, 1e-5, R))
    It = torch.from_numpy(I).cuda()
    ops.m2l_fft(True)
    a = K.eval(tree, ops, It, w.prefactor).double().cpu().numpy()
    ops.m2l_fft(False)
    b = K.eval(tree, ops, It, w.prefactor).double().cpu().numpy()
    ref = odirect.fft_full(I.reshape(256, 256, 256).astype(np.float64), (w.h,) * 3, w.p_o2,
                           prefactor=w.prefactor, workers=16).ravel()
    e = rel_l2(a, ref)
    record_property("rel_l2_full", e)
    print("lattice R=%.1f, %g Torr: FFT form %.3e, dense form %.3e" % (R, p, e, rel_l2(b, ref)))
    assert rel_l2(a, b) < 2e-6
    assert e < bar
    # the single-part FP16 and BF16 parent-pair products on the same workload: FP16 stays
    # under 1e-4 over the whole field at every pressure (measured 1.8e-5 ... 7.0e-5), BF16
    # does not (1.2e-4 ... 6.3e-4)
    ops.m2l_fft(True)
    for prec, pbar in (("m2l_fp16", 1e-4), ("m2l_bf16", 1e-3)):
        c = K.eval(tree, ops, It, w.prefactor, precision=prec).double().cpu().numpy()
        ec = rel_l2(c, ref)
        record_property("rel_l2_full_" + prec, ec)
        print("  %s: %.3e (%.3e from the FP32 FFT form)" % (prec, ec, rel_l2(c, a)))
        assert ec < pbar
