"""Near field in Fourier space (HIP) against the dense near field and the oracle's exact
sum: the same sums of eq. (nearfar), direct part, up to FP32 rounding."""
import numpy as np
import pytest
import torch

from oracle import direct as odirect
from oracle import metrics
from paper_2006_03515_amd import embedding, workloads
from tests.gpu_common import rel_l2

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def K():
    from paper_2006_03515_amd import kifmm
    return kifmm


@pytest.mark.parametrize("n,layout", [(32, "nested"), (64, "nested"), (128, "lattice")])
def test_near_fft_is_the_dense_near_field(K, n, layout):
    # random sources; leaves of 8^3 (4 to 16 per axis); FP32 and split BF16 evaluations with
    # the near field in Fourier space against the dense near field and the exact sum
    L, p_o2 = n * 1.5625e-3, 150.0
    I = np.random.default_rng(50 + n).random((n, n, n)).astype(np.float32)
    tree = K.build_tree(K.Grid.cube(n, L), 512)
    lay = K.LAYOUT_NESTED if layout == "nested" else K.LAYOUT_LATTICE
    ops = K.precompute_operators(tree, K.Kernel(p_o2), K.Opts(lay, 5, 10, 1e-5))
    It = torch.from_numpy(I.ravel()).cuda()
    ref = odirect.fft_full(I.astype(np.float64), (L / n,) * 3, p_o2).ravel()
    for prec in ("fp32", "bf16x3"):
        ops.p2p_fft(False)
        a = K.eval(tree, ops, It, 1.0, precision=prec).double().cpu().numpy()
        ops.p2p_fft(True)
        b = K.eval(tree, ops, It, 1.0, precision=prec).double().cpu().numpy()
        assert rel_l2(b, a) < (1e-6 if prec == "fp32" else 1e-5), prec
        assert rel_l2(b, ref) < 1e-4
    ops.p2p_fft(False)


def test_near_fft_streamer_256(K, record_property):
    # the benchmark channel: a source spanning six orders of magnitude; the Fourier-space
    # near field against the dense one, whole field and at 4,096 sampled cells
    w = workloads.streamer_channel(n=256, L=0.4, p=760.0)
    tree = K.build_tree(K.Grid.cube(256, w.L), 512)
    ops = K.precompute_operators(tree, K.Kernel(w.p_o2), K.Opts(K.LAYOUT_LATTICE, 5, 10, 1e-5, 1.0))
    It = torch.from_numpy(np.ascontiguousarray(w.I.astype(np.float32).ravel())).cuda()
    a = K.eval(tree, ops, It, w.prefactor).double().cpu().numpy()
    ops.p2p_fft(True)
    b = K.eval(tree, ops, It, w.prefactor).double().cpu().numpy()
    tg = workloads.sample_targets(256 ** 3, 4096, seed=1009)
    full, samp = rel_l2(b, a), rel_l2(b[tg], a[tg])
    record_property("near_fft_vs_dense_full", full)
    print("near field in Fourier space vs dense: full %.2e, sampled %.2e" % (full, samp))
    assert full < 1e-6 and samp < 2e-6


def test_near_fft_with_skipping_and_restriction(K):
    n, L, p_o2 = 64, 0.1, 150.0
    shape = (40, 24, 36)
    I = np.zeros((n, n, n), dtype=np.float32)
    I[:shape[0], :shape[1], :shape[2]] = np.random.default_rng(52).random(shape).astype(np.float32)
    tree = K.build_tree(K.Grid.cube(n, L), 512)
    ops = K.precompute_operators(tree, K.Kernel(p_o2), K.Opts(K.LAYOUT_LATTICE, 5, 10, 1e-5))
    ops.p2p_fft(True)
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


def test_near_fft_needs_leaves_of_8(K):
    tree = K.build_tree(K.Grid.cube(32, 0.1), 64)
    ops = K.precompute_operators(tree, K.Kernel(150.0), K.Opts(K.LAYOUT_NESTED, 5, 10, 1e-5))
    ops.p2p_fft(False)
    with pytest.raises(K.KifmmError) as e:
        ops.p2p_fft(True)
    assert e.value.code == K.EUNSUPPORTED


def test_bright_sources_on_fine_cells_stay_finite(K):
    # the Section 4.1 case-2 regime: cells of 1.25 um and sources near 1.5e25; the cell volume
    # enters with the sources, so neither the spectra nor the dense sums leave FP32's range
    n, h, p_o2 = 32, 1.25e-4, 150.0
    I = (1.5e25 * (0.5 + 0.5 * np.random.default_rng(53).random((n, n, n)))).astype(np.float32)
    tree = K.build_tree(K.Grid.cube(n, n * h), 512)
    ops = K.precompute_operators(tree, K.Kernel(p_o2), K.Opts(K.LAYOUT_LATTICE, 5, 10, 1e-5))
    It = torch.from_numpy(I.ravel()).cuda()
    a = K.eval(tree, ops, It, 1.0).double().cpu().numpy()
    ops.p2p_fft(True)
    b = K.eval(tree, ops, It, 1.0).double().cpu().numpy()
    assert np.isfinite(a).all() and np.isfinite(b).all()
    assert rel_l2(b, a) < 1e-6
    ref = odirect.fft_full(I.astype(np.float64), (h,) * 3, p_o2).ravel()
    assert rel_l2(b, ref) < 1e-4


@pytest.mark.parametrize("p,R", [(760.0, 1.2), (100.0, 1.2), (10.0, 1.2), (760.0, 1.0)])
def test_benchmark_configuration_against_the_oracle(K, p, R, record_property):
    # exactly what bench.py times: the 256^3 channel, lattice layout (R = 1.2, the library
    # default, at each of the three pressures; R = 1.0 at 760 Torr), M2L in its FFT form,
    # near field in Fourier space, FP32; against the oracle's exact field (its FFT form,
    # checked at sampled cells against its one-target-at-a-time direct sum).  Bounds: the
    # whole field, bench.py's 4,096 cells (seed 1009), every leaf's own rel-L2 (an error
    # confined to a few dim leaves would hide in the whole-field norm: the worst leaves are
    # the background at the domain's faces, 0.7-3e-3 measured) and E_delta of eq.
    # (relativefun) within 5 sigma of the head.
    w = workloads.streamer_channel(n=256, L=0.4, p=p)
    I = np.ascontiguousarray(w.I.astype(np.float32).ravel())
    tree = K.build_tree(K.Grid.cube(256, w.L), 512)
    ops = K.precompute_operators(tree, K.Kernel(w.p_o2), K.Opts(K.LAYOUT_LATTICE, 5, 10, 1e-5, R))
    ops.m2l_fft(True)
    ops.p2p_fft(True)
    S = K.eval(tree, ops, torch.from_numpy(I).cuda(), w.prefactor).double().cpu().numpy()
    I3 = I.reshape(256, 256, 256).astype(np.float64)
    ref = odirect.fft_full(I3, (w.h,) * 3, w.p_o2, prefactor=w.prefactor, workers=16).ravel()
    t64 = workloads.sample_targets(256 ** 3, 64, seed=1010)
    d = odirect.direct_targets(I3, (w.h,) * 3, w.p_o2, t64, prefactor=w.prefactor)
    assert np.max(np.abs(ref[t64] / d - 1)) < 1e-10
    tg = workloads.sample_targets(256 ** 3, 4096, seed=1009)

    def bounds(X):
        dS = (X - ref).reshape(32, 8, 32, 8, 32, 8)
        rS = ref.reshape(32, 8, 32, 8, 32, 8)
        leaf = np.sqrt((dS ** 2).sum(axis=(1, 3, 5)) / (rS ** 2).sum(axis=(1, 3, 5)))
        c = (np.arange(256) + 0.5) * w.h
        x0, delta = (0.2, 0.2, 0.35), 5 * 0.008          # the head (sigma 0.008 cm)
        sub = tuple(slice(int(np.nonzero(np.abs(c - x0[a]) <= delta)[0][0]),
                          int(np.nonzero(np.abs(c - x0[a]) <= delta)[0][-1]) + 1) for a in range(3))
        cen = np.stack(np.meshgrid(*[c[s] for s in sub], indexing="ij"), -1)
        ed = metrics.e_delta(X.reshape(256, 256, 256)[sub], ref.reshape(256, 256, 256)[sub], cen, x0, delta)
        return rel_l2(X, ref), rel_l2(X[tg], ref[tg]), float(leaf.max()), ed

    full, samp, leaf, ed = bounds(S)
    for k, v in (("rel_l2_full", full), ("rel_l2_sampled", samp), ("max_leaf_rel_l2", leaf), ("E_delta_head", ed)):
        record_property(k, v)
    print("benchmark configuration %g Torr R %.1f: full field %.2e, 4,096 cells %.2e, worst leaf %.2e, "
          "E_delta(head) %.2e" % (p, R, full, samp, leaf, ed))
    assert full < 6e-5 and samp < 1e-4
    assert leaf < 5e-3 and ed < 2e-4
    # the mixed-precision form the bench reports beside it (split-BF16 M2L products):
    # within 1e-5 of the FP32 evaluation, and the same bars against the exact field
    Sx = K.eval(tree, ops, torch.from_numpy(I).cuda(), w.prefactor, precision="bf16x3").double().cpu().numpy()
    record_property("rel_l2_bf16x3_vs_fp32", rel_l2(Sx, S))
    assert rel_l2(Sx, S) < 1e-5
    fx, sx, lx, ex = bounds(Sx)
    assert fx < 6e-5 and sx < 1e-4 and lx < 5e-3 and ex < 2e-4
