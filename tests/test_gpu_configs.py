"""Full-size parity: the FMM at the benchmark configurations against the FP64
oracle evaluated one target at a time (sampled cells)."""
import numpy as np
import pytest
import torch

from oracle import direct as odirect
from paper_2006_03515_amd import workloads

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def K():
    from paper_2006_03515_amd import kifmm
    return kifmm


def _run(K, w, opts, precisions, max_leaf=512):
    I = np.ascontiguousarray(w.I.astype(np.float32).ravel())
    grid = K.Grid.cube(w.n, w.L)
    tree = K.build_tree(grid, max_leaf)
    ops = K.precompute_operators(tree, K.Kernel(w.p_o2), opts)
    It = torch.from_numpy(I).cuda()
    out = {}
    for p in precisions:
        x = It.double() if p == "fp64" else It
        out[p] = K.eval(tree, ops, x, w.prefactor, precision=p).double().cpu().numpy()
    return I, out


def _err(S, ref, tg):
    return float(np.linalg.norm(S[tg] - ref) / np.linalg.norm(ref))


@pytest.mark.parametrize("p", [760.0, 100.0])
def test_config2_128_two_heads(K, p, record_property):
    # 128^3 on 4 mm, two random heads (seed 8), 4,096 seeded targets (seed 1008)
    w = workloads.two_heads_random(n=128, L=0.4, p=p, seed=8)
    I, S = _run(K, w, K.Opts(K.LAYOUT_NESTED, 8, 10, 1e-7), ["fp32", "fp64"])
    tg = workloads.sample_targets(128 ** 3, 4096, seed=1008)
    ref = odirect.direct_targets(I.reshape(128, 128, 128).astype(np.float64), (w.h,) * 3, w.p_o2, tg,
                                 prefactor=w.prefactor)
    e32, e64 = _err(S["fp32"], ref, tg), _err(S["fp64"], ref, tg)
    record_property("rel_l2_fp32", e32)
    print("config 2, %g Torr, nested m0=8: fp32 %.3e fp64 %.3e" % (p, e32, e64))
    # the benchmark spec's FP32 bar (measured 2.8e-7 / 5.3e-7 at 760 / 100 Torr)
    assert e64 < 1e-6
    assert e32 < 1e-6


@pytest.mark.parametrize("p", [760.0, 100.0, 10.0])
def test_config3_256_streamer_all_precisions(K, p, record_property):
    # the benchmark configuration: 256^3, nested m0=5, rcond 1e-5, leaves 8^3, against
    # the exact full field (zero-padded FFT convolution of the FP64 oracle)
    w = workloads.streamer_channel(n=256, L=0.4, p=p)
    precs = ["fp32", "m2l_fp16", "m2l_bf16x3", "bf16x3", "m2l_bf16", "fp16", "bf16"]
    I, S = _run(K, w, K.Opts(K.LAYOUT_NESTED, 5, 10, 1e-5), precs)
    ref = odirect.fft_full(I.reshape(256, 256, 256).astype(np.float64), (w.h,) * 3, w.p_o2,
                           prefactor=w.prefactor, workers=16).ravel()
    errs = {q: float(np.linalg.norm(S[q] - ref) / np.linalg.norm(ref)) for q in precs}
    # and at single cells against the direct form of the oracle
    tg = workloads.sample_targets(256 ** 3, 64, seed=1009)
    d = odirect.direct_targets(I.reshape(256, 256, 256).astype(np.float64), (w.h,) * 3, w.p_o2, tg,
                               prefactor=w.prefactor)
    assert np.max(np.abs(ref[tg] / d - 1)) < 1e-10
    for q, e in errs.items():
        record_property("rel_l2_" + q, e)
    print("config 3, %g Torr, full field:" % p, {q: "%.2e" % e for q, e in errs.items()})
    for q in ("fp32", "m2l_bf16x3", "bf16x3"):
        assert errs[q] < 3e-5, q
    assert errs["m2l_fp16"] < 5e-5
    assert abs(errs["bf16x3"] - errs["fp32"]) < 0.2 * errs["fp32"]
    assert errs["m2l_bf16"] < 1e-3
    # every translation GEMM (P2M, M2M, M2L, L2L, L2P) with FP16 or BF16 operands: below the
    # format's unit roundoff, 2^-11 (FP16) and 2^-8 (BF16), and no better than FP32
    assert errs["fp32"] <= errs["fp16"] < 2.0 ** -11
    assert errs["fp32"] <= errs["bf16"] < 2.0 ** -8


def test_config3_256_accurate_layout_fp32_within_1e6(K):
    # nested m0 = 6, rcond 1e-7: the FP32 FMM within 1e-6 of the exact sum at 256^3
    w = workloads.streamer_channel(n=256, L=0.4, p=760.0)
    I, S = _run(K, w, K.Opts(K.LAYOUT_NESTED, 6, 10, 1e-7), ["fp32"])
    ref = odirect.fft_full(I.reshape(256, 256, 256).astype(np.float64), (w.h,) * 3, w.p_o2,
                           prefactor=w.prefactor, workers=16).ravel()
    e = float(np.linalg.norm(S["fp32"] - ref) / np.linalg.norm(ref))
    print("config 3 accurate layout, fp32 full field %.3e" % e)
    assert e < 1e-6
