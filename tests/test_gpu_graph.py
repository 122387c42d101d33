"""One evaluation captured in a HIP graph (torch.cuda.CUDAGraph around kifmm_eval).

kifmm_eval allocates nothing, never synchronises the host and forks its side streams from
the calling stream (and joins them back) through events, so a capture on the calling
stream records the whole evaluation.  Every replay, with eager evaluations of other data
and synchronisations between the replays, must give the eager result bit for bit."""
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


@pytest.mark.parametrize("n,prec,m2l_fft,near_fft", [(64, "fp32", True, True), (64, "bf16x3", True, True),
                                                     (64, "fp32", False, False),
                                                     # depth 4: the coarse levels' M2L on the near
                                                     # field's stream, gated by per-level events
                                                     (128, "fp32", True, True), (128, "bf16x3", True, True),
                                                     # depth 5: the benchmark's schedule, levels 3
                                                     # and 4 each on a stream of its own
                                                     (256, "fp32", True, True), (256, "bf16x3", True, True)])
def test_graph_replay_is_the_eager_evaluation(K, n, prec, m2l_fft, near_fft):
    L, p_o2 = 0.1 * n / 64, 150.0
    I = np.random.default_rng(71).random((n, n, n)).astype(np.float32)
    tree = K.build_tree(K.Grid.cube(n, L), 512)
    ops = K.precompute_operators(tree, K.Kernel(p_o2), K.Opts(K.LAYOUT_LATTICE, 5, 10, 1e-5, 1.0))
    ops.m2l_fft(m2l_fft)
    ops.p2p_fft(near_fft)
    It = torch.from_numpy(I.ravel()).cuda()
    other = torch.flip(It, (0,)).contiguous()   # different data for the eager runs in between
    ref = K.eval(tree, ops, It, 1.0, precision=prec)
    torch.cuda.synchronize()
    S, T = torch.zeros_like(It), torch.empty_like(It)
    side = torch.cuda.Stream()   # warm-up off the capture, as torch asks
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        K.eval(tree, ops, It, 1.0, out=S, precision=prec)
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        K.eval(tree, ops, It, 1.0, out=S, precision=prec)
    torch.cuda.synchronize()
    for r in range(3):
        S.zero_()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(S, ref), "replay %d differs from the eager evaluation" % r
        K.eval(tree, ops, other, 1.0, out=T, precision=prec)
        torch.cuda.synchronize()
    exact = odirect.fft_full(I.astype(np.float64), (L / n,) * 3, p_o2).ravel()
    assert rel_l2(S.double().cpu().numpy(), exact) < 1e-4
    # a replay reads the input buffer as it is at replay time: new contents, new field
    ref_other = K.eval(tree, ops, other, 1.0, precision=prec)
    It.copy_(other)
    g.replay()
    torch.cuda.synchronize()
    assert torch.equal(S, ref_other)
    del g


@pytest.mark.parametrize("n,prec,m2l_fft", [(128, "fp32", False), (128, "bf16x3", False), (128, "fp64", False),
                                            # depth 5 with both Fourier forms: the schedule of the
                                            # benchmark (the finest level, level 3 and level 4 on
                                            # streams of their own)
                                            (256, "fp32", True), (256, "bf16x3", True)])
def test_serial_schedule_is_the_concurrent_evaluation(K, n, prec, m2l_fft):
    # every pass on the calling stream in order (the measurement schedule) runs the same
    # kernels on the same data: the same field bit for bit
    L, p_o2 = 0.2 * n / 128, 150.0
    I = np.random.default_rng(72).random((n, n, n))
    tree = K.build_tree(K.Grid.cube(n, L), 512)
    ops = K.precompute_operators(tree, K.Kernel(p_o2), K.Opts(K.LAYOUT_LATTICE, 5, 10, 1e-5, 1.0))
    ops.m2l_fft(m2l_fft)
    ops.p2p_fft(prec != "fp64")
    It = torch.from_numpy(I.ravel()).cuda()
    It = It if prec == "fp64" else It.float()
    a = K.eval(tree, ops, It, 1.0, precision=prec)
    ops.serial(True)
    b = K.eval(tree, ops, It, 1.0, precision=prec)
    ops.serial(False)
    c = K.eval(tree, ops, It, 1.0, precision=prec)
    torch.cuda.synchronize()
    assert torch.equal(a, b) and torch.equal(a, c)
