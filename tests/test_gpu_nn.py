"""Surrogate-network kernels (HIP) against the FP64 reference network."""
import numpy as np
import pytest
import torch

from oracle import conv3d_ref as C
from oracle import morton
from oracle import surrogate_ref as S

pytestmark = pytest.mark.gpu

KIND = {"conv3": 0, "down2": 1, "up2": 2, "point": 3}
TAPS = {"conv3": 27, "down2": 8, "up2": 8, "point": 1}


@pytest.fixture(scope="module")
def K():
    from paper_2006_03515_amd import kifmm
    return kifmm


def to_dev(xs):
    """list of [C, n, n, n] -> [B * n^3, C] Morton channels-last float32 CUDA tensor."""
    n = xs[0].shape[1]
    perm = morton.leaf_order(n, 1)
    a = np.concatenate([x.reshape(x.shape[0], -1)[:, perm].T for x in xs])
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.float32, device="cuda")


def from_dev(t, B, c, n):
    perm = morton.leaf_order(n, 1)
    a = t.reshape(B, n ** 3, c).double().cpu().numpy()
    out = []
    for s in range(B):
        g = np.empty((c, n ** 3))
        g[:, perm] = a[s].T
        out.append(g.reshape(c, n, n, n))
    return out


def rel(a, b):
    a, b = np.concatenate([x.ravel() for x in a]), np.concatenate([x.ravel() for x in b])
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def _layer_case(kind, ci, co, n_in, B, seed):
    rng = np.random.default_rng(seed)
    n_out = n_in // 2 if kind == "down2" else (2 * n_in if kind == "up2" else n_in)
    xs = [rng.standard_normal((ci, n_in, n_in, n_in)) for _ in range(B)]
    w = rng.standard_normal((TAPS[kind], co, ci)) / np.sqrt(TAPS[kind] * ci)
    gys = [rng.standard_normal((co, n_out, n_out, n_out)) for _ in range(B)]
    return xs, w, gys, n_out


@pytest.mark.parametrize("bf16,tol", [(0, 2e-6), (1, 2e-2)])
@pytest.mark.parametrize("kind,ci,co,n_in", [("conv3", 32, 32, 8), ("conv3", 64, 32, 16), ("down2", 32, 64, 8),
                                             ("up2", 64, 32, 4), ("up2", 128, 128, 4), ("point", 32, 64, 8),
                                             # operators of 96/160/192 rows: the 128-row staged tiles with
                                             # rows past M clamped; 16 output boxes: a ragged box tile
                                             ("conv3", 96, 96, 4), ("point", 96, 160, 2), ("down2", 96, 192, 4)])
def test_layer_forward_and_gradients(K, kind, ci, co, n_in, bf16, tol):
    B = 2
    xs, w, gys, n_out = _layer_case(kind, ci, co, n_in, B, seed=ci + co + n_in)
    f, fb = getattr(C, kind), getattr(C, kind + "_backward")
    w5 = S._w5(kind, w)
    ys = [f(x, w5) for x in xs]
    back = [fb(x, w5, gy) for x, gy in zip(xs, gys)]
    gxs = [b[0] for b in back]
    gw = S._w_back(kind, sum(b[1] for b in back))
    wt = torch.tensor(w.ravel(), dtype=torch.float32, device="cuda")
    dt = torch.bfloat16 if bf16 else torch.float32
    wf = torch.empty(w.size, dtype=dt, device="cuda")
    wb = torch.empty(w.size, dtype=dt, device="cuda")
    K.nn_call("kifmm_nn_prepare_weights", TAPS[kind], co, ci, wt, wf, wb, bf16)
    x = to_dev(xs)
    gy = to_dev(gys)
    work = torch.empty(1 << 22, dtype=torch.float32, device="cuda")
    y = torch.empty(B * n_out ** 3 * co, dtype=torch.float32, device="cuda")
    K.nn_call("kifmm_nn_layer_forward", KIND[kind], B, n_in, x, ci, wf, co, y, 0, bf16, work, work.numel())
    gx = torch.empty(B * n_in ** 3 * ci, dtype=torch.float32, device="cuda")
    K.nn_call("kifmm_nn_layer_backward_data", KIND[kind], B, n_in, gy, co, wb, ci, gx, 0, bf16, work, work.numel())
    gwd = torch.empty(w.size, dtype=torch.float32, device="cuda")
    if co % 32 == 0:
        K.nn_call("kifmm_nn_layer_backward_weight", KIND[kind], B, n_in, x, ci, gy, co, gwd, bf16, work,
                  work.numel())
    torch.cuda.synchronize()
    assert rel(from_dev(y, B, co, n_out), ys) < tol
    assert rel(from_dev(gx, B, ci, n_in), gxs) < tol
    if co % 32 == 0:
        assert rel([gwd.cpu().numpy().reshape(w.shape)], [gw]) < tol
    # accumulate = 1 adds to what is there
    y2 = y.clone()
    K.nn_call("kifmm_nn_layer_forward", KIND[kind], B, n_in, x, ci, wf, co, y2, 1, bf16, work, work.numel())
    torch.cuda.synchronize()
    assert rel(from_dev(y2, B, co, n_out), [2 * a for a in ys]) < tol


def test_elementwise_kernels(K):
    rng = np.random.default_rng(3)
    B, n, c = 2, 8, 32
    # bias + leaky and its backward with the bias gradient
    pre = rng.standard_normal((B * n ** 3, c)).astype(np.float32)
    bias = rng.standard_normal(c).astype(np.float32)
    y = torch.tensor(pre, device="cuda").reshape(-1)
    bt = torch.tensor(bias, device="cuda")
    K.nn_call("kifmm_nn_bias_act", B * n ** 3, c, y, bt, 0.1)
    ref = C.leaky(pre.astype(np.float64) + bias, 0.1)
    g = rng.standard_normal(ref.shape).astype(np.float32)
    gt = torch.tensor(g, device="cuda").reshape(-1)
    db = torch.empty(c, device="cuda")
    work = torch.empty(1 << 20, device="cuda")
    K.nn_call("kifmm_nn_bias_act_backward", B * n ** 3, c, y, gt, db, 0.1, work, work.numel())
    torch.cuda.synchronize()
    np.testing.assert_allclose(y.cpu().numpy().reshape(ref.shape), ref, rtol=1e-6, atol=1e-6)
    gpre = C.leaky_backward(pre.astype(np.float64) + bias, 0.1, g.astype(np.float64))
    np.testing.assert_allclose(gt.cpu().numpy().reshape(ref.shape), gpre, rtol=1e-6, atol=1e-7)
    np.testing.assert_allclose(db.cpu().numpy(), gpre.sum(0), rtol=1e-5, atol=1e-5)
    # input packing, output unpacking, maxima, resampling
    f = [rng.standard_normal((n, n, n)) for _ in range(B)]
    grid = torch.tensor(np.stack(f).ravel(), dtype=torch.float32, device="cuda")
    mx = torch.empty(B, device="cuda")
    K.nn_call("kifmm_nn_max_abs", B, n ** 3, grid, mx, 1, work, work.numel())
    feat = torch.empty(B * n ** 3 * 32, device="cuda")
    K.nn_call("kifmm_nn_pack_input", B, n, grid, mx, feat)
    torch.cuda.synchronize()
    inv = np.array([1 / np.abs(x.astype(np.float32)).max() for x in f])
    np.testing.assert_allclose(mx.cpu().numpy(), inv, rtol=1e-6)
    ref_feat = [C.neighbourhood27(x) * s for x, s in zip(f, inv)]
    assert rel(from_dev(feat, B, 32, n), ref_feat) < 1e-6
    out = torch.empty(B * n ** 3, device="cuda")
    K.nn_call("kifmm_nn_unpack_output", B, n, feat, 32, None, out)
    torch.cuda.synchronize()
    np.testing.assert_allclose(out.cpu().numpy(), np.stack([r[0] for r in ref_feat]).ravel(), rtol=1e-6, atol=1e-7)
    co = torch.empty(B * (n // 2) ** 3, device="cuda")
    K.nn_call("kifmm_nn_coarsen2", B, n // 2, grid, co)
    up = torch.empty(B * n ** 3, device="cuda")
    K.nn_call("kifmm_nn_upsample2", B, n // 2, co, up)
    torch.cuda.synchronize()
    cref = np.stack([C.coarsen2(x) for x in f])
    np.testing.assert_allclose(co.cpu().numpy(), cref.ravel(), rtol=1e-5, atol=1e-6)
    np.testing.assert_allclose(up.cpu().numpy(), np.stack([C.upsample2(c) for c in cref]).ravel(), rtol=1e-5,
                               atol=1e-6)


def _oracle_params(net):
    p = {}
    for name, kind, ci, co, act, skip in S.LAYERS:
        L = net.layers[name]
        p[name] = (L["w"].double().cpu().numpy().reshape(L["taps"], co, ci), L["b"].double().cpu().numpy())
    return p


@pytest.mark.parametrize("bf16,tol", [(0, 1e-4), (1, 5e-2)])
def test_network_loss_and_gradients(K, bf16, tol):
    from paper_2006_03515_amd.surrogate import Surrogate
    net = Surrogate(seed=1, bf16=bf16)
    rng = np.random.default_rng(4)
    B, n = 2, 8
    I = [np.abs(rng.standard_normal((n, n, n))) + 0.1 for _ in range(B)]
    T = [rng.standard_normal((n, n, n)) for _ in range(B)]
    It = torch.tensor(np.stack(I).ravel(), dtype=torch.float32, device="cuda")
    Tt = torch.tensor(np.stack(T).ravel(), dtype=torch.float32, device="cuda")
    loss = net.loss_and_backward(It, Tt, n, B)
    torch.cuda.synchronize()
    params = _oracle_params(net)
    Lref, grads, preds = 0.0, None, []
    for s in range(B):
        Is = I[s].astype(np.float32).astype(np.float64)
        feat = C.neighbourhood27(Is / np.abs(Is).max())
        pred, cache = S.forward(feat, params)
        preds.append(pred)
        _, g = C.rel_l2_loss([pred], [T[s].astype(np.float32).astype(np.float64)])
        gs = S.backward(cache, params, g[0] / B)
        grads = gs if grads is None else {k: (grads[k][0] + gs[k][0], grads[k][1] + gs[k][1]) for k in gs}
    Lref = np.mean([np.sum((p - t.astype(np.float32)) ** 2) / np.sum(t.astype(np.float32) ** 2)
                    for p, t in zip(preds, T)])
    assert loss[0].item() == pytest.approx(Lref, rel=tol)
    gpu = np.concatenate([np.concatenate([net.layers[nm]["gw"].double().cpu().numpy(),
                                          net.layers[nm]["gb"].double().cpu().numpy()]) for nm, *_ in S.LAYERS])
    ref = np.concatenate([np.concatenate([grads[nm][0].ravel(), grads[nm][1]]) for nm, *_ in S.LAYERS])
    assert np.linalg.norm(gpu - ref) / np.linalg.norm(ref) < tol


def test_training_reduces_loss_and_checkpoint_is_exact(K, tmp_path):
    from paper_2006_03515_amd.surrogate import Surrogate
    rng = np.random.default_rng(5)
    B, n = 2, 16
    I = torch.tensor(np.abs(rng.standard_normal((B, n, n, n))).ravel() + 0.1, dtype=torch.float32, device="cuda")
    T = torch.tensor(rng.standard_normal((B, n, n, n)).ravel(), dtype=torch.float32, device="cuda")

    def run(net, steps):
        out = []
        for _ in range(steps):
            out.append(net.loss_and_backward(I, T, n, B)[0].item())
            net.adam_step(1e-3)
        return out

    a = Surrogate(seed=2)
    la = run(a, 6)
    assert la[-1] < la[0]
    b = Surrogate(seed=2)
    run(b, 3)
    path = str(tmp_path / "ck.npz")
    b.save(path)
    c = Surrogate(seed=99)
    c.load(path)
    run(c, 3)
    assert torch.equal(a.master, c.master)
