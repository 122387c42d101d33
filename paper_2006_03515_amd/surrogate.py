"""Learned surrogate of the photoionization map I -> S_ph (not in the paper).

A 3D convolutional encoder-decoder (4 resolution levels, 32 -> 128 channels,
about 1.15 M parameters) maps a source field, normalised by its maximum, to
S_ph / max|I|.  S is linear in I, so the normalisation is exact and the network
only has to learn the shape of the response.  It is trained on (I, S) pairs
produced by kifmm_eval on the GPU, and in serving its output is checked on
sampled targets against direct_eval, with kifmm_eval as the fallback.

Every numeric step runs in libkifmm (kifmm_nn_* layer kernels on MFMA, BF16
operands with FP32 master weights); this module only sequences the calls and
owns the device buffers.

Layers (name, kind, in channels, out channels, input level, leaky ReLU, skip):
  in   POINT  32 -> 32   on the 27-neighbourhood features of the input (a 3x3x3 conv)
  e0   CONV3  32 -> 32   level 0 (n)
  d1   DOWN2  32 -> 64   n -> n/2
  e1   CONV3  64 -> 64
  d2   DOWN2  64 -> 128  n/2 -> n/4
  e2   CONV3 128 -> 128
  d3   DOWN2 128 -> 128  n/4 -> n/8
  u2   UP2   128 -> 128  n/8 -> n/4, + e2
  u1   UP2   128 -> 64   n/4 -> n/2, + e1
  b1   CONV3  64 -> 64
  u0   UP2    64 -> 32   n/2 -> n,   + e0
  b0   CONV3  32 -> 32
  head POINT  32 -> 32   channel 0 is the prediction (no activation)
A skip is added before the bias and activation: y = leaky(W x + s + b).
"""
import numpy as np
import torch

from . import kifmm as K

ALPHA = 0.1
ARCH = [
    ("in", K.NN_POINT, 32, 32, 0, True, None),
    ("e0", K.NN_CONV3, 32, 32, 0, True, None),
    ("d1", K.NN_DOWN2, 32, 64, 0, True, None),
    ("e1", K.NN_CONV3, 64, 64, 1, True, None),
    ("d2", K.NN_DOWN2, 64, 128, 1, True, None),
    ("e2", K.NN_CONV3, 128, 128, 2, True, None),
    ("d3", K.NN_DOWN2, 128, 128, 2, True, None),
    ("u2", K.NN_UP2, 128, 128, 3, True, "e2"),
    ("u1", K.NN_UP2, 128, 64, 2, True, "e1"),
    ("b1", K.NN_CONV3, 64, 64, 1, True, None),
    ("u0", K.NN_UP2, 64, 32, 1, True, "e0"),
    ("b0", K.NN_CONV3, 32, 32, 0, True, None),
    ("head", K.NN_POINT, 32, 32, 0, False, None),
]
HEAD_LD = 32


def out_level(kind, level):
    return level + 1 if kind == K.NN_DOWN2 else (level - 1 if kind == K.NN_UP2 else level)


class Surrogate:
    """Parameters, optimizer state and work buffers on one GPU."""

    def __init__(self, seed=0, bf16=True, device="cuda", work_floats=64 << 20):
        self.bf16 = bool(bf16)
        self.dev = torch.device(device)
        shapes = []
        for name, kind, ci, co, lev, act, skip in ARCH:
            shapes.append((name, K.NN_TAPS[kind], co, ci))
        self.nparams = sum(t * co * ci + co for _, t, co, ci in shapes)
        f32 = dict(dtype=torch.float32, device=self.dev)
        self.master = torch.zeros(self.nparams, **f32)
        self.grad = torch.zeros(self.nparams, **f32)
        self.m = torch.zeros(self.nparams, **f32)
        self.v = torch.zeros(self.nparams, **f32)
        self.step = 0
        self.layers = {}
        rng = np.random.default_rng(seed)
        init = np.zeros(self.nparams, dtype=np.float32)
        off = 0
        wdt = torch.bfloat16 if self.bf16 else torch.float32
        for (name, kind, ci, co, lev, act, skip), (_, taps, _, _) in zip(ARCH, shapes):
            nw = taps * co * ci
            fan_in = taps * ci
            gain = np.sqrt(2.0 / (1 + ALPHA ** 2)) if act else 0.1
            init[off:off + nw] = rng.standard_normal(nw) * gain / np.sqrt(fan_in)
            self.layers[name] = dict(kind=kind, ci=ci, co=co, level=lev, act=act, skip=skip, taps=taps,
                                     w=self.master[off:off + nw], b=self.master[off + nw:off + nw + co],
                                     gw=self.grad[off:off + nw], gb=self.grad[off + nw:off + nw + co],
                                     wf=torch.empty(nw, dtype=wdt, device=self.dev),
                                     wb=torch.empty(nw, dtype=wdt, device=self.dev))
            off += nw + co
        self.master.copy_(torch.from_numpy(init))
        self.work = torch.empty(work_floats, **f32)
        self.dwork = torch.empty(1 << 16, dtype=torch.float64, device=self.dev)
        self.loss_buf = torch.zeros(1 + 256, dtype=torch.float64, device=self.dev)
        self.scale = torch.empty(256, **f32)
        self._cache = {}
        self.refresh()

    # ------------------------------------------------------------ weights ----
    def refresh(self):
        """Copies of the FP32 masters used by the layer kernels (BF16 or FP32)."""
        for L in self.layers.values():
            K.nn_call("kifmm_nn_prepare_weights", L["taps"], L["co"], L["ci"], L["w"], L["wf"], L["wb"],
                      1 if self.bf16 else 0)

    def state_dict(self):
        return {"master": self.master.cpu().numpy(), "m": self.m.cpu().numpy(), "v": self.v.cpu().numpy(),
                "step": np.array(self.step), "bf16": np.array(int(self.bf16))}

    def load_state_dict(self, d):
        for k in ("master", "m", "v"):
            getattr(self, k).copy_(torch.from_numpy(np.asarray(d[k], dtype=np.float32)))
        self.step = int(d["step"])
        self.refresh()

    def save(self, path):
        np.savez(path, **self.state_dict())

    def load(self, path):
        with np.load(path, allow_pickle=False) as d:
            self.load_state_dict(dict(d))

    # -------------------------------------------------------------- buffers --
    def _buffers(self, batch, n):
        key = (batch, n)
        if key not in self._cache:
            f32 = dict(dtype=torch.float32, device=self.dev)
            bufs = {"feat": torch.empty(batch * n ** 3 * 32, **f32)}
            for name, kind, ci, co, lev, act, skip in ARCH:
                side = n >> out_level(kind, lev)
                bufs[name] = torch.empty(batch * side ** 3 * co, **f32)
                bufs["g_" + name] = torch.empty(batch * side ** 3 * co, **f32)
            self._cache = {key: bufs}   # keep one shape at a time
        return self._cache[key]

    # -------------------------------------------------------------- forward --
    def forward(self, I, n, batch, scale=None):
        """I: [batch * n^3] FP32 grid-ordered sources.  Returns the head buffer
        (Morton order, HEAD_LD channels) in units of S / max|I| (or scale * I when
        `scale` gives the per-sample input multipliers)."""
        if n < 8 or n & (n - 1):
            raise ValueError("grid side must be a power of two >= 8")
        B = self._buffers(batch, n)
        if scale is None:
            K.nn_call("kifmm_nn_max_abs", batch, n ** 3, I, self.scale, 1, self.work, self.work.numel())
            scale = self.scale
        K.nn_call("kifmm_nn_pack_input", batch, n, I, scale, B["feat"])
        x = B["feat"]
        bf = 1 if self.bf16 else 0
        for name, kind, ci, co, lev, act, skip in ARCH:
            L = self.layers[name]
            y = B[name]
            acc = 0
            if skip is not None:
                y.copy_(B[skip])
                acc = 1
            K.nn_call("kifmm_nn_layer_forward", kind, batch, n >> lev, x, ci, L["wf"], co, y, acc, bf,
                      self.work, self.work.numel())
            nvox = y.numel() // co
            K.nn_call("kifmm_nn_bias_act", nvox, co, y, L["b"], ALPHA if act else 1.0)
            x = y
        return B["head"]

    def predict(self, I, n, batch, out):
        """out[batch * n^3] (grid order) = predicted S for sources I (same units as I * h^3-weighted S)."""
        head = self.forward(I, n, batch)
        K.nn_call("kifmm_nn_max_abs", batch, n ** 3, I, self.scale, 0, self.work, self.work.numel())
        K.nn_call("kifmm_nn_unpack_output", batch, n, head, HEAD_LD, self.scale, out)
        return out

    # ------------------------------------------------------------- training --
    def loss_and_backward(self, I, T, n, batch):
        """Squared relative L2 loss of the prediction against targets T (grid order,
        already divided by max|I| per sample) and gradients into self.grad."""
        B = self._buffers(batch, n)
        head = self.forward(I, n, batch)
        K.nn_call("kifmm_nn_rel_l2_loss", batch, n, head, HEAD_LD, T, B["g_head"], self.loss_buf, self.dwork,
                  self.dwork.numel())
        bf = 1 if self.bf16 else 0
        have = {"head": True}
        names = [a[0] for a in ARCH]
        for idx in range(len(ARCH) - 1, -1, -1):
            name, kind, ci, co, lev, act, skip = ARCH[idx]
            L = self.layers[name]
            y, gy = B[name], B["g_" + name]
            nvox = y.numel() // co
            K.nn_call("kifmm_nn_bias_act_backward", nvox, co, y, gy, L["gb"], ALPHA if act else 1.0,
                      self.work, self.work.numel())
            x = B[names[idx - 1]] if idx > 0 else B["feat"]
            K.nn_call("kifmm_nn_layer_backward_weight", kind, batch, n >> lev, x, ci, gy, co, L["gw"], bf,
                      self.work, self.work.numel())
            if skip is not None:
                gs = B["g_" + skip]
                if have.get(skip):
                    K.nn_call("kifmm_nn_add", gy.numel(), gy, gs)
                else:
                    gs.copy_(gy)
                    have[skip] = True
            if idx > 0:
                prev = names[idx - 1]
                gx = B["g_" + prev]
                acc = 1 if have.get(prev) else 0
                K.nn_call("kifmm_nn_layer_backward_data", kind, batch, n >> lev, gy, co, L["wb"], ci, gx, acc, bf,
                          self.work, self.work.numel())
                have[prev] = True
        return self.loss_buf

    def adam_step(self, lr, b1=0.9, b2=0.999, eps=1e-8):
        self.step += 1
        K.nn_call("kifmm_nn_adam", self.nparams, self.master, self.grad, self.m, self.v, self.step, float(lr),
                  float(b1), float(b2), float(eps))
        self.refresh()
