"""Training and time-stepped serving of the learned surrogate.

    python -m paper_2006_03515_amd.surrogate_tasks train [--n-train 2000] [--epochs 20] ...
    python -m paper_2006_03515_amd.surrogate_tasks serve --checkpoint ck.npz [--steps 200] ...

train: 2,000 seeded fields on a 64^3 grid (4 mm cube), each 1-4 anisotropic Gaussian
heads (workloads.anisotropic_heads, seeds 40000 + i), targets S_ph from kifmm_eval on
the GPU (nested layout, FP32) at 760 Torr, divided by max|I| per field (S is linear
in I).  Adam on FP32 master weights, BF16 MFMA products, squared relative-L2 loss.
200 held-out fields (seeds 42000 + i) are judged against the FMM.

serve: 200 steps of two interacting heads on a 128^3 grid (workloads.interacting_heads).
Per step (Served): 2x2x2 block-mean coarsening to 64^3, surrogate inference, trilinear
upsampling to 128^3, relative error at 1,024 sampled cells against the FMM evaluated at
those cells' leaves (the judge), and kifmm_eval on the 128^3 grid whenever that error
exceeds the tolerance.  The FMM-only loop (the same fast configuration) is timed beside
it.

Both print one JSON line; progress goes to stderr.
"""
import argparse
import json
import multiprocessing
import sys
import time
from concurrent.futures import ProcessPoolExecutor

import numpy as np

from . import workloads

L_CM = 0.4
P_TORR = 760.0
OPTS = dict(layout=2, m0=5, check_edge=10, rcond=1e-5)          # training targets (64^3)
FAST_OPTS = dict(layout=3, m0=5, check_edge=10, rcond=1e-5, lattice_radius=1.2)
LAST_NET = None   # the network of the last train() call in this process


def log(*a):
    print("[surrogate]", *a, file=sys.stderr, flush=True)


def _field(seed):
    return workloads.anisotropic_heads(n=64, L=L_CM, seed=seed, p=P_TORR).I.astype(np.float32).ravel()


def make_fields(seeds, workers=8):
    # the workers are spawned, never forked: the calling process may already have initialised
    # the GPU runtime (through torch or through the library's own HIP calls), and a forked
    # copy of it is unusable
    if workers <= 1:
        return np.stack([_field(s) for s in seeds])
    with ProcessPoolExecutor(max_workers=workers, mp_context=multiprocessing.get_context("spawn")) as ex:
        return np.stack(list(ex.map(_field, seeds, chunksize=16)))


def fast_fmm(K, tree, kern):
    """The library's fastest configuration at the 1e-4 bar: lattice layout (R = 1.2) with M2L
    in its FFT form and the near field in Fourier space (leaves of 8^3)."""
    ops = K.precompute_operators(tree, kern, K.Opts(**FAST_OPTS))
    ops.m2l_fft(True)
    ops.p2p_fft(True)
    return ops


class Served:
    """Serving one field per step with the FMM as judge and fallback.

    step(I, S): 2x2x2 block means down to 64^3, inference, trilinear upsampling back to
    the grid (S = the prediction, times the prefactor); then the FMM evaluated only at the
    leaves of the sampled targets (the judge: kifmm_ops_restrict_targets) and the relative
    error of the prediction at those targets (kifmm_nn_sampled_rel_diff; the step's one
    device-to-host copy); above the tolerance S is replaced by the full FMM evaluation.
    The judge and the fallback use the library's fastest configuration."""

    def __init__(self, K, net, tree, kern, tol, n_net=64):
        import torch
        self.K, self.net, self.tree, self.tol = K, net, tree, tol
        self.fmm = fast_fmm(K, tree, kern)
        self.judge = fast_fmm(K, tree, kern)
        n = tree.grid.n[0]
        self.n, self.n_net = n, n_net
        dev = torch.device("cuda")
        self.levels = []
        m = n
        while m > n_net:
            m //= 2
            self.levels.append(torch.empty(m ** 3, dtype=torch.float32, device=dev))
        self.pred = torch.empty(n_net ** 3, dtype=torch.float32, device=dev)
        self.ups = [torch.empty((n_net * 2 ** (i + 1)) ** 3, dtype=torch.float32, device=dev)
                    for i in range(len(self.levels) - 1)]
        self.chk = torch.empty(n ** 3, dtype=torch.float32, device=dev)
        self.err = torch.empty(1, dtype=torch.float64, device=dev)
        self.tg = None

    def set_targets(self, tg):
        """Flat cell indices of the check (host int64 array): the judge evaluates their leaves."""
        import torch
        ell = self.tree.leaf_side
        nb = self.n // ell
        i, j, k = np.unravel_index(tg, (self.n,) * 3)
        mask = np.zeros((nb, nb, nb), dtype=np.uint8)
        mask[i // ell, j // ell, k // ell] = 1
        self.judge.restrict_targets(mask)
        self.tg = torch.from_numpy(np.ascontiguousarray(tg, dtype=np.int64)).cuda()

    def predict(self, I, S, prefactor):
        K = self.K
        x, side = I, self.n
        for buf in self.levels:
            side //= 2
            K.nn_call("kifmm_nn_coarsen2", 1, side, x, buf)
            x = buf
        self.net.predict(x, self.n_net, 1, self.pred)
        y, side = self.pred, self.n_net
        for buf in self.ups + [S]:
            K.nn_call("kifmm_nn_upsample2", 1, side, y, buf)
            y, side = buf, side * 2
        if prefactor != 1.0:
            # the network predicts S for prefactor 1; S is linear in the prefactor
            K.nn_call("kifmm_nn_scale", S.numel(), S, float(prefactor))

    def step(self, I, S, prefactor=1.0):
        """Returns (sampled relative error of the prediction, whether the FMM was served)."""
        K = self.K
        self.predict(I, S, prefactor)
        K.eval(self.tree, self.judge, I, prefactor, out=self.chk, precision=K.FP32)
        K.nn_call("kifmm_nn_sampled_rel_diff", self.tg.numel(), S, self.chk, self.tg, self.err)
        e = float(self.err.item())
        fb = e > self.tol
        if fb:
            K.eval(self.tree, self.fmm, I, prefactor, out=S, precision=K.FP32)
        return e, fb


def fmm_normalised_targets(K, fields, n):
    """kifmm_eval of every field with prefactor 1/max|I|: S / max|I| (FP32, grid order)."""
    import torch
    grid = K.Grid.cube(n, L_CM)
    tree = K.build_tree(grid, 512)
    ops = K.precompute_operators(tree, K.Kernel(workloads.p_o2_of(P_TORR)), K.Opts(**OPTS))
    I = torch.from_numpy(fields).cuda()
    T = torch.empty_like(I)
    mx = np.abs(fields).max(axis=1).astype(np.float64)
    for i in range(fields.shape[0]):
        K.eval(tree, ops, I[i], 1.0 / mx[i], out=T[i], precision=K.FP32)
    torch.cuda.synchronize()
    return I, T


def evaluate(net, I, T, n, batch=8):
    """Relative L2 error (not squared) of the prediction against T for every field."""
    errs = []
    for b0 in range(0, I.shape[0], batch):
        nb = min(batch, I.shape[0] - b0)
        net.forward(I[b0:b0 + nb].reshape(-1), n, nb)
        from . import kifmm as K
        from .surrogate import HEAD_LD
        K.nn_call("kifmm_nn_rel_l2_loss", nb, n, net._buffers(nb, n)["head"], HEAD_LD,
                  T[b0:b0 + nb].reshape(-1), None, net.loss_buf, net.dwork, net.dwork.numel())
        errs.extend(np.sqrt(net.loss_buf[1:1 + nb].cpu().numpy()).tolist())
    return np.array(errs)


def train(args):
    n = 64
    t0 = time.perf_counter()
    log("generating %d + %d fields" % (args.n_train, args.n_test))
    # CPU workers draw the inputs before this process loads the GPU runtime
    train_f = make_fields(range(40000, 40000 + args.n_train), args.workers)
    test_f = make_fields(range(42000, 42000 + args.n_test), args.workers)
    t_gen = time.perf_counter() - t0
    import torch
    from . import kifmm as K
    from .surrogate import Surrogate

    torch.cuda.set_device(0)
    t0 = time.perf_counter()
    Itr, Ttr = fmm_normalised_targets(K, train_f, n)
    Ite, Tte = fmm_normalised_targets(K, test_f, n)
    t_fmm = time.perf_counter() - t0
    log("data: generation %.1f s, FMM targets %.1f s" % (t_gen, t_fmm))
    net = Surrogate(seed=args.seed, bf16=not args.fp32)
    e_init = evaluate(net, Ite, Tte, n)
    rng = np.random.default_rng(args.seed)
    nb = args.n_train // args.batch
    total = args.epochs * nb
    history = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    it = 0
    for ep in range(args.epochs):
        order = rng.permutation(args.n_train)
        losses = []
        for b in range(nb):
            idx = torch.from_numpy(np.sort(order[b * args.batch:(b + 1) * args.batch])).cuda()
            lr = args.lr * 0.5 * (1 + np.cos(np.pi * it / total))
            loss = net.loss_and_backward(Itr[idx].reshape(-1), Ttr[idx].reshape(-1), n, args.batch)
            net.adam_step(lr)
            losses.append(loss[0:1].clone())
            it += 1
        ep_loss = float(torch.cat(losses).mean().item())
        history.append(ep_loss)
        log("epoch %d: mean squared rel-L2 %.4e (lr %.2e, %.1f s)" % (ep, ep_loss, lr, time.perf_counter() - t0))
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    e_test = evaluate(net, Ite, Tte, n)
    e_train = evaluate(net, Itr[:200], Ttr[:200], n)
    # inference time of one field vs one FMM evaluation at the same size
    x = Ite[0].reshape(-1)
    out = torch.empty_like(x)
    for _ in range(3):
        net.predict(x, n, 1, out)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for _ in range(20):
        net.predict(x, n, 1, out)
    torch.cuda.synchronize()
    t_inf = (time.perf_counter() - t1) / 20
    if args.checkpoint:
        net.save(args.checkpoint)
    global LAST_NET
    LAST_NET = net
    rep = {"task": "surrogate_train", "grid": "64^3 / 4 mm", "p_torr": P_TORR, "n_train": args.n_train,
           "n_test": args.n_test, "epochs": args.epochs, "batch": args.batch, "lr": args.lr,
           "params": net.nparams, "precision": "fp32" if args.fp32 else "bf16 (fp32 masters)",
           "held_out_rel_l2": {"mean": float(e_test.mean()), "median": float(np.median(e_test)),
                               "max": float(e_test.max()), "frac_below_1e-3": float((e_test < 1e-3).mean()),
                               "frac_below_1e-2": float((e_test < 1e-2).mean())},
           "untrained_rel_l2_mean": float(e_init.mean()), "train_rel_l2_mean": float(e_train.mean()),
           "loss_history": history, "train_s": round(t_train, 2), "data_gen_s": round(t_gen, 2),
           "fmm_targets_s": round(t_fmm, 2), "inference_ms_64": round(t_inf * 1e3, 3),
           "samples_per_s": args.epochs * nb * args.batch / t_train}
    print(json.dumps(rep), flush=True)
    return rep


def serve(args):
    import torch
    from . import kifmm as K
    from .surrogate import Surrogate

    torch.cuda.set_device(0)
    n = 128
    log("building %d sources" % args.steps)
    src = np.stack([workloads.interacting_heads(k, n=n, L=L_CM, steps=args.steps, p=P_TORR).I.astype(np.float32)
                    .ravel() for k in range(args.steps)])
    Id = torch.from_numpy(src).cuda()
    grid = K.Grid.cube(n, L_CM)
    kern = K.Kernel(workloads.p_o2_of(P_TORR))
    tree = K.build_tree(grid, 512)
    net = LAST_NET if args.checkpoint == "last" else Surrogate(bf16=True)
    if args.checkpoint and args.checkpoint != "last":
        net.load(args.checkpoint)
    sv = Served(K, net, tree, kern, args.tol)
    tgs = [workloads.sample_targets(n ** 3, args.check_targets, seed=50000 + k) for k in range(args.steps)]
    S = torch.empty(n ** 3, dtype=torch.float32, device="cuda")

    for k in range(3):   # warm-up of both paths
        sv.set_targets(tgs[k])
        sv.step(Id[k], S)
        K.eval(tree, sv.fmm, Id[k], 1.0, out=S, precision=K.FP32)
    torch.cuda.synchronize()
    # the served path: the check's target leaves change every step (the restriction flags
    # are set on the host and copied, part of the step's cost)
    t0 = time.perf_counter()
    errs, fbs = [], []
    for k in range(args.steps):
        sv.set_targets(tgs[k])
        e, fb = sv.step(Id[k], S)
        errs.append(e)
        fbs.append(fb)
    torch.cuda.synchronize()
    t_sur = time.perf_counter() - t0
    t0 = time.perf_counter()
    for k in range(args.steps):
        K.eval(tree, sv.fmm, Id[k], 1.0, out=S, precision=K.FP32)
    torch.cuda.synchronize()
    t_fmm = time.perf_counter() - t0
    # error of the served field (prediction or fallback) and of the FMM at the same cells,
    # against the exact sum there; the coarse floor is the FMM run on the 64^3 coarsening and
    # upsampled the same way (the best any 64^3 predictor can do at these cells), and
    # net_vs_coarse the network's full-field rel-L2 against that 64^3 FMM answer
    grid64 = K.Grid.cube(64, L_CM)
    tree64 = K.build_tree(grid64, 512)
    ops64 = fast_fmm(K, tree64, kern)
    c64 = torch.empty(64 ** 3, dtype=torch.float32, device="cuda")
    ref = torch.empty(args.check_targets, dtype=torch.float64, device="cuda")
    err = torch.empty(1, dtype=torch.float64, device="cuda")
    served_fb, served_pred, fmm_err, floor, net_vs_coarse = [], [], [], [], []
    for k in range(0, args.steps, max(1, args.steps // 20)):
        sv.set_targets(tgs[k])
        e, fb = sv.step(Id[k], S)
        tg = sv.tg
        K.direct_eval(grid, kern, Id[k], 1.0, tg, out=ref, fp64=True)
        K.nn_call("kifmm_nn_sampled_rel_err", args.check_targets, S, tg, ref, 1.0, err)
        (served_fb if fb else served_pred).append(float(err.item()))
        K.eval(tree, sv.fmm, Id[k], 1.0, out=S, precision=K.FP32)
        K.nn_call("kifmm_nn_sampled_rel_err", args.check_targets, S, tg, ref, 1.0, err)
        fmm_err.append(float(err.item()))
        K.nn_call("kifmm_nn_coarsen2", 1, 64, Id[k], sv.levels[0])
        K.eval(tree64, ops64, sv.levels[0], 1.0, out=c64, precision=K.FP32)
        net.predict(sv.levels[0], 64, 1, sv.pred)
        K.nn_call("kifmm_nn_sampled_rel_diff", 64 ** 3, sv.pred, c64,
                  torch.arange(64 ** 3, device="cuda"), err)
        net_vs_coarse.append(float(err.item()))
        K.nn_call("kifmm_nn_upsample2", 1, 64, c64, S)
        K.nn_call("kifmm_nn_sampled_rel_err", args.check_targets, S, tg, ref, 1.0, err)
        floor.append(float(err.item()))
    errs = np.array(errs)
    sur_sps, fmm_sps = args.steps / t_sur, args.steps / t_fmm
    rep = {"task": "surrogate_serve", "grid": "128^3 / 4 mm, surrogate on 64^3", "steps": args.steps,
           "tol": args.tol, "check_targets": args.check_targets,
           "fmm": "lattice layout R = 1.2, FFT-form M2L, near field in Fourier space, FP32 (judge: the same "
                  "restricted to the check targets' leaves)",
           "surrogate_path_steps_per_s": sur_sps, "fmm_only_steps_per_s": fmm_sps,
           "gain_over_fmm_only": sur_sps / fmm_sps,
           "fallback_rate": float(np.mean(fbs)),
           "surrogate_rel_err": {"mean": float(errs.mean()), "median": float(np.median(errs)),
                                 "min": float(errs.min()), "max": float(errs.max())},
           "served_rel_err_max": float(np.max(served_fb + served_pred)),
           "served_rel_err_max_fallback": float(np.max(served_fb)) if served_fb else None,
           "served_rel_err_max_prediction": float(np.max(served_pred)) if served_pred else None,
           "fmm_rel_err_max": float(np.max(fmm_err)),
           "coarse_floor_rel_err": {"mean": float(np.mean(floor)), "max": float(np.max(floor))},
           "net_vs_coarse_fmm_rel_l2": {"mean": float(np.mean(net_vs_coarse)), "max": float(np.max(net_vs_coarse))},
           "checkpoint": args.checkpoint}
    print(json.dumps(rep), flush=True)
    return rep


def main(argv=None):
    """Command line entry; returns the report dict."""
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    a = sub.add_parser("train")
    a.add_argument("--n-train", type=int, default=2000)
    a.add_argument("--n-test", type=int, default=200)
    a.add_argument("--epochs", type=int, default=20)
    a.add_argument("--batch", type=int, default=8)
    a.add_argument("--lr", type=float, default=1e-3)
    a.add_argument("--seed", type=int, default=0)
    a.add_argument("--workers", type=int, default=8)
    a.add_argument("--fp32", action="store_true")
    a.add_argument("--checkpoint", default="")
    s = sub.add_parser("serve")
    s.add_argument("--checkpoint", default="")
    s.add_argument("--steps", type=int, default=200)
    s.add_argument("--tol", type=float, default=1e-3)
    s.add_argument("--check-targets", type=int, default=1024)
    args = ap.parse_args(argv)
    return train(args) if args.cmd == "train" else serve(args)


if __name__ == "__main__":
    main()
