"""Benchmark: target points/s of the KIFMM evaluation of the photoionization sum
on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--n 256] [--precision fp32]

One step = one kifmm_eval over the whole grid (permute in, P2M, M2M, M2L, L2L,
L2P, P2P with the self cell, permute out) with the source already resident in
HBM.  The operators are precomputed once before the timed region (per pressure)
and their time is reported separately.  Accuracy is checked after the timed
region against FP64 direct evaluation (direct_eval) at 4,096 seeded targets.

Prints one JSON line (see the design doc for every field).
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_FP32_MFMA = 157.3e12  # FLOP/s, dense FP32 matrix, MI355X
PEAK_BF16_MFMA = 2.5e15
PEAK_HBM = 8.0e12


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def near_pairs(nb, s):
    """(target, source) pairs of the near field: leaves x existing neighbour leaves."""
    per_axis = 3 * nb - 2 if nb > 1 else 1
    return per_axis ** 3 * s * s


def m2l_pairs(level):
    """Number of (target box, interaction-list box) pairs at a level."""
    n = 1 << level
    i = np.arange(n)
    total = 0
    for o in np.ndindex(7, 7, 7):
        o = np.array(o) - 3
        if np.abs(o).max() <= 1:
            continue
        cnt = 1
        for v in o:
            ok = (np.abs((i + v) // 2 - i // 2) <= 1) & (i + v >= 0) & (i + v < n)
            cnt *= int(ok.sum())
        total += cnt
    return total


TRAFFIC_FILES = {   # (summary with the counters, source file of the kernel they were taken on)
    "dense": (os.path.join(ROOT, "profiles", "tapgemm_p2p_traffic_streamer256.md"),
              os.path.join(ROOT, "paper_2006_03515_amd", "csrc", "tapgemm.hip")),
    "fft": (os.path.join(ROOT, "profiles", "near_products_traffic_streamer256.md"),
            os.path.join(ROOT, "paper_2006_03515_amd", "csrc", "near_fft.hip")),
}
# FP32 FMA on the vector ALUs without packed math: 256 CUs x 4 SIMDs x 16 lanes x 2 flops x 2.4 GHz
PEAK_FP32_VALU = 78.6e12


def p2p_traffic(args):
    """HBM-side bytes of one launch of the near field's dominant kernel from the committed
    --pmc summary, or None when that summary is missing, was taken on another
    configuration, or the kernel source has changed since."""
    import hashlib
    traffic_file, kernel_src = TRAFFIC_FILES[args.p2p]
    if args.precision != "fp32" or args.n != 256 or not os.path.exists(traffic_file):
        return None
    h = hashlib.sha256(open(kernel_src, "rb").read()).hexdigest()
    vals = {}
    for line in open(traffic_file):
        if ":" in line and line.startswith("- "):
            k, v = line[2:].split(":", 1)
            vals[k.strip()] = v.strip().strip("`")
    if vals.get("kernel_source_sha256") != h:
        return None
    try:
        return float(vals["traffic_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def surrogate_variant(args, K, w, I, S, N, accuracy, timed_fn=None):
    """The learned surrogate on the same workload: block-mean coarsening to 64^3,
    inference, trilinear upsampling back to the grid; timed like a step, judged on
    the same sampled cells.  'quick' trains a small network here (256 fields,
    4 epochs) on FMM-made 64^3 data; a checkpoint path loads a trained one."""
    import torch
    from paper_2006_03515_amd import surrogate_tasks as T
    from paper_2006_03515_amd.surrogate import Surrogate
    if args.surrogate == "quick":
        log("training a quick surrogate (256 fields, 4 epochs)")
        import contextlib
        with contextlib.redirect_stdout(sys.stderr):   # bench prints one JSON line only
            rep = T.main(["train", "--n-train", "256", "--n-test", "16", "--epochs", "4", "--workers", "1"])
        net = T.LAST_NET
        how = "quick: 256 fields x 4 epochs, held-out rel-L2 %.3g" % rep["held_out_rel_l2"]["mean"]
    else:
        net = Surrogate(bf16=True)
        net.load(args.surrogate)
        how = "checkpoint " + os.path.basename(args.surrogate)
    levels = []
    n = w.n
    while n > 64:
        n //= 2
        levels.append(torch.empty(n ** 3, dtype=torch.float32, device=I.device))
    s64 = torch.empty(64 ** 3, dtype=torch.float32, device=I.device)
    ups = [torch.empty((64 * 2 ** (i + 1)) ** 3, dtype=torch.float32, device=I.device)
           for i in range(len(levels) - 1)]

    def step():
        x = I
        side = w.n
        for buf in levels:
            side //= 2
            K.nn_call("kifmm_nn_coarsen2", 1, side, x, buf)
            x = buf
        net.predict(x, 64, 1, s64)
        y, side = s64, 64
        for buf in ups + [S]:
            K.nn_call("kifmm_nn_upsample2", 1, side, y, buf)
            y, side = buf, side * 2
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(args.steps):
        step()
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / args.steps
    # S carries the prediction for prefactor 1; the sampled check uses w.prefactor
    S.mul_(w.prefactor)
    return {"value": N / (ms * 1e-3), "ms_per_step": round(ms, 4), "rel_l2": accuracy(), "network": how,
            "note": "inference on a 64^3 block-mean coarsening, trilinear upsampling; not a bound-"
                    "respecting method (no accuracy guarantee without the FMM check/fallback)"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--n", type=int, default=256)
    ap.add_argument("--p", type=float, default=760.0, help="air pressure [Torr]")
    ap.add_argument("--max-leaf", type=int, default=512)
    ap.add_argument("--layout", default="lattice", choices=["paper", "single", "nested", "lattice"])
    ap.add_argument("--lattice-radius", type=float, default=1.0,
                    help="lattice layout: half-width of its point lattices in box half-widths (1.0 "
                         "measured best for 760 Torr air; 0 = the library default 1.2, robust over pressures)")
    ap.add_argument("--p2p", default="fft", choices=["fft", "dense"],
                    help="near field: dense 512 x 512 blocks on MFMA, or in Fourier space (leaves of 8^3)")
    ap.add_argument("--m2l", default="fft", choices=["fft", "dense"],
                    help="M2L form for the lattice layout (the other layouts have only the dense form)")
    ap.add_argument("--rcond", type=float, default=1e-5)
    ap.add_argument("--m0", type=int, default=5)
    ap.add_argument("--precision", default="fp32")
    ap.add_argument("--variants", default="fp32/graph,bf16x3/graph,bf16x3,fp16,bf16,m2l_bf16x3,m2l_fp16,m2l_bf16,bf16x3/near_dense,fp32/near_dense,fp32/dense/near_dense,bf16x3/dense/near_dense",
                    help="extra precisions timed after the headline one ('' for none); "
                         "'<precision>/dense' or '/fft' also sets the M2L form (lattice layout), "
                         "'/near_fft' or '/near_dense' the near-field form, '/graph' times replays "
                         "of one evaluation captured in a HIP graph")
    ap.add_argument("--check-targets", type=int, default=4096)
    ap.add_argument("--cpu-targets", type=int, default=2048,
                    help="targets of the oracle CPU baseline sample (0 = skip)")
    ap.add_argument("--calibrate-copy-mib", type=int, default=0,
                    help="after timing, copy a buffer of this size twice (plain copy kernel used to "
                         "scale the FETCH_SIZE / WRITE_SIZE counters of a --pmc run)")
    ap.add_argument("--surrogate", default="quick",
                    help="'quick' (train a small surrogate here), a checkpoint path, or '' to skip")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py runs on one GPU only: this build has no multi-GPU path "
              "(see DESIGN.md for how the evaluation would shard).", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2006_03515_amd import kifmm as K
    from paper_2006_03515_amd import workloads

    torch.cuda.set_device(0)
    dev = torch.device("cuda:0")
    log("generating streamer channel %d^3" % args.n)
    w = workloads.streamer_channel(n=args.n, L=0.4, p=args.p, dtype=np.float32)
    I_host = np.ascontiguousarray(w.I.reshape(-1))
    I = torch.from_numpy(I_host).to(dev)
    grid = K.Grid.cube(w.n, w.L)
    kern = K.Kernel(w.p_o2)
    layout = {"paper": K.LAYOUT_PAPER, "single": K.LAYOUT_SINGLE, "nested": K.LAYOUT_NESTED,
              "lattice": K.LAYOUT_LATTICE}[args.layout]
    opts = K.Opts(layout, args.m0, 10, args.rcond, args.lattice_radius)

    t0 = time.perf_counter()
    tree = K.build_tree(grid, args.max_leaf)
    ops = K.precompute_operators(tree, kern, opts)
    torch.cuda.synchronize()
    t_pre = time.perf_counter() - t0
    m2l_form = args.m2l if args.layout == "lattice" else "dense"
    if args.layout == "lattice":
        ops.m2l_fft(m2l_form == "fft")
    ops.p2p_fft(args.p2p == "fft")
    ranks = {l: ops.rank(l) for l in range(2, tree.depth + 1)}
    log("tree depth %d, leaf %d^3, precompute %.2f s, ranks %s" % (tree.depth, tree.leaf_side, t_pre, ranks))

    S = torch.empty_like(I)
    stream = torch.cuda.current_stream()

    def timed(precision, steps, warmup, profile):
        for _ in range(warmup):
            K.eval(tree, ops, I, w.prefactor, out=S, precision=precision)
        torch.cuda.synchronize()
        if profile:
            ops.profile(True)
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record(stream)
        for _ in range(steps):
            K.eval(tree, ops, I, w.prefactor, out=S, precision=precision)
        e1.record(stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / steps
        prof = ops.profile_read() if profile else None
        if profile:
            ops.profile(False)
        return ms, prof

    def timed_graph(precision, steps, warmup):
        # one evaluation captured in a HIP graph (its side streams join the capture through
        # the library's fork/join events), then replayed
        side = torch.cuda.Stream()
        side.wait_stream(stream)
        with torch.cuda.stream(side):
            K.eval(tree, ops, I, w.prefactor, out=S, precision=precision)
        stream.wait_stream(side)
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            K.eval(tree, ops, I, w.prefactor, out=S, precision=precision)
        torch.cuda.synchronize()
        for _ in range(warmup):
            g.replay()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record(stream)
        for _ in range(steps):
            g.replay()
        e1.record(stream)
        torch.cuda.synchronize()
        del g
        return e0.elapsed_time(e1) / steps

    # accuracy sample: FP64 direct at seeded targets (computed once)
    tg = workloads.sample_targets(w.n ** 3, args.check_targets, seed=1009)
    tgt = torch.from_numpy(tg).to(dev)
    log("direct_eval FP64 at %d targets" % tg.size)
    ref = K.direct_eval(grid, kern, I, w.prefactor, tgt, fp64=True).cpu().numpy()

    def accuracy():
        got = S[tgt].double().cpu().numpy()
        return float(np.linalg.norm(got - ref) / np.linalg.norm(ref))

    # headline precision: timed once without instrumentation, once with per-pass events
    log("timing %s: %d warmup + %d steps" % (args.precision, args.warmup, args.steps))
    ms, _ = timed(args.precision, args.steps, args.warmup, profile=False)
    err = accuracy()
    _, prof = timed(args.precision, args.steps, 1, profile=True)
    log("%s: %.3f ms/step, rel-L2 %.3e" % (args.precision, ms, err))

    N = w.n ** 3
    nb, s = tree.grid.n[0] // tree.leaf_side, tree.leaf_side ** 3
    p2p_flops = 2.0 * near_pairs(nb, s)
    if m2l_form == "fft":
        # FFT form: coefficients -> lattice values and back (two GEMMs per box, m0^3 x rank),
        # plus one complex multiply-add (8 flops) per interaction pair and frequency (all on
        # MFMA at levels >= 3; the parent-pair products also multiply the zero entries of
        # adjacent children, and the separable transforms run on the VALU: neither counted)
        nf = (2 * args.m0 - 1) ** 2 * args.m0
        m2l_flops = sum(2.0 * 8 ** l * args.m0 ** 3 * (ranks[l][0] + ranks[l][1]) + 8.0 * m2l_pairs(l) * nf
                        for l in ranks)
    else:
        m2l_flops = sum(2.0 * m2l_pairs(l) * ranks[l][0] * ranks[l][1] for l in ranks)
    pass_ms = {k: v[0] / max(v[1], 1) for k, v in prof.items()}        # mean per launch
    pass_step = {k: v[0] / args.steps for k, v in prof.items()}       # per step
    calls_step = {k: v[1] / args.steps for k, v in prof.items()}
    # Roofline of the near field (P2P): the largest kernel when each pass runs alone,
    # one launch per step.  The M2L launches (one per level) are reported beside it.
    peak = PEAK_FP32_MFMA if args.precision in ("fp32", "fp64") else PEAK_BF16_MFMA
    if args.p2p == "fft" and pass_ms.get("near_products", 0) > 0:
        # near field in Fourier space: the dominant kernel is the products kernel, one
        # complex multiply-add (8 flops) per frequency of the half spectrum (15 x 15 x 8;
        # the kernel's 16th slot per column, kept zero for alignment, is not counted) and
        # existing leaf pair
        leaf_pairs = float(3 * nb - 2) ** 3
        prod_flops = 8.0 * 1800 * leaf_pairs
        t = pass_ms["near_products"]
        achieved = prod_flops / (t * 1e-3) / 1e12
        roofline = {"bound": "alu", "kernel": "near_products (near field in Fourier space)",
                    "achieved": round(achieved, 3), "peak": PEAK_FP32_VALU / 1e12, "unit": "TFLOP/s",
                    "frac": round(achieved * 1e12 / PEAK_FP32_VALU, 4), "traffic": p2p_traffic(args),
                    "flops_per_launch": prod_flops, "avg_launch_ms": round(t, 4),
                    "near_field_pass_ms": round(pass_ms["p2p"], 4)}
    else:
        achieved = p2p_flops / (pass_ms["p2p"] * 1e-3) / 1e12
        roofline = {"bound": "mfma", "kernel": "p2p (tapgemm near field)", "achieved": round(achieved, 3),
                    "peak": peak / 1e12, "unit": "TFLOP/s", "frac": round(achieved * 1e12 / peak, 4),
                    "traffic": p2p_traffic(args), "flops_per_launch": p2p_flops,
                    "avg_launch_ms": round(pass_ms["p2p"], 4)}
    m2l_launch = m2l_flops / max(calls_step["m2l"], 1)
    m2l_ach = m2l_launch / (pass_ms["m2l"] * 1e-3) / 1e12
    roofline_m2l = {"bound": "mfma",
                    "kernel": "m2l (all levels, %s form)" % m2l_form, "achieved": round(m2l_ach, 3),
                    "peak": peak / 1e12, "unit": "TFLOP/s", "frac": round(m2l_ach * 1e12 / peak, 4),
                    "flops_per_launch": m2l_launch, "avg_launch_ms": round(pass_ms["m2l"], 4),
                    "launches_per_step": calls_step["m2l"]}

    # tree passes (permute into leaf order, and far + near field back to grid order):
    # HBM-bound, algorithmic bytes = values read + written once
    esz = 8 if args.precision == "fp64" else 4
    tree_bytes = {"permute_in": 2 * N * esz, "permute_out": 3 * N * esz}
    tree_passes = {k: {"avg_launch_ms": round(pass_ms[k], 4), "bytes": b,
                       "GB_per_s": round(b / (pass_ms[k] * 1e-3) / 1e9, 1),
                       "frac_of_8TBps": round(b / (pass_ms[k] * 1e-3) / PEAK_HBM, 4)}
                   for k, b in tree_bytes.items() if k in pass_ms}

    variants = {}
    for v in [x for x in args.variants.split(",") if x]:
        log("timing variant %s" % v)
        prec, *forms = v.split("/")
        for form in forms:
            if form in ("fft", "dense") and args.layout == "lattice":
                ops.m2l_fft(form == "fft")
            if form in ("near_fft", "near_dense"):
                ops.p2p_fft(form == "near_fft")
        if "graph" in forms:
            vms = timed_graph(prec, args.steps, args.warmup)
        else:
            vms, _ = timed(prec, args.steps, args.warmup, profile=False)
        variants[v] = {"value": N / (vms * 1e-3), "ms_per_step": round(vms, 4), "rel_l2": accuracy(),
                       "speedup_vs_headline": round(ms / vms, 3)}
        if args.layout == "lattice":
            ops.m2l_fft(m2l_form == "fft")
        ops.p2p_fft(args.p2p == "fft")

    if args.calibrate_copy_mib > 0:
        src = torch.ones(args.calibrate_copy_mib << 18, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        for _ in range(2):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    if args.surrogate:
        variants["surrogate"] = surrogate_variant(args, K, w, I, S, N, accuracy, timed_fn=None)

    cpu = None
    if args.cpu_targets > 0:
        from oracle import direct as odirect
        ctg = workloads.sample_targets(N, args.cpu_targets, seed=77)
        log("oracle CPU baseline: %d targets x %d sources" % (ctg.size, N))
        Ih = I_host.reshape(w.n, w.n, w.n).astype(np.float64)
        t1 = time.perf_counter()
        odirect.direct_targets(Ih, (w.h,) * 3, w.p_o2, ctg, prefactor=w.prefactor)
        dt = time.perf_counter() - t1
        cpu = {"value": ctg.size / dt, "unit": "target points/s", "cores": odirect.num_threads(),
               "kind": "oracle", "sample": "FP64 direct sum (C/OpenMP) at %d seeded targets of the "
                                           "same %d^3 workload, %.1f s" % (ctg.size, w.n, dt)}

    out = {
        "metric": "target points/s at <=1e-4 rel-L2 vs FP64 direct (KIFMM evaluation)",
        "value": N / (ms * 1e-3),
        "unit": "target points/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"fp32": "f32", "fp64": "f64"}.get(args.precision, "f32+" + args.precision),
        "data": "synthetic",
        "config": {"workload": "streamer_channel_%d" % w.n, "n": w.n, "L_cm": w.L, "p_torr": w.p,
                   "p_o2_torr": w.p_o2, "layout": args.layout, "m0": args.m0, "check_edge": 10,
                   "rcond": args.rcond, "max_leaf": args.max_leaf, "leaf_side": tree.leaf_side,
                   "depth": tree.depth, "precision": args.precision, "m2l": m2l_form, "p2p": args.p2p,
                   "lattice_radius": (args.lattice_radius or 1.2) if args.layout == "lattice" else None,
                   "parallelism": "none"},
        "rel_l2_sampled": err,
        "accuracy_ok": err <= 1e-4,
        "pair_interactions_per_s": near_pairs(nb, s) / (ms * 1e-3),
        "precompute_s": round(t_pre, 3),
        "pass_ms_per_step": {k: round(v, 4) for k, v in pass_step.items()},
        "m2l_flops_per_step": m2l_flops,
        "p2p_flops_per_step": p2p_flops,
        "roofline": roofline,
        "roofline_m2l": roofline_m2l,
        "tree_passes": tree_passes,
        "variants": variants,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
