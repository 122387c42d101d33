"""Benchmark: target points/s of the KIFMM evaluation of the photoionization sum
on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--n 256] [--precision fp32]

One step = one kifmm_eval over the whole grid (P2M fused with the way into leaf
order, M2M, M2L, L2L, the near field with the self cell, L2P fused with the sum and
the way out) with the source already resident in HBM.  The operators are
precomputed once before the timed region (per pressure) and their time is reported
separately.  Accuracy is checked after the timed region against FP64 direct
evaluation (direct_eval) at 4,096 seeded targets; a result above the 1e-4 bar gets
no points/s value.

The headline workload is the 256^3 streamer channel at 760 Torr; the same
configuration is also timed at 100 and 10 Torr (`pressures`) and on the 128^3
two-head workload at 760 and 100 Torr (`config_128`).

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
# FP32 FMA on the vector ALUs without packed math: 256 CUs x 4 SIMDs x 16 lanes x 2 flops x 2.4 GHz
PEAK_FP32_VALU = 78.6e12
BAR = 1e-4


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


class Case:
    """One workload with its tree, operators, resident source and accuracy sample."""

    def __init__(self, args, K, workloads, w, layout, m0, rcond, radius, p2p, m2l, check_targets, seed):
        import torch
        self.K, self.w = K, w
        self.dev = torch.device("cuda:0")
        self.I = torch.from_numpy(np.ascontiguousarray(w.I.astype(np.float32).reshape(-1))).to(self.dev)
        self.grid = K.Grid.cube(w.n, w.L)
        self.kern = K.Kernel(w.p_o2)
        lay = {"paper": K.LAYOUT_PAPER, "single": K.LAYOUT_SINGLE, "nested": K.LAYOUT_NESTED,
               "lattice": K.LAYOUT_LATTICE}[layout]
        t0 = time.perf_counter()
        self.tree = K.build_tree(self.grid, args.max_leaf)
        self.ops = K.precompute_operators(self.tree, self.kern, K.Opts(lay, m0, 10, rcond, radius))
        torch.cuda.synchronize()
        self.t_pre = time.perf_counter() - t0
        self.m2l = m2l if layout == "lattice" else "dense"
        if layout == "lattice":
            self.ops.m2l_fft(self.m2l == "fft")
        self.p2p = p2p
        self.ops.p2p_fft(p2p == "fft")
        self.S = torch.empty_like(self.I)
        self.stream = torch.cuda.current_stream()
        tg = workloads.sample_targets(w.n ** 3, check_targets, seed=seed)
        self.tgt = torch.from_numpy(tg).to(self.dev)
        self.ref = K.direct_eval(self.grid, self.kern, self.I, w.prefactor, self.tgt, fp64=True).cpu().numpy()
        self.N = w.n ** 3

    def eval(self, precision):
        self.K.eval(self.tree, self.ops, self.I, self.w.prefactor, out=self.S, precision=precision)

    def accuracy(self):
        got = self.S[self.tgt].double().cpu().numpy()
        return float(np.linalg.norm(got - self.ref) / np.linalg.norm(self.ref))

    def timed(self, precision, steps, warmup, profile=False):
        """(mean ms over `steps` back-to-back steps bracketed by synchronisations, median
        of `steps` single-step event timings, per-pass profile or None)."""
        import torch
        for _ in range(warmup):
            self.eval(precision)
        torch.cuda.synchronize()
        if profile:
            self.ops.profile(True)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record(self.stream)
        for _ in range(steps):
            self.eval(precision)
        e1.record(self.stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / steps
        prof = self.ops.profile_read() if profile else None
        if profile:
            self.ops.profile(False)
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
        ev[0].record(self.stream)
        for i in range(steps):
            self.eval(precision)
            ev[i + 1].record(self.stream)
        torch.cuda.synchronize()
        med = float(np.median([ev[i].elapsed_time(ev[i + 1]) for i in range(steps)]))
        return ms, med, prof

    def timed_graph(self, precision, steps, warmup):
        """One evaluation captured in a HIP graph (its side streams join the capture through
        the library's fork/join events), then replayed: (mean ms over `steps` back-to-back
        replays, median of `steps` single-replay event timings).  Every replay runs every
        kernel of the evaluation on the current contents of I (tests/test_gpu_graph.py)."""
        import torch
        side = torch.cuda.Stream()
        side.wait_stream(self.stream)
        with torch.cuda.stream(side):
            self.eval(precision)
        self.stream.wait_stream(side)
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            self.eval(precision)
        torch.cuda.synchronize()
        for _ in range(warmup):
            g.replay()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record(self.stream)
        for _ in range(steps):
            g.replay()
        e1.record(self.stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / steps
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
        ev[0].record(self.stream)
        for i in range(steps):
            g.replay()
            ev[i + 1].record(self.stream)
        torch.cuda.synchronize()
        med = float(np.median([ev[i].elapsed_time(ev[i + 1]) for i in range(steps)]))
        del g
        return ms, med

    def timed_launch(self, precision, steps, warmup, launch):
        """(mean ms, median ms) of the evaluation issued as `launch`: 'graph' or 'eager'."""
        if launch == "graph":
            return self.timed_graph(precision, steps, warmup)
        ms, med, _ = self.timed(precision, steps, warmup)
        return ms, med


def result(N, ms, err, **extra):
    """Throughput entry; no points/s value when the accuracy bar is missed."""
    ok = err <= BAR
    d = {"value": N / (ms * 1e-3) if ok else None, "ms_per_step": round(ms, 4), "rel_l2": err, "accuracy_ok": ok}
    d.update(extra)
    return d


def surrogate_variant(args, K, case, ms_head):
    """The learned surrogate served as the FMM-judged loop does it (surrogate_tasks.Served):
    block-mean coarsening to 64^3, inference, trilinear upsampling, the FMM restricted to
    the sampled targets' leaves as judge, and the full FMM whenever the prediction misses
    the 1e-4 bar at those targets.  'quick' trains a small network here (256 fields,
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
    w = case.w
    sv = T.Served(K, net, case.tree, case.kern, BAR)
    sv.set_targets(workloads_targets(w.n, 1024))
    fbs, errs = [], []
    for _ in range(args.warmup):
        sv.step(case.I, case.S, w.prefactor)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(case.stream)
    for _ in range(args.steps):
        e, fb = sv.step(case.I, case.S, w.prefactor)
        errs.append(e)
        fbs.append(fb)
    e1.record(case.stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / args.steps
    err = case.accuracy()
    # the prediction alone (no check, no fallback): its time and error, for context
    sv.predict(case.I, case.S, w.prefactor)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        sv.predict(case.I, case.S, w.prefactor)
    torch.cuda.synchronize()
    ms_pred = (time.perf_counter() - t0) * 1e3 / args.steps
    err_pred = case.accuracy()
    return result(case.N, ms, err, speedup_vs_headline=round(ms_head / ms, 3), network=how,
                  fallback_rate=float(np.mean(fbs)), prediction_rel_err_at_check=float(np.median(errs)),
                  prediction_only={"ms_per_step": round(ms_pred, 4), "rel_l2": err_pred,
                                   "accuracy_ok": err_pred <= BAR},
                  served="64^3 inference + upsampling, judged at 1,024 cells by the FMM restricted to their "
                         "leaves, full FMM fallback above 1e-4")


def workloads_targets(n, count):
    from paper_2006_03515_amd import workloads
    return workloads.sample_targets(n ** 3, count, seed=2024)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    # the first few dozen evaluations after setup run up to 20 % slower than the rest while the
    # GPU's clocks ramp (measured replay by replay); 30 untimed steps (about 30 ms) cover it
    ap.add_argument("--warmup", type=int, default=30)
    ap.add_argument("--n", type=int, default=256)
    ap.add_argument("--p", type=float, default=760.0, help="air pressure of the headline [Torr]")
    ap.add_argument("--pressures", default="100,10",
                    help="further pressures timed with the headline configuration ('' for none)")
    ap.add_argument("--config-128", type=int, default=1, help="also time the 128^3 two-head workload")
    ap.add_argument("--section42", type=int, default=1,
                    help="also time the paper's Section 4.2 workload (256 x 256 x 320 cells, hz = 4.48 hx)")
    ap.add_argument("--max-leaf", type=int, default=512)
    ap.add_argument("--layout", default="lattice", choices=["paper", "single", "nested", "lattice"])
    ap.add_argument("--lattice-radius", type=float, default=0.0,
                    help="lattice layout: half-width of its point lattices in box half-widths (0 = the "
                         "library default 1.2, under the 1e-4 bar at 10, 100 and 760 Torr)")
    ap.add_argument("--p2p", default="fft", choices=["fft", "dense"],
                    help="near field: dense 512 x 512 blocks on MFMA, or in Fourier space (leaves of 8^3)")
    ap.add_argument("--m2l", default="fft", choices=["fft", "dense"],
                    help="M2L form for the lattice layout (the other layouts have only the dense form)")
    ap.add_argument("--rcond", type=float, default=1e-5)
    ap.add_argument("--m0", type=int, default=5)
    ap.add_argument("--precision", default="fp32")
    ap.add_argument("--schedule", default="concurrent", choices=["concurrent", "serial"],
                    help="serial: every pass of the headline on the calling stream (per-kernel profiles "
                         "without overlap; the headline value is then the serial step)")
    ap.add_argument("--launch", default="graph", choices=["graph", "eager"],
                    help="how the timed evaluations are issued: replays of one evaluation captured in a "
                         "HIP graph (the launches of all four streams recorded once), or one kifmm_eval "
                         "call per step")
    ap.add_argument("--variants", default="fp32/eager,bf16x3,bf16x3/eager,m2l_fp16,m2l_bf16,fp16,bf16,bf16x3/near_dense,fp32/near_dense,fp32/dense/near_dense",
                    help="extra precisions timed after the headline one ('' for none); "
                         "'<precision>/dense' or '/fft' also sets the M2L form (lattice layout), "
                         "'/near_fft' or '/near_dense' the near-field form, '/graph' or '/eager' the "
                         "launch (default: that of the headline)")
    ap.add_argument("--check-targets", type=int, default=4096)
    ap.add_argument("--cpu-targets", type=int, default=2048,
                    help="targets of the oracle CPU baseline's direct-sum sample (0 = skip the CPU baseline)")
    ap.add_argument("--cpu-threads", type=int, default=16, help="threads of the oracle CPU baseline")
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

    def channel_case(p):
        log("streamer channel %d^3 at %g Torr" % (args.n, p))
        w = workloads.streamer_channel(n=args.n, L=0.4, p=p, dtype=np.float32)
        return Case(args, K, workloads, w, args.layout, args.m0, args.rcond, args.lattice_radius, args.p2p,
                    args.m2l, args.check_targets, 1009)

    case = channel_case(args.p)
    tree, ops, w = case.tree, case.ops, case.w
    serial_default = args.schedule == "serial"
    ops.serial(serial_default)
    ranks = {l: ops.rank(l) for l in range(2, tree.depth + 1)}
    log("tree depth %d, leaf %d^3, precompute %.2f s, ranks %s" % (tree.depth, tree.leaf_side, case.t_pre, ranks))

    # headline precision: timed without instrumentation, then once with per-pass events on
    # the launch streams, then once with every pass on the calling stream (no overlap)
    log("timing %s (%s): %d warmup + %d steps" % (args.precision, args.launch, args.warmup, args.steps))
    ms, med = case.timed_launch(args.precision, args.steps, args.warmup, args.launch)
    err = case.accuracy()   # the field the timed launches wrote
    ms_eager, med_eager, _ = case.timed(args.precision, args.steps, args.warmup)
    _, _, prof = case.timed(args.precision, args.steps, 1, profile=True)
    ops.serial(True)
    ms_serial, _, prof_serial = case.timed(args.precision, args.steps, 1, profile=True)
    ops.serial(serial_default)
    log("%s: %.3f ms/step (median %.3f, serial %.3f), rel-L2 %.3e" % (args.precision, ms, med, ms_serial, err))

    N = case.N
    nb, s = tree.grid.n[0] // tree.leaf_side, tree.leaf_side ** 3
    if case.m2l == "fft":
        # FFT form: coefficients -> lattice values and back (two GEMMs per box, m0^3 x rank),
        # plus one complex multiply-add (8 flops) per interaction pair and stored frequency
        # (one of each conjugate pair of the N^3 grid, N = 2 m0 - 1: (N^3 + 1) / 2; the
        # parent-pair products also multiply the zero entries of adjacent children, and the
        # separable transforms run on the VALU: neither counted)
        nf = ((2 * args.m0 - 1) ** 3 + 1) // 2
        m2l_flops = sum(2.0 * 8 ** l * args.m0 ** 3 * (ranks[l][0] + ranks[l][1]) + 8.0 * m2l_pairs(l) * nf
                        for l in ranks)
    else:
        m2l_flops = sum(2.0 * m2l_pairs(l) * ranks[l][0] * ranks[l][1] for l in ranks)

    def per_launch(p):
        return {k: v[0] / v[1] for k, v in p.items() if v[1] > 0}
    pass_ms = per_launch(prof)
    pass_ms_serial = per_launch(prof_serial)
    pass_step = {k: v[0] / args.steps for k, v in prof.items() if v[1] > 0}
    pass_step_serial = {k: v[0] / args.steps for k, v in prof_serial.items() if v[1] > 0}
    calls_step = {k: v[1] / args.steps for k, v in prof.items() if v[1] > 0}
    peak = PEAK_FP32_MFMA if args.precision in ("fp32", "fp64") else PEAK_BF16_MFMA

    def near_roofline(pm, tag):
        if case.p2p == "fft" and pm.get("near_products", 0) > 0:
            # near field in Fourier space: the dominant kernel is the products kernel, one
            # complex multiply-add (8 flops) per multiplied frequency (113 columns (ky, kz) of
            # 15 kx: the half spectrum less the mirrored half of the plane kz = 0; the 16th
            # slot per column, kept zero for alignment, is not counted) and existing leaf pair
            prod_flops = 8.0 * 113 * 15 * float(3 * nb - 2) ** 3
            t = pm["near_products"]
            a = prod_flops / (t * 1e-3) / 1e12
            return {"bound": "alu", "kernel": "near_products (near field in Fourier space)%s" % tag,
                    "achieved": round(a, 3), "peak": PEAK_FP32_VALU / 1e12, "unit": "TFLOP/s",
                    "frac": round(a * 1e12 / PEAK_FP32_VALU, 4), "traffic": p2p_traffic(args),
                    "flops_per_launch": prod_flops, "avg_launch_ms": round(t, 4),
                    "near_field_pass_ms": round(pm["p2p"], 4)}
        p2p_flops = 2.0 * near_pairs(nb, s)
        a = p2p_flops / (pm["p2p"] * 1e-3) / 1e12
        return {"bound": "mfma", "kernel": "p2p (tapgemm near field)%s" % tag, "achieved": round(a, 3),
                "peak": peak / 1e12, "unit": "TFLOP/s", "frac": round(a * 1e12 / peak, 4),
                "traffic": p2p_traffic(args), "flops_per_launch": p2p_flops, "avg_launch_ms": round(pm["p2p"], 4)}

    # the dominant kernel timed alone (every pass on the calling stream, the serial pass
    # above), and the same kernel inside the concurrent step, where it shares the GPU
    roofline = near_roofline(pass_ms_serial, " (alone: serial schedule)")
    roofline_in_step = near_roofline(pass_ms, " (in the concurrent step)")
    # the whole M2L of one step (every level, every launch) timed alone: its algorithmic
    # FLOP over the summed durations of its passes
    m2l_ach = m2l_flops / (pass_step_serial["m2l"] * 1e-3) / 1e12
    roofline_m2l = {"bound": "mfma",
                    "kernel": "m2l, all levels (%s form, alone: serial schedule)" % case.m2l,
                    "achieved": round(m2l_ach, 3),
                    "peak": peak / 1e12, "unit": "TFLOP/s", "frac": round(m2l_ach * 1e12 / peak, 4),
                    "flops_per_step": m2l_flops, "ms_per_step": round(pass_step_serial["m2l"], 4)}

    # leaf passes fused with the permutes (HBM-side algorithmic bytes: values read and written
    # once; the operators come from L2): way in + P2M reads I and writes c_u (and q, when the
    # near field reads it); L2P + way out reads c_d and the near field and writes S
    esz = 8 if args.precision == "fp64" else 4
    KU, KD = ranks[tree.depth]
    # (with the near field in Fourier space it reads the grid-order input itself and P2M writes
    # no leaf-ordered copy of the sources)
    p2m_q = 0 if case.p2p == "fft" else N
    leaf_bytes = {"p2m": (N + p2m_q + (N // s) * KU) * esz, "l2p": (2 * N + (N // s) * KD) * esz,
                  "permute_in": 2 * N * esz, "permute_out": 3 * N * esz}
    leaf_flops = {"p2m": 2.0 * N * KU, "l2p": 2.0 * N * KD}
    leaf_passes = {}
    for k, b in leaf_bytes.items():
        if k not in pass_ms_serial:
            continue
        t = pass_ms_serial[k]
        e = {"avg_launch_ms_serial": round(t, 4), "avg_launch_ms_in_step": round(pass_ms.get(k, 0.0), 4),
             "bytes": b, "GB_per_s": round(b / (t * 1e-3) / 1e9, 1), "frac_of_8TBps": round(b / (t * 1e-3) / PEAK_HBM, 4)}
        if k in leaf_flops:
            e["TFLOP_per_s"] = round(leaf_flops[k] / (t * 1e-3) / 1e12, 2)
            e["frac_of_fp32_mfma"] = round(leaf_flops[k] / (t * 1e-3) / PEAK_FP32_MFMA, 4)
        leaf_passes[k] = e

    # the same configuration at the other pressures of the workload
    pressures = {str(int(args.p)): result(N, ms, err, ms_median=round(med, 4), precompute_s=round(case.t_pre, 3))}
    for p in [float(x) for x in args.pressures.split(",") if x]:
        c = channel_case(p)
        pms, pmed = c.timed_launch(args.precision, args.steps, args.warmup, args.launch)
        pressures[str(int(p))] = result(N, pms, c.accuracy(), ms_median=round(pmed, 4), precompute_s=round(c.t_pre, 3))
        log("%g Torr: %.3f ms/step, rel-L2 %.3e" % (p, pms, pressures[str(int(p))]["rel_l2"]))
        del c

    config_128 = {}
    if args.config_128:
        for p in (760.0, 100.0):
            w2 = workloads.two_heads_random(n=128, L=0.4, p=p, seed=8)
            for name, lay, m0, rc in (("fast", "lattice", args.m0, args.rcond), ("surface_order_8", "nested", 8, 1e-7)):
                log("128^3 two heads at %g Torr, %s" % (p, name))
                c = Case(args, K, workloads, w2, lay, m0, rc, args.lattice_radius, "fft", "fft", 4096, 1008)
                cms, cmed = c.timed_launch(args.precision, args.steps, args.warmup, args.launch)
                config_128["%s/%d" % (name, p)] = result(
                    c.N, cms, c.accuracy(), ms_median=round(cmed, 4),
                    layout="%s m0=%d rcond=%g" % (lay, m0, rc), precompute_s=round(c.t_pre, 3))
                del c

    section42 = {}
    if args.section42:
        # the paper's pressure study at full size: a column of 5 cubes of leaves of 8 x 8 x 2
        # cells, nested shells m0 = 5 (the lattice layout's FFT forms need a cube)
        for p_o2 in (160.0, 10.0):
            w42 = workloads.paper_pressure(p_o2)
            log("Section 4.2, pO2 %g" % p_o2)
            g42 = K.Grid(w42.shape, w42.h)
            k42 = K.Kernel(w42.p_o2)
            t0 = time.perf_counter()
            t42 = K.build_tree(g42, args.max_leaf)
            o42 = K.precompute_operators(t42, k42, K.Opts(K.LAYOUT_NESTED, 5, 10, 1e-5))
            torch.cuda.synchronize()
            pre42 = time.perf_counter() - t0
            I42 = torch.from_numpy(np.ascontiguousarray(w42.I.reshape(-1))).to(case.dev)
            S42 = torch.empty_like(I42)
            for _ in range(args.warmup):
                K.eval(t42, o42, I42, w42.prefactor, out=S42)
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(case.stream)
            for _ in range(args.steps):
                K.eval(t42, o42, I42, w42.prefactor, out=S42)
            e1.record(case.stream)
            torch.cuda.synchronize()
            ms42 = e0.elapsed_time(e1) / args.steps
            N42 = int(np.prod(w42.shape))
            tg42 = torch.from_numpy(workloads.sample_targets(N42, 4096, seed=1042)).to(case.dev)
            ref42 = K.direct_eval(g42, k42, I42, w42.prefactor, tg42, fp64=True).cpu().numpy()
            got42 = S42[tg42].double().cpu().numpy()
            err42 = float(np.linalg.norm(got42 - ref42) / np.linalg.norm(ref42))
            section42["pO2_%d" % int(p_o2)] = result(
                N42, ms42, err42, grid="256 x 256 x 320, hz = %.2f hx" % (w42.h[2] / w42.h[0]),
                tree="%d cubes of leaves %s" % (t42.roots, "x".join(map(str, t42.leaf_shape))),
                layout="nested m0=5 rcond=1e-5", precompute_s=round(pre42, 3),
                paper_80_cores_s=24.7371 if p_o2 == 160.0 else 24.8619)
            del o42, t42, I42, S42

    variants = {}
    for v in [x for x in args.variants.split(",") if x]:
        log("timing variant %s" % v)
        prec, *forms = v.split("/")
        for form in forms:
            if form in ("fft", "dense") and args.layout == "lattice":
                ops.m2l_fft(form == "fft")
            if form in ("near_fft", "near_dense"):
                ops.p2p_fft(form == "near_fft")
        launch = "graph" if "graph" in forms else ("eager" if "eager" in forms else args.launch)
        vms, _ = case.timed_launch(prec, args.steps, args.warmup, launch)
        variants[v] = result(N, vms, case.accuracy(), launch=launch, speedup_vs_headline=round(ms / vms, 3))
        if args.layout == "lattice":
            ops.m2l_fft(case.m2l == "fft")
        ops.p2p_fft(case.p2p == "fft")

    if args.calibrate_copy_mib > 0:
        src = torch.ones(args.calibrate_copy_mib << 18, dtype=torch.float32, device=case.dev)
        dst = torch.empty_like(src)
        for _ in range(2):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    if args.surrogate:
        variants["surrogate"] = surrogate_variant(args, K, case, ms)

    cpu = None
    if args.cpu_targets > 0:
        # the oracle as it stands, on the host: its full-field form (zero-padded FFT
        # convolution, all N targets) and its direct form at a sample of targets
        from oracle import direct as odirect
        Ih = case.I.cpu().numpy().reshape(w.n, w.n, w.n).astype(np.float64)
        log("oracle CPU baseline: FFT full field (%d threads)" % args.cpu_threads)
        t1 = time.perf_counter()
        odirect.fft_full(Ih, (w.h,) * 3, w.p_o2, prefactor=w.prefactor, workers=args.cpu_threads)
        dt_fft = time.perf_counter() - t1
        ctg = workloads.sample_targets(N, args.cpu_targets, seed=77)
        log("oracle CPU baseline: direct sum, %d targets x %d sources" % (ctg.size, N))
        t1 = time.perf_counter()
        odirect.direct_targets(Ih, (w.h,) * 3, w.p_o2, ctg, prefactor=w.prefactor)
        dt = time.perf_counter() - t1
        cpu = {"value": N / dt_fft, "unit": "target points/s", "cores": args.cpu_threads, "kind": "oracle",
               "sample": "the oracle's FFT form of the exact sum (zero-padded FP64 convolution, scipy, %d "
                         "workers): all %d targets of the same %d^3 workload in %.1f s" % (args.cpu_threads, N, w.n, dt_fft),
               "host_cpus": os.cpu_count(),
               "direct_form": {"value": ctg.size / dt, "unit": "target points/s", "cores": odirect.num_threads(),
                               "sample": "FP64 direct sum (C/OpenMP) at %d seeded targets, %.1f s" % (ctg.size, dt),
                               "pairs_per_s_per_core": ctg.size * N / dt / odirect.num_threads()}}

    out = {
        "metric": "target points/s at <=1e-4 rel-L2 vs FP64 direct (KIFMM evaluation)",
        "value": N / (ms * 1e-3),
        "unit": "target points/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms, 4),
        "ms_per_step_median": round(med, 4),
        "ms_per_step_eager": round(ms_eager, 4),
        "ms_per_step_eager_median": round(med_eager, 4),
        "ms_per_step_serial": round(ms_serial, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"fp32": "f32", "fp64": "f64"}.get(args.precision, "f32+" + args.precision),
        "data": "synthetic",
        "config": {"workload": "streamer_channel_%d" % w.n, "n": w.n, "L_cm": w.L, "p_torr": w.p,
                   "p_o2_torr": w.p_o2, "layout": args.layout, "m0": args.m0, "check_edge": 10,
                   "rcond": args.rcond, "max_leaf": args.max_leaf, "leaf_side": tree.leaf_side,
                   "depth": tree.depth, "precision": args.precision, "m2l": case.m2l, "p2p": case.p2p,
                   "lattice_radius": (args.lattice_radius or 1.2) if args.layout == "lattice" else None,
                   "schedule": args.schedule, "launch": args.launch, "parallelism": "none"},
        "rel_l2_sampled": err,
        "accuracy_ok": err <= BAR,
        "pair_interactions_per_s_dense_equivalent": near_pairs(nb, s) / (ms * 1e-3),
        "precompute_s": round(case.t_pre, 3),
        "pass_ms_per_step": {k: round(v, 4) for k, v in pass_step.items()},
        "pass_ms_per_step_serial": {k: round(v, 4) for k, v in pass_step_serial.items()},
        "m2l_flops_per_step": m2l_flops,
        "roofline": roofline,
        "roofline_in_step": roofline_in_step,
        "roofline_m2l": roofline_m2l,
        "leaf_passes": leaf_passes,
        "pressures": pressures,
        "config_128": config_128,
        "section42": section42,
        "variants": variants,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
