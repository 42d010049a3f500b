#!/usr/bin/env python3
"""Benchmark of the SFMM gravity solve on one MI355X.

Workload: one n = 1.5 polytrope (Lane-Emden, R = 1, M = 1) of 10^6 equal-mass
particles, softening lengths from the 58th nearest neighbour, FP64, expansion
order p = 3, opening angle 0.5, leaf size 10.  A step is one full solve --
keys, sort, tree, moments, per-leaf walk, M2L/L2L/L2P, P2P, output and the
momentum reduction -- with the inputs already resident in HBM.

Prints one JSON line (see the "roofline" and "cpu_baseline" fields for the
dominant kernel's fraction of the chip's peak and the CPU oracle's rate).
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "particle gravity evals/sec (SFMM, N=1e6, theta=0.5); serving p50/p99 latency"
PEAK_FP64_TFLOPS = 78.6      # MI355X vector FP64 (256 CUs x 128 flop/clk x 2.4 GHz)
P2P_FLOPS_PER_PAIR = 22      # a pair outside both kernels (FMA = 2, rsqrt = 1)
P2P_FLOPS_SOFT = 40          # more for a pair inside a kernel: one branch of each of
                             # the two cubic-spline kernels (force and potential)


# dominant kernel of each phase: name prefix in the profiler's output and the
# sources whose hash must match the profiled build for its counters to apply
KERNELS = {
    ("fp64", "far"): ("void k_far<", ["k_far.hip", "expansions_gen.h", "sfmm_internal.h"],
                      "k_far: per-leaf M2L + L2L chain + L2P"),
    ("fp64", "near"): ("void k_p2p_wave<", ["k_near.hip", "sfmm_internal.h", "softening.h"],
                       "k_p2p_wave: softened P2P, one wave per work item, targets in scalar "
                       "registers"),
    ("fp32c", "far"): ("void k_far32<", ["k_f32c.hip", "expansions_gen.h", "sfmm_internal.h"],
                       "k_far32: per-leaf M2L (FP32 terms, FP64 sums) + L2L + L2P"),
    ("fp32c", "near"): ("void k_p2p_wave32<", ["k_f32c.hip", "sfmm_internal.h"],
                        "k_p2p_wave32: softened P2P, FP32 terms, FP64 sums, one wave per "
                        "work item"),
    # the earlier P2P shapes, still selectable (near kernel 1 to 6)
    ("fp64", "near_leaf"): ("void k_p2p_leaf<", ["k_near.hip", "sfmm_internal.h", "softening.h"],
                            "k_p2p_leaf: softened P2P, targets of a leaf in LDS"),
    ("fp64", "near_thread"): ("void k_near<", ["k_near.hip", "sfmm_internal.h", "softening.h"],
                              "k_near: softened P2P, one target particle per thread"),
    ("fp64", "near_tile"): ("void k_p2p_tile<", ["k_p2p_tile.hip", "sfmm_internal.h",
                                                 "softening.h"],
                            "k_p2p_tile: softened P2P, targets of a leaf in lane stripes, "
                            "sources staged in LDS"),
    ("fp32c", "near_leaf"): ("void k_p2p_leaf32<", ["k_f32c.hip", "sfmm_internal.h"],
                             "k_p2p_leaf32: softened P2P, FP32 terms, FP64 sums"),
    ("mutual", "far"): (("void k_m2l_mutual<", "void k_far_shared<"),
                        ["k_far.hip", "expansions_gen.h", "sfmm_internal.h"],
                        "k_m2l_mutual + k_far_shared: each unordered node pair's M2L once for "
                        "both nodes, then per-leaf L2L + L2P"),
    ("shared", "far"): (("void k_m2l_nodes<", "void k_far_shared<"),
                        ["k_far.hip", "expansions_gen.h", "sfmm_internal.h"],
                        "k_m2l_nodes + k_far_shared: per-node M2L sums, then per-leaf L2L + L2P"),
}


def near_shape(precision, leaf_size, variant):
    """Which P2P kernel a near-kernel number launches (the shapes that
    sfmm_config.near_kernel documents)."""
    if precision == "fp32c":
        return "near_leaf" if variant == 6 else "near"
    if leaf_size > 32 or variant == 1:
        return "near_thread"
    if variant == 13:
        return "near_tile"
    if variant == 6:
        return "near_leaf"
    return "near"


def measured_traffic(args, kern):
    """HBM bytes per launch of the kernel from the committed counter summary
    (FETCH_SIZE and WRITE_SIZE, each scaled by a plain copy of known size),
    or None when there is none for this workload or the kernel's sources
    have changed since the counters were taken."""
    import hashlib

    path = os.path.join(ROOT, "profiles", "traffic.json")
    n_tag = f"{args.n:.0e}".replace("+0", "").replace("+", "")
    tag = f"{args.workload}_{n_tag}_{args.precision}"
    if not os.path.exists(path):
        return None
    entry = json.load(open(path)).get(tag)
    if entry is None:
        return None
    prefixes = kern[0] if isinstance(kern[0], tuple) else (kern[0],)
    h = hashlib.sha256()
    for fn in kern[1]:
        with open(os.path.join(ROOT, "paper_2602_05804_amd", "csrc", fn), "rb") as f:
            h.update(f.read())
    total = 0.0
    for pre in prefixes:  # every kernel of the phase, each profiled on these sources
        recs = [r for name, r in entry["kernels"].items() if name.startswith(pre)]
        if len(recs) != 1 or recs[0].get("sources") != kern[1] \
                or recs[0].get("sources_sha256") != h.hexdigest():
            return None
        total += recs[0]["bytes_per_dispatch"]
    return round(total)


# algorithmic HBM bytes per particle of the tree phase: keys (24 B read,
# 12 B written), 8 radix passes over (key, index) (12 B read + 12 B written
# each), the gather (40 B read + 4 B index, 80 B written: arrays + records)
TREE_BYTES_PER_PARTICLE = 36 + 8 * 24 + 124
PEAK_HBM_GBS = 8000.0


def solve_fraction(args, work, total_ms):
    """Whole-solve fraction: the sum over phases of the time each would take at
    its own bound (far and near at the FP64 peak, the tree at the HBM peak)
    over the measured time of a solve.  The walk has no arithmetic or
    bandwidth roof of its own (dependent gathers and branches); it counts as
    measured time only."""
    ideal = {"far": work["far"] / (PEAK_FP64_TFLOPS * 1e12) * 1e3,
             "near": work["near"] / (PEAK_FP64_TFLOPS * 1e12) * 1e3,
             "tree": args.n * TREE_BYTES_PER_PARTICLE / (PEAK_HBM_GBS * 1e9) * 1e3}
    tot = sum(ideal.values())
    return {"ideal_ms": {k: round(v, 4) for k, v in ideal.items()}, "ideal_total_ms": round(tot, 4),
            "measured_ms": round(total_ms, 4), "frac": round(tot / total_ms, 4)}


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--n", type=int, default=1_000_000)
    ap.add_argument("--workload", choices=["polytrope", "binary", "cloud", "plummer"],
                    default="polytrope",
                    help="polytrope: one n=1.5 star (the headline); binary: two stars of "
                         "N/2 at 3R; cloud: log-normal clumpy cloud; plummer: Plummer sphere")
    ap.add_argument("--precision", choices=["fp64", "fp32c"], default="fp64")
    ap.add_argument("--theta", type=float, default=0.5)
    ap.add_argument("--order", type=int, default=3)
    ap.add_argument("--leaf-size", type=int, default=16,
                    help="leaf size of the headline solve (16: the autotuner's pick for the 1e6 "
                         "polytrope, 5.8 ms per solve against 6.1 at 10)")
    ap.add_argument("--near-kernel", type=int, default=13,
                    help="P2P kernel shape of the headline solve (13, targets in lanes: the "
                         "autotuner's pick at leaf size 16)")
    ap.add_argument("--no-same-fp32c", dest="same_fp32c", action="store_false",
                    help="skip the FP32C solve of the headline workload (same input and leaf "
                         "size, its error measured over every particle by the CPU oracle)")
    ap.add_argument("--fp32c-leaf-size", type=int, default=10,
                    help="leaf size of the FP32C block")
    ap.add_argument("--fp32c-same-near-kernel", type=int, default=6,
                    help="P2P shape of the FP32C solve on the headline input (leaf size "
                         "16: shape 6 is the faster FP32C shape there)")
    ap.add_argument("--serve-leaf-size", type=int, default=10,
                    help="leaf size of the serving runs without tuned settings")
    ap.add_argument("--walk", choices=["level", "leaf"], default="level",
                    help="level: each (ancestor, source) test once per level; "
                         "leaf: Algorithm 1 with one stack walk per leaf")
    ap.add_argument("--far", choices=["leaf", "shared", "mutual"], default="shared",
                    help="shared: each node's M2L list once, then L2L per leaf (the caching "
                         "the paper proposes); leaf: every leaf evaluates its ancestors' "
                         "lists (the paper's replicated walk), also timed beside shared")
    ap.add_argument("--autotune", action="store_true",
                    help="pick the kernel shapes (and with --autotune-leaf the leaf size) by a "
                         "timed search on this input before the timed run")
    ap.add_argument("--autotune-leaf", action="store_true")
    ap.add_argument("--cpu-leaves", type=int, default=1500,
                    help="leaves the CPU oracle walks for the baseline and the parity sample")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--calib-copy-mib", type=int, default=0,
                    help="before the workload, copy a buffer of this many MiB three times "
                         "(a plain copy kernel of known size, to scale HBM counters)")
    ap.add_argument("--serve-requests", type=int, default=512,
                    help="requests in the serving run (Poisson arrivals at 200/s, N log-uniform "
                         "in [1e3, 1e6], 4 KDK steps each); 0 skips it")
    ap.add_argument("--no-serve-fp32c", dest="serve_fp32c", action="store_false",
                    help="serve the trace in FP64 only (by default it is also served in FP32C)")
    ap.add_argument("--no-serve-tuned", dest="serve_tuned", action="store_false",
                    help="skip the FP64 serving run whose packs take the leaf size and P2P "
                         "shape the autotuner picked for their size bucket")
    ap.add_argument("--serve-low-rate", type=float, default=100.0,
                    help="arrival rate of a second FP64 serving run below the GPU's capacity "
                         "(0 skips it)")
    ap.add_argument("--fp32c-n", type=int, default=2_000_000,
                    help="particles of the FP32C block: the binary polytrope (two stars of "
                         "N/2 at 3R); 0 skips it")
    ap.add_argument("--fp32c-steps", type=int, default=5)
    ap.add_argument("--serve-pack", type=float, default=16e6,
                    help="particles per packed solve in the serving run")
    ap.add_argument("--serve-inflight", type=float, default=24e6,
                    help="particles admitted at once in the serving run (bounds a step)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: this build runs on one GPU only (asked for --gpus {args.gpus}); "
              "a multi-GPU solve is not part of it.", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_2602_05804_amd as sfmm
    import workloads

    if not torch.cuda.is_available():
        print("bench.py: no GPU visible", file=sys.stderr)
        sys.exit(1)
    if args.calib_copy_mib > 0:
        nb = args.calib_copy_mib * 2 ** 20 // 8
        src = torch.ones(nb, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        log(f"copy calibration: 3 x {args.calib_copy_mib} MiB read + written")
        del src, dst
    log(f"generating {args.workload} N={args.n}")
    if args.workload == "polytrope":
        x, m, h = workloads.polytrope(args.n, seed=2)
        wl = f"n=1.5 polytrope, N={args.n}, h from 58 neighbours, seed 2"
    elif args.workload == "binary":
        x, m, h, _ = workloads.binary_polytrope(args.n // 2)
        wl = f"binary n=1.5 polytrope, 2 x {args.n // 2}, separation 3R, seeds 3/4"
    elif args.workload == "cloud":
        x, m, h = workloads.lognormal_cloud(args.n)
        wl = f"log-normal cloud (sigma 2, k^-4, 128^3), N={args.n}, seeds 5/6"
    else:
        x, m, h = workloads.plummer(args.n, seed=1)
        wl = f"Plummer sphere a=1 M=1, N={args.n}, seed 1"
    xd, md, hd = (torch.from_numpy(a).cuda() for a in (x, m, h))
    cfg = {"leaf_size": args.leaf_size, "walk": args.walk, "far": args.far,
           "near_kernel": args.near_kernel}
    if args.autotune:
        from paper_2602_05804_amd import autotune

        log("autotune")
        res = autotune.search(xd, md, hd, theta=args.theta, order=args.order,
                              precision=args.precision, log=log,
                              leaf_sizes=autotune.LEAF_SIZES if args.autotune_leaf
                              else (args.leaf_size,),
                              base={"walk": args.walk, "far": args.far})
        cfg = res["config"]
        args.leaf_size = cfg["leaf_size"]
    solver = sfmm.Solver(**cfg)
    acc = torch.empty((args.n, 3), dtype=torch.float64, device="cuda")
    pot = torch.empty((args.n,), dtype=torch.float64, device="cuda")
    log(f"warmup {args.warmup}")
    for _ in range(args.warmup):
        solver.solve(xd, md, hd, theta=args.theta, order=args.order, acc=acc, pot=pot,
                     precision=args.precision)
    torch.cuda.synchronize()
    st = solver.stats()
    log(f"timed {args.steps} steps")
    solver.timing_start(args.steps)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        solver.solve(xd, md, hd, theta=args.theta, order=args.order, acc=acc, pot=pot,
                     precision=args.precision)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    phases = solver.timing_stop()
    dt = (t1 - t0) / args.steps
    value = args.n / dt
    st = solver.stats()
    mom = float(np.linalg.norm(st["momentum"]) / st["momentum_abs"])
    ph_mean = {k: float(np.mean([p[k] for p in phases])) for k in sfmm.PHASES}
    log("phase ms: " + ", ".join(f"{k}={v:.3f}" for k, v in ph_mean.items()))

    # algorithmic work of the arithmetic kernels
    p = args.order
    # M2L evaluations actually made: replicated per leaf, or once per node pair
    n_m2l = st["n_m2l_unique"] if args.far in ("shared", "mutual") else st["n_m2l"]
    m2l_flops = (n_m2l // 2 * (sfmm.FLOPS["m2l_pair"][p] + 1) if args.far == "mutual"
                 else n_m2l * (sfmm.FLOPS["m2l"][p] + 1))
    far_flops = (m2l_flops + st["n_l2l"] * sfmm.FLOPS["l2l"][p]
                 + args.n * sfmm.FLOPS["l2p"][p])
    near_flops = st["n_p2p_pairs"] * P2P_FLOPS_PER_PAIR + st["n_p2p_soft_pairs"] * P2P_FLOPS_SOFT
    work = {"far": far_flops, "near": near_flops}
    dom = max(("far", "near"), key=lambda k: ph_mean[k])
    # the dominant kernel's own duration: the P2P kernel alone is timed by
    # its own events (phase near_kernel); the far phase is its kernels
    dom_ms = ph_mean["near_kernel"] if dom == "near" and ph_mean["near_kernel"] > 0 else ph_mean[dom]
    achieved = work[dom] / (dom_ms * 1e-3) / 1e12
    kern = KERNELS[(args.far if args.far in ("shared", "mutual") and dom == "far" else args.precision,
                    near_shape(args.precision, args.leaf_size, cfg.get("near_kernel", 0))
                    if dom == "near" else dom)]
    roofline = {"bound": "alu", "kernel": kern[2],
                "achieved": round(achieved, 3), "peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s",
                "frac": round(achieved / PEAK_FP64_TFLOPS, 4),
                "traffic": measured_traffic(args, kern),
                "flops_per_launch": work[dom], "ms_per_launch": round(dom_ms, 4)}
    per_phase = {k: {"ms": round(v, 4)} for k, v in ph_mean.items()}
    for k, wk in (("far", "far"), ("near", "near"), ("near_kernel", "near")):
        if ph_mean[k] <= 0:
            continue
        tf = work[wk] / (ph_mean[k] * 1e-3) / 1e12
        per_phase[k].update(tflops=round(tf, 3), frac=round(tf / PEAK_FP64_TFLOPS, 4))

    result = {
        "metric": METRIC, "value": value, "unit": "particles/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": dt * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": {"fp64": "f64", "fp32c": "f32+f64"}[args.precision],
        "data": "synthetic",
        "config": {"workload": wl,
                   "N": args.n, "theta": args.theta, "order": p, "leaf_size": args.leaf_size,
                   "precision": args.precision, "G": 1.0, "r_kern": 2.0, "walk": args.walk,
                   "far": args.far, "h_min": float(h.min()), "h_max": float(h.max()),
                   "kernels": {k: cfg.get(k, 0) for k in ("near_kernel", "far_kernel")},
                   "autotuned": bool(args.autotune)},
        "roofline": roofline,
        "phases": per_phase,
        "counts": {k: st[k] for k in ("num_nodes", "num_leaves", "max_depth", "n_m2l",
                                      "n_m2l_unique", "n_l2l", "n_p2p_leaf_pairs",
                                      "n_p2p_pairs", "n_p2p_soft_pairs", "leaf_slot_m2l",
                                      "leaf_slot_p2p", "n_leaf_overflow", "max_leaf_m2l",
                                      "max_leaf_p2p")},
        "momentum_residual": mom,
        "solve_fraction": solve_fraction(args, work, dt * 1e3),
    }

    if args.far == "shared":
        # the paper's replicated far field on the same input, for comparison
        rep = sfmm.Solver(leaf_size=args.leaf_size, walk=args.walk, far="leaf")
        for _ in range(args.warmup):
            rep.solve(xd, md, hd, theta=args.theta, order=args.order, acc=acc, pot=pot,
                      precision=args.precision)
        rep.timing_start(args.steps)
        torch.cuda.synchronize()
        r0 = time.perf_counter()
        for _ in range(args.steps):
            rep.solve(xd, md, hd, theta=args.theta, order=args.order, acc=acc, pot=pot,
                      precision=args.precision)
        torch.cuda.synchronize()
        r1 = time.perf_counter()
        rph = rep.timing_stop()
        rst = rep.stats()
        rdt = (r1 - r0) / args.steps
        result["far_leaf_mode"] = {
            "value": args.n / rdt, "ms_per_step": rdt * 1e3,
            "far_ms": float(np.mean([q["far"] for q in rph])),
            "n_m2l": rst["n_m2l"],
            "note": "every leaf evaluates all of its ancestors' M2L lists (replicated)"}
        log(f"replicated far field: {args.n / rdt:.4g} particles/s")
        rep.close()
        # the headline solve's outputs again (the comparison run overwrote them)
        solver.solve(xd, md, hd, theta=args.theta, order=args.order, acc=acc, pot=pot,
                     precision=args.precision)
        torch.cuda.synchronize()

    same32 = None
    if args.precision == "fp64" and args.same_fp32c and args.leaf_size <= 16:
        same32 = fp32c_same_workload(args, xd, md, hd, wl)
        result["fp32c_same_workload"] = same32["line"]
    if not args.no_cpu:
        result.update(cpu_baseline(args, x, m, h, acc, pot, p, same32))
    if args.fp32c_n > 0 and args.precision == "fp64" and args.workload == "polytrope":
        del xd, md, hd, acc, pot
        solver.close()
        torch.cuda.empty_cache()
        result["fp32c"] = fp32c_block(args)
    if args.serve_requests > 0:
        result["serving"] = serving(args)
    print(json.dumps(result), flush=True)


def cpu_info():
    """Host CPU model and core counts (nproc = cores this process may use)."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        nproc = len(os.sched_getaffinity(0))
    except AttributeError:
        nproc = os.cpu_count()
    return model, nproc, os.cpu_count()


# the paper's own timings (Sect. 4), context only: relative to its non-symmetric
# FMM on CPUs, no absolute throughput is published
PAPER_TIMINGS = ("SFMM wall time +7% vs the paper's FMM at theta=0.5 (+12% mean over "
                 "theta 0.1-0.6), Plummer sphere of 1e5 particles, Xeon Gold 6244 nodes, "
                 "16 cores; O(N log N) scaling, +7% to +26% vs FMM for N > 1e5 (Sect. 4)")


def fp32c_same_workload(args, xd, md, hd, wl):
    """The FP32-compensated form on the headline's input and leaf size, timed
    like the headline (its error against the oracle is filled in by
    cpu_baseline, over every particle)."""
    import numpy as np
    import torch

    import paper_2602_05804_amd as sfmm

    log("fp32c on the headline workload")
    s = sfmm.Solver(leaf_size=args.leaf_size, walk=args.walk, far=args.far,
                    near_kernel=args.fp32c_same_near_kernel)
    a32 = torch.empty((args.n, 3), dtype=torch.float64, device="cuda")
    p32 = torch.empty((args.n,), dtype=torch.float64, device="cuda")
    for _ in range(max(args.warmup, 1)):
        s.solve(xd, md, hd, theta=args.theta, order=args.order, acc=a32, pot=p32,
                precision="fp32c")
    torch.cuda.synchronize()
    s.timing_start(args.steps)
    t0 = time.perf_counter()
    for _ in range(args.steps):
        s.solve(xd, md, hd, theta=args.theta, order=args.order, acc=a32, pot=p32,
                precision="fp32c")
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / args.steps
    ph = s.timing_stop()
    st = s.stats()
    s.close()
    line = {"workload": wl, "leaf_size": args.leaf_size,
            "near_kernel": args.fp32c_same_near_kernel, "value": args.n / dt,
            "unit": "particles/s", "ms_per_step": dt * 1e3,
            "phases_ms": {k: round(float(np.mean([q[k] for q in ph])), 4) for k in sfmm.PHASES},
            "momentum_residual": float(np.linalg.norm(st["momentum"]) / st["momentum_abs"]),
            "error_vs_fp64_oracle": None}
    return {"line": line, "acc": a32.cpu().numpy(), "pot": p32.cpu().numpy()}


def cpu_baseline(args, x, m, h, acc, pot, p, same32=None):
    """The oracle on the host: Algorithm 1's loop over leaves on all host cores
    for every particle (also the parity check of every particle, of the FP64
    solve and, when given, of the FP32-compensated one on the same input),
    and the serial oracle on one core over a sample of leaves, extrapolated."""
    import numpy as np

    import oracle

    a_gpu = acc.cpu().numpy()
    p_gpu = pot.cpu().numpy()
    model, nproc, ncpu = cpu_info()
    log("cpu oracle: tree build")
    c0 = time.perf_counter()
    t = oracle.Tree(x, m, h, leaf_size=args.leaf_size, order=p)
    c1 = time.perf_counter()
    log(f"cpu oracle: every leaf on the host cores ({nproc} available)")
    oa, op, ost = t.solve_parallel(args.theta, nthreads=nproc)
    c2 = time.perf_counter()
    nb = np.linalg.norm(oa, axis=1)
    floor = 1e-6 * np.sqrt((nb ** 2).mean())
    err = np.linalg.norm(a_gpu - oa, axis=1) / np.maximum(nb, floor)
    perr = np.abs(p_gpu - op) / np.abs(op)
    out = {"cpu_baseline": {
        "value": args.n / (c2 - c0), "unit": "particles/s", "cores": ost["threads"],
        "kind": "oracle",
        "sample": (f"FP64 oracle, Algorithm 1's loop over leaves on {ost['threads']} OpenMP "
                   f"threads: serial tree + moments ({c1 - c0:.1f} s) and the per-leaf "
                   f"walk/M2L/L2L/L2P/P2P of all {ost['n_leaves_done']} leaves "
                   f"({c2 - c1:.1f} s), every particle of the workload"),
        "cpu_model": model, "nproc": nproc, "os_cpu_count": ncpu,
        "paper_timings_context": PAPER_TIMINGS}}
    out["parity_all"] = {"particles": int(args.n), "max_rel_acc_err": float(err.max()),
                         "rms_rel_acc_err": float(np.sqrt((err ** 2).mean())),
                         "max_rel_pot_err": float(perr.max()),
                         "rms_rel_pot_err": float(np.sqrt((perr ** 2).mean()))}
    if same32 is not None:
        e32 = np.linalg.norm(same32["acc"] - oa, axis=1) / np.maximum(nb, floor)
        p32 = np.abs(same32["pot"] - op) / np.abs(op)
        same32["line"]["error_vs_fp64_oracle"] = {
            "particles": int(args.n), "rms_rel_acc_err": float(np.sqrt((e32 ** 2).mean())),
            "max_rel_acc_err": float(e32.max()), "rms_rel_pot_err": float(np.sqrt((p32 ** 2).mean()))}
    # the serial oracle on one core: a sample of leaves, extrapolated
    rng = np.random.default_rng(0)
    nl = t.num_leaves
    leaves = t.leaves()
    pick = rng.choice(nl, min(args.cpu_leaves, nl), replace=False)
    nd = t.nodes()
    perm = t.perm()
    tg = perm[nd["lo"][leaves[pick]]]  # one particle per picked leaf
    log(f"cpu oracle: {len(pick)} leaves on one core")
    c3 = time.perf_counter()
    sa, sp, sst = t.solve(args.theta, targets=tg)
    c4 = time.perf_counter()
    same = bool(np.array_equal(sa, oa[tg]) and np.array_equal(sp, op[tg]))
    per_leaf = (c4 - c3) / max(sst["n_leaves_done"], 1)
    t_full = (c1 - c0) + per_leaf * nl
    out["cpu_baseline"]["serial_1core"] = {
        "value": args.n / t_full, "unit": "particles/s", "cores": 1,
        "sample": (f"serial FP64 oracle: full tree + moments ({c1 - c0:.1f} s) plus the "
                   f"per-leaf walk/M2L/L2L/L2P/P2P of {sst['n_leaves_done']} random leaves "
                   f"({c4 - c3:.1f} s), extrapolated to all {nl} leaves"),
        "equals_threaded_result": same}
    return out


PEAK_FP32_TFLOPS = 157.3  # MI355X vector FP32 (packed FP32 issue; this build issues FP32
                          # unpacked, at the FP64 rate)


def fp32c_block(args):
    """The FP32-compensated form on the binary polytrope (two n=1.5 stars of
    N/2 particles at 3R): throughput, phase split, the P2P kernel against the
    FP32 vector peak, and its error against the FP64 oracle on sampled targets
    with the momentum residual."""
    import numpy as np
    import torch

    import oracle
    import paper_2602_05804_amd as sfmm
    import workloads

    n = args.fp32c_n
    log(f"fp32c: generating binary polytrope 2 x {n // 2}")
    x, m, h, _ = workloads.binary_polytrope(n // 2)
    xd, md, hd = (torch.from_numpy(a).cuda() for a in (x, m, h))
    solver = sfmm.Solver(leaf_size=args.fp32c_leaf_size)
    acc = torch.empty((n, 3), dtype=torch.float64, device="cuda")
    pot = torch.empty((n,), dtype=torch.float64, device="cuda")
    for _ in range(2):
        solver.solve(xd, md, hd, theta=args.theta, order=args.order, acc=acc, pot=pot,
                     precision="fp32c")
    torch.cuda.synchronize()
    solver.timing_start(args.fp32c_steps)
    t0 = time.perf_counter()
    for _ in range(args.fp32c_steps):
        solver.solve(xd, md, hd, theta=args.theta, order=args.order, acc=acc, pot=pot,
                     precision="fp32c")
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / args.fp32c_steps
    phases = solver.timing_stop()
    st = solver.stats()
    ph = {k: float(np.mean([q[k] for q in phases])) for k in sfmm.PHASES}
    flops = st["n_p2p_pairs"] * P2P_FLOPS_PER_PAIR + st["n_p2p_soft_pairs"] * P2P_FLOPS_SOFT
    ach = flops / (ph["near_kernel"] * 1e-3) / 1e12
    a_gpu, p_gpu = acc.cpu().numpy(), pot.cpu().numpy()
    solver.close()
    log("fp32c: oracle on 1500 sampled targets")
    t = oracle.Tree(x, m, h, leaf_size=args.fp32c_leaf_size, order=args.order)
    tg = np.random.default_rng(2).choice(n, 1500, replace=False)
    oa, op, _ = t.solve(args.theta, targets=tg)
    nb = np.linalg.norm(oa, axis=1)
    err = np.linalg.norm(a_gpu[tg] - oa, axis=1) / nb
    perr = np.abs(p_gpu[tg] - op) / np.abs(op)
    out = {"workload": f"binary n=1.5 polytrope, 2 x {n // 2}, separation 3R, seeds 3/4",
           "value": n / dt, "unit": "particles/s", "ms_per_step": dt * 1e3,
           "phases_ms": {k: round(v, 4) for k, v in ph.items()},
           "roofline": {"bound": "alu", "kernel": "P2P, FP32 pair terms, FP64 sums",
                        "achieved": round(ach, 3), "peak": PEAK_FP32_TFLOPS, "unit": "TFLOP/s",
                        "frac": round(ach / PEAK_FP32_TFLOPS, 4), "traffic": None,
                        "flops_per_launch": flops, "ms_per_launch": round(ph["near_kernel"], 4)},
           "parity_sample": {"targets": 1500, "rms_rel_acc_err": float(np.sqrt((err ** 2).mean())),
                             "max_rel_acc_err": float(err.max()),
                             "rms_rel_pot_err": float(np.sqrt((perr ** 2).mean()))},
           "momentum_residual": float(np.linalg.norm(st["momentum"]) / st["momentum_abs"]),
           "counts": {k: st[k] for k in ("num_nodes", "num_leaves", "n_m2l_unique",
                                         "n_p2p_pairs", "n_p2p_soft_pairs")}}
    log(f"fp32c: {out['value']:.4g} particles/s, rms err {out['parity_sample']['rms_rel_acc_err']:.3g}")
    del xd, md, hd, acc, pot
    torch.cuda.empty_cache()
    return out


def serving(args):
    """Continuous batching of a stream of independent solves: FP64 and FP32C on
    the same arrival trace (200 requests/s) with the HBM budget at 0.8 x free
    memory, FP64 again under a small budget so that admission queues
    requests, and FP64 with the same trace stretched to a lower arrival rate
    that the GPU keeps up with (latency then measures service, not queueing),
    and FP64 once more with each pack's leaf size and P2P shape taken from the
    autotuner's pick for its size bucket."""
    import numpy as np
    import torch

    import workloads
    from paper_2602_05804_amd import serve

    log(f"serving: generating {args.serve_requests} requests")
    reqs = workloads.serving_stream(count=args.serve_requests, seed=7, rate=200.0,
                                    nmin=1e3, nmax=1e6)
    ntot = sum(len(q.m) for q in reqs)
    out = {"requests": len(reqs), "particles": ntot, "rate_per_s": 200.0, "steps_per_request": 4,
           "pack_particles": args.serve_pack, "max_particles_in_flight": args.serve_inflight,
           "trace": "Poisson arrivals at 200/s, N = 10^U(3,6), Plummer/polytrope alternating, "
                    "seed 7"}
    runs = [("fp64", None, 200.0, False)] + (
        [("fp32c", None, 200.0, False)] if args.serve_fp32c else []) + [
        ("fp64", 3_000_000, 200.0, False)]
    if args.serve_low_rate > 0:
        runs.append(("fp64", None, args.serve_low_rate, False))
    tuned = None
    if args.serve_tuned:
        # one search per size bucket from 2^10 to the pack cap, on one system
        # of that size mixing the trace's two kinds (a Plummer sphere and a
        # polytrope side by side)
        from paper_2602_05804_amd import autotune

        def make_input(n):
            xa, ma, ha = workloads.plummer(n // 2, seed=21)
            xb, mb, hb = workloads.polytrope(n - n // 2, seed=22)
            xb = xb + np.array([250.0, 0.0, 0.0])  # beyond the sphere's 100 a
            return tuple(torch.from_numpy(np.ascontiguousarray(np.concatenate(p))).cuda()
                         for p in ((xa, xb), (ma * 0.5, mb * 0.5), (ha, hb)))

        t0 = time.perf_counter()
        sizes = [2 ** k for k in range(10, int(np.log2(args.serve_pack)) + 1)]
        tuned = autotune.tune_buckets(sizes, make_input, theta=args.theta, order=args.order,
                                      base={"walk": args.walk, "far": args.far}, log=log)
        out["tuned_buckets"] = {str(k): v for k, v in tuned.items()}
        out["tuning_s"] = round(time.perf_counter() - t0, 2)
        runs.append(("fp64", None, 200.0, True))
    for prec, small_budget_n, rate, use_tuned in runs:
        ex = serve.GpuExecutor(precision=prec, theta=args.theta, order=args.order,
                               leaf_size=args.serve_leaf_size, far=args.far,
                               pack_particles=args.serve_pack,
                               tuned=tuned if use_tuned else None)
        free, _ = torch.cuda.mem_get_info()
        budget = 0.8 * free if small_budget_n is None else ex.footprint(small_budget_n)
        jobs = serve.jobs_from_stream(reqs, steps=4)
        for j in jobs:  # the same trace, stretched to the run's arrival rate
            j.arrival *= 200.0 / rate
        log(f"serving: {prec} at {rate:g}/s, budget {budget / 2**30:.1f} GiB "
            f"({ex.bytes_per_particle} B/particle)")
        rep = serve.Server(ex, hbm_budget=budget,
                           max_particles=args.serve_inflight).run(jobs)
        summ = rep.summary()
        summ["hbm_budget_gib"] = budget / 2 ** 30
        summ["bytes_per_particle"] = ex.bytes_per_particle
        key = prec if small_budget_n is None else f"{prec}_small_budget"
        if rate != 200.0:
            key = f"{prec}_rate{rate:g}"
        if use_tuned:
            key = f"{prec}_tuned"
        out[key] = {k: (round(v, 4) if isinstance(v, float) else v) for k, v in summ.items()}
        log(f"serving {key}: " + ", ".join(f"{k}={v}" for k, v in out[key].items()))
        del ex
        torch.cuda.empty_cache()
    return out


if __name__ == "__main__":
    main()
