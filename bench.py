#!/usr/bin/env python3
"""Benchmark of the PDE signature-kernel Gram batch on one MI355X.

Workload (a "step"): the full 128 x 128 Gram matrix of two batches of 256-point
paths in R^8 with a time channel appended (d = 9), Gaussian increments with std
0.3/sqrt(256), dyadic order 1: increments, increment Gram and the explicit
sweep over 16384 pairs x 510 x 510 fine cells = 4.26e9 cell updates.  Inputs
are resident in HBM before the timed region; every step recomputes everything.

Prints ONE JSON line:
  value       grid-cell updates per second (whole job, one GPU)
  roofline    the sweep kernel against the FP64 VALU issue rate (3.125
              FP64-equivalent operations per fine cell: two FP64 cell
              operations and 9/4 FP32 FMAs counted at half an operation)
  cpu_baseline the FP64 oracle on the host cores, on a bounded sample
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "Goursat grid-cell updates/s (Gram batch) and pairs/s at stated rel err vs FP64"

# MI355X FP64 VALU: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz double operations
# per second (78.6 TFLOP/s counting an FMA as two).  The published float32
# peak is twice this (packed float32 instructions, which these kernels do not
# use).
VALU_PEAK_TOPS = 256 * 4 * 16 * 2.4e9 / 1e12


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--eager", action="store_true",
                    help="launch the library call every step instead of replaying its hipGraph")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="run only a plain 1 GiB device-to-device copy (the known-size kernel that "
                         "scales the FETCH_SIZE / WRITE_SIZE counters)")
    ap.add_argument("--no-autotune", action="store_true",
                    help="keep the built-in launch rules instead of autotuning (untimed) first")
    ap.add_argument("--scheme", choices=["explicit", "implicit"], default="explicit",
                    help="gram workload: the explicit scheme (default, the reported metric) or the "
                         "implicit one")
    ap.add_argument("--cpu-sample-pairs", type=int, default=0,
                    help="pairs of the workload timed on the CPU oracle (0: all)")
    ap.add_argument("--workload", choices=["gram", "mmd", "ragged", "increment_gram", "corrector",
                                           "lifted", "fig3", "reduce", "pair"],
                    default="gram",
                    help="gram: the 128 x 128 Gram batch (default, the reported metric); "
                         "pair: one 32-point pair in R^2 at order 0 (latency per call); "
                         "mmd: unbiased MMD^2 of 64 vs 64 512-point paths with its gradient; "
                         "ragged: 4096 independent pairs of uneven lengths; "
                         "increment_gram: the coarse Gram of the Gram batch written to HBM; "
                         "corrector: order-3 values of 65536 held-out pairs by the learned "
                         "corrector with fallback, against the plain order-3 solve; "
                         "lifted: the RBF-lifted Gram (sigma 0.5) of the Gram batch; "
                         "fig3: the Figure 3 protocol (time to reach 1e-3 of a P5 target on 5 "
                         "Brownian pairs, against length and against channels); "
                         "reduce: the reduced measure of 30 fBM paths (support 6)")
    return ap.parse_args()


def sweep_ops_per_cell(d: int, lam: int) -> float:
    """VALU work per fine cell in FP64-operation equivalents: the cell update
    (one double add and one double FMA) plus the coarse inner product (d float
    FMAs per coarse cell, shared by 4^lam fine cells; a float FMA counts 1/2,
    after the published float32 peak, which is twice the double one)."""
    return 2.0 + 0.5 * d / float(4 ** lam)


def grad_ops_per_cell(d: int, lam: int) -> float:
    """VALU work per fine cell of the Gram gradient, in FP64-operation
    equivalents: the forward cell and its share of the coarse inner product
    (as in sweep_ops_per_cell), the adjoint cell (two double FMAs), its
    coefficient-gradient product (one FMA) and the two increment contractions
    (2 d double FMAs per coarse cell, shared by 4^lam fine cells).  The
    recomputation of the forward values from checkpoints is not counted."""
    return sweep_ops_per_cell(d, lam) + 3.0 + 2.0 * d / float(4 ** lam)


# checkpoint traffic of the gradient kernel per fine cell (written once, read
# once): R + 2^lam doubles per lane every C steps of R 2^lam cells, with R = 4
# rows per lane and C the segment length (see grad_args.h)
def grad_checkpoint_bytes_per_cell(d: int, lam: int) -> float:
    R = 4
    S = 1 << lam
    floats_reg = 32 // (2 if lam == 0 else 1)
    C = max(1, floats_reg // (R * S)) + max(1, 64 // (R * S))
    return 2.0 * 8.0 * (R + S) / (R * S * C)


# the files the Gram sweep kernel compiles from (its translation unit and headers)
SWEEP_SOURCES = ("sweep_k0_l1.hip", "sweep_inst.h", "dispatch.h", "sweep_fwd_kernel.h",
                 "sweep_args.h")
TRAFFIC_PROFILE = os.path.join(ROOT, "profiles", "pmc_traffic_sweep_kernel_gram128_L256_d9_lam1.md")


def measured_traffic():
    """HBM bytes per sweep launch from the committed counter summary, or None
    when the sweep's sources have changed since the counters were taken."""
    import hashlib
    import re
    try:
        text = open(TRAFFIC_PROFILE).read()
        rec = json.loads(re.search(r"```json\n(.*?)\n```", text, re.S).group(1))
        csrc = os.path.join(ROOT, "paper_2006_14794_amd", "csrc")
        h = hashlib.sha256(b"".join(open(os.path.join(csrc, f), "rb").read()
                                    for f in SWEEP_SOURCES)).hexdigest()[:16]
    except (OSError, AttributeError, ValueError):
        return None
    return rec["traffic_bytes"] if h == rec["source_hash"] else None


def host_cpu():
    """The host's CPU model (first "model name" line of /proc/cpuinfo) and its
    logical CPU count."""
    model = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return {"cpu_model": model, "nproc": os.cpu_count()}


def single_thread_rate(solve, xs, ys, lam, n=32):
    """Cells/s of the oracle on one thread over the first n pairs of a sample."""
    xs, ys = xs[:n], ys[:n]
    t0 = time.perf_counter()
    solve(xs, ys, lam, nthreads=1)
    dt = time.perf_counter() - t0
    cells = sum(((len(a) - 1) << lam) * ((len(b) - 1) << lam) for a, b in zip(xs, ys))
    return cells / dt


def cpu_baseline(X, Y, lam, n_sample, K_gpu, repeats=3, scheme="explicit"):
    """Time the FP64 oracle on the workload's pairs (all of them unless
    n_sample is given: a seeded sample), on all host threads, median of
    ``repeats`` runs, and report the GPU output's error on the same pairs."""
    import oracle
    solve = oracle.pairs_implicit if scheme == "implicit" else oracle.pairs
    nx, ny = X.shape[0], Y.shape[0]
    if n_sample and n_sample < nx * ny:
        idx = np.random.default_rng(1).choice(nx * ny, size=n_sample, replace=False)
    else:
        idx = np.arange(nx * ny)
    xs = [X[i // ny].astype(np.float64) for i in idx]
    ys = [Y[i % ny].astype(np.float64) for i in idx]
    threads = oracle.max_threads()
    solve(xs[:8], ys[:8], lam)  # load + warm
    times = []
    for _ in range(repeats):
        t0 = time.perf_counter()
        ref = solve(xs, ys, lam, nthreads=threads)
        times.append(time.perf_counter() - t0)
    dt = float(np.median(times))
    cells = len(idx) * ((X.shape[1] - 1) << lam) * ((Y.shape[1] - 1) << lam)
    err = np.abs(K_gpu.reshape(-1)[idx] - ref) / np.maximum(1.0, np.abs(ref))
    what = (f"all {nx * ny} Gram pairs" if len(idx) == nx * ny
            else f"{len(idx)} of the {nx * ny} Gram pairs (seeded)")
    return {"value": cells / dt, "unit": "cells/s", "cores": threads, "kind": "oracle",
            "sample": f"{what}, all host threads, median of {repeats} runs of {dt:.2f} s",
            "gpu_max_err_on_sample": float(err.max()),
            "single_thread_cells_per_s": single_thread_rate(solve, xs, ys, lam), **host_cpu()}


SETTLE_S = 0.25  # untimed, synchronised repetitions of a step before its warm-up
_settled = {"steps": 0}


def time_steps(fn, steps, warmup):
    """Run fn untimed until the device has executed it back to back for
    SETTLE_S seconds (each repetition synchronised, so nothing queues up:
    after the untimed set-up the GPU clocks take a few tens of milliseconds of
    work to come up, and a short warm-up alone leaves the first timed steps
    slow), then warmup + steps times; the timed steps run back to back between
    two synchronisations, with one HIP event pair on the launch stream around
    them.  Returns ([average step duration from the events, ms] * steps, wall
    seconds of the timed steps).  (Events around every single step would
    separate consecutive launches and add about a tenth of a millisecond per
    step on this hardware.)"""
    import torch
    t_end = time.perf_counter() + SETTLE_S
    n = 0
    while n < 1 or time.perf_counter() < t_end:
        fn()
        torch.cuda.synchronize()
        n += 1
    _settled["steps"] += n
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    start = torch.cuda.Event(enable_timing=True)
    end = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    start.record(stream)
    for _ in range(steps):
        fn()
    end.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    return [start.elapsed_time(end) / steps] * steps, wall


def emit(rec):
    """Print the JSON line, with the untimed settle repetitions it ran."""
    rec["settle"] = {"seconds_per_timing": SETTLE_S, "steps": _settled["steps"]}
    print(json.dumps(rec), flush=True)


def make_step(call, capture, eager):
    """The timed step: a replay of the call's hipGraph (captured once, before
    the warm-up), or with ``eager`` the call itself."""
    if eager:
        return call, "eager"
    g = capture()
    return g.replay, "hipGraph replay"


def bench_mmd(args):
    """Unbiased MMD^2 between 64 generated paths (the parameters) and 64 OU
    targets, 512 points in R^4, dyadic order 1: value and gradient in X."""
    import torch
    import paper_2006_14794_amd as sk
    import workloads
    lam = 1
    X, Y = workloads.mmd_paths()
    n, L, d = X.shape
    m = Y.shape[0]
    dev = torch.device("cuda:0")
    Xt, Yt = torch.from_numpy(X).to(dev), torch.from_numpy(Y).to(dev)
    ws = torch.empty(sk.workspace_bytes(3, Xt, Yt, lam, 4), dtype=torch.uint8, device=dev)

    def call():
        sk.sigkernel_mmd2(Xt, Yt, lam, grad=True, workspace=ws)

    step, launch = make_step(call, lambda: sk.capture_mmd2(Xt, Yt, lam, grad=True)[0],
                             args.eager)
    per, wall = time_steps(step, args.steps, args.warmup)
    ms = wall * 1e3 / args.steps
    cells = ((L - 1) << lam) ** 2
    fwd_pairs = n * (n - 1) // 2 + m * (m - 1) // 2 + n * m
    # the gradient solves the off-diagonal upper triangle of Kxx and all of Kxy
    bwd_pairs = n * (n - 1) // 2 + n * m
    work = (fwd_pairs + bwd_pairs) * cells
    # the dominant kernel on its own: the gradient launch of the cross term
    # (64 x 64 pairs), with its increments and point-gradient launches, timed
    # with events over the same number of back-to-back calls
    wxy = torch.full((n, m), -2.0 / (n * m), dtype=torch.float32, device=dev)
    ws_b = torch.empty(sk.workspace_bytes(2, Xt, Yt, lam, 0), dtype=torch.uint8, device=dev)

    def cross():
        sk.sigkernel_gram_backward(Xt, Yt, wxy, lam, need_y=False, workspace=ws_b)

    per_b, _ = time_steps(cross, args.steps, args.warmup)
    t_b = float(np.mean(per_b)) / 1e3
    ops = grad_ops_per_cell(d, lam) * n * m * cells
    rec = {
        "metric": "Goursat grid-cell updates/s, MMD^2 forward + adjoint",
        "value": work / (ms / 1e3), "unit": "cells/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": "unbiased MMD^2, 64 random walks vs 64 OU paths, 512 points, "
                               "d=4, dyadic order 1, value + gradient in X",
                   "forward_pairs": fwd_pairs, "adjoint_pairs": bwd_pairs,
                   "fine_cells_per_pair": cells},
        "avg_event_ms": float(np.mean(per)), "launch": launch,
        "roofline": {"bound": "alu", "achieved": ops / t_b / 1e12, "peak": VALU_PEAK_TOPS,
                     "unit": "Tops/s", "frac": ops / t_b / 1e12 / VALU_PEAK_TOPS,
                     "traffic": None,
                     "kernel": "grad_kernel: gradient of the cross term (64 x 64 pairs), events "
                               "around the backward call (increments, gradient, point sums)",
                     "avg_launch_ms": t_b * 1e3, "ops_per_cell": grad_ops_per_cell(d, lam),
                     "checkpoint_bytes_per_cell": grad_checkpoint_bytes_per_cell(d, lam)},
    }
    if not args.no_cpu_baseline:
        import oracle
        ns = X.shape[0]  # the whole workload: all 64 generated and 64 target paths
        Xs, Ys = X[:ns].astype(np.float64), Y[:ns].astype(np.float64)
        threads = oracle.max_threads()
        t0 = time.perf_counter()
        Kxx = oracle.gram(Xs, Xs, lam, nthreads=threads)
        Kyy = oracle.gram(Ys, Ys, lam, nthreads=threads)
        Kxy = oracle.gram(Xs, Ys, lam, nthreads=threads)
        oracle.mmd2_unbiased(Kxx, Kyy, Kxy)
        wxx, _, wxy_s = oracle.mmd2_weights(ns, ns)
        oracle.gram_backward(Xs, Xs, wxx, lam, nthreads=threads)
        oracle.gram_backward(Xs, Ys, wxy_s, lam, nthreads=threads)
        dt = time.perf_counter() - t0
        # the oracle solves full Gram blocks (both halves of the symmetric ones)
        # and both backward blocks in full: count the cells it actually sweeps
        s_cells = (3 * ns * ns + 2 * ns * ns) * cells
        rec["cpu_baseline"] = {
            "value": s_cells / dt, "unit": "cells/s", "cores": threads, "kind": "oracle",
            "sample": f"the whole workload: MMD^2 value and gradient of all {ns} vs {ns} paths "
                      f"(full Gram blocks and full backward blocks, {s_cells:.3g} cells), all "
                      f"host threads, {dt:.2f} s", **host_cpu()}
    emit(rec)


def bench_ragged(args):
    """4096 independent pairs, lengths uniform in [64, 1024] (drawn per path),
    d = 16, dyadic order 2, one persistent length-sorted launch."""
    import torch
    import paper_2006_14794_amd as sk
    import workloads
    from paper_2006_14794_amd import RaggedPaths
    lam = 2
    xs, ys = workloads.ragged_pairs()
    X = RaggedPaths.from_list(xs, "cuda")
    Y = RaggedPaths.from_list(ys, "cuda")
    tune = None if args.no_autotune else sk.autotune("pair", X, Y, lam)[0]
    out = torch.empty(len(xs), dtype=torch.float32, device="cuda")
    ws = torch.empty(sk.workspace_bytes(0, X, Y, lam, 0), dtype=torch.uint8, device="cuda")

    def call():
        sk.sigkernel_pair(X, Y, lam, out=out, workspace=ws)

    graph = None
    if not args.eager:
        graph, out = sk.capture_pair(X, Y, lam)
    step, launch = (call, "eager") if graph is None else (graph.replay, "hipGraph replay")
    per, wall = time_steps(step, args.steps, args.warmup)
    ms = wall * 1e3 / args.steps
    cells = sum(((len(a) - 1) << lam) * ((len(b) - 1) << lam) for a, b in zip(xs, ys))
    # the same pairs with bf16-rounded increments (float32 products and sums)
    out16 = torch.empty_like(out)

    def step16():
        sk.sigkernel_pair(X, Y, lam, gram_precision="bf16", out=out16, workspace=ws)
    per16, wall16 = time_steps(step16, args.steps, args.warmup)
    d = xs[0].shape[1]
    ops = cells * sweep_ops_per_cell(d, lam)
    avg_s = float(np.mean(per)) / 1e3
    rec = {
        "metric": "Goursat grid-cell updates/s, batched uneven lengths",
        "value": cells / (ms / 1e3), "unit": "cells/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": "4096 independent pairs, lengths U[64,1024], d=16, dyadic order 2",
                   "fine_cells": cells},
        "pairs_per_s": len(xs) / (ms / 1e3),
        "avg_event_ms": float(np.mean(per)), "launch": launch, "tuning": tune,
        "bf16_increments_ms_per_step": wall16 * 1e3 / args.steps,
        "roofline": {"bound": "alu", "achieved": ops / avg_s / 1e12, "peak": VALU_PEAK_TOPS,
                     "unit": "Tops/s", "frac": ops / avg_s / 1e12 / VALU_PEAK_TOPS,
                     "traffic": None, "kernel": "pair_band_kernel (events around the timed calls)",
                     "ops_per_cell": sweep_ops_per_cell(d, lam)},
    }
    if not args.no_cpu_baseline:
        import oracle
        rng = np.random.default_rng(1)
        idx = rng.choice(len(xs), size=args.cpu_sample_pairs or len(xs), replace=False)
        sx = [xs[i].astype(np.float64) for i in idx]
        sy = [ys[i].astype(np.float64) for i in idx]
        t0 = time.perf_counter()
        ref = oracle.pairs(sx, sy, lam, nthreads=oracle.max_threads())
        dt = time.perf_counter() - t0
        scells = sum(((len(a) - 1) << lam) * ((len(b) - 1) << lam) for a, b in zip(sx, sy))
        got = out.cpu().numpy()[idx]
        got16 = out16.cpu().numpy()[idx]

        def errs(g):
            e = np.abs(g - ref) / np.maximum(1, np.abs(ref))
            return {"max": float(e.max()), "median": float(np.median(e))}
        rec["cpu_baseline"] = {
            "value": scells / dt, "unit": "cells/s", "cores": oracle.max_threads(),
            "kind": "oracle", "sample": f"{len(idx)} of the 4096 pairs, all host threads, "
                                        f"{dt:.2f} s",
            "gpu_max_err_on_sample": errs(got)["max"],
            "single_thread_cells_per_s": single_thread_rate(oracle.pairs, sx, sy, lam),
            **host_cpu()}
        rec["err_vs_fp64_oracle"] = {"f32_increments": errs(got), "bf16_increments": errs(got16)}
    emit(rec)


# FP64 operations counted for one double-precision exp: a two-constant range
# reduction (round, two FMAs), a degree-12 polynomial (12 FMAs) and the
# scaling by the power of two (about 4 operations).
EXP_OPS = 20


def lifted_ops_per_pair(m: int, n: int, d: int, lam: int) -> int:
    """Algorithmic FP64 operations of one RBF-lifted pair on P_lambda: per
    node pair the static kernel (d differences, d FMAs, one scaling, one exp),
    per coarse cell the second difference and the cell factor (5), per fine
    cell the update (2)."""
    return ((m + 1) * (n + 1) * (2 * d + 1 + EXP_OPS) + m * n * 5
            + (m << lam) * (n << lam) * 2)


def bench_lifted(args):
    """The RBF-lifted Gram (Gaussian static kernel, sigma 0.5) of the Gram
    batch: 128 x 128 pairs of 256-point paths, d = 8 + time, dyadic order 1."""
    import torch
    import paper_2006_14794_amd as sk
    import workloads
    lam, sigma = 1, 0.5
    X, Y = workloads.gram_batch()
    nx, L, d = X.shape
    ny = Y.shape[0]
    Xt, Yt = torch.from_numpy(X).cuda(), torch.from_numpy(Y).cuda()
    out = torch.empty((nx, ny), dtype=torch.float32, device="cuda")
    ws = torch.empty(sk.workspace_bytes(8, Xt, Yt, lam, 0), dtype=torch.uint8, device="cuda")
    recs = {}
    for scheme in ("explicit", "implicit"):
        def call(scheme=scheme):
            sk.sigkernel_gram_lifted(Xt, Yt, lam, sigma=sigma, scheme=scheme, out=out,
                                     workspace=ws)
        graph = None if args.eager else sk.CapturedCalls(call)
        step, launch = (call, "eager") if graph is None else (graph.replay, "hipGraph replay")
        per, wall = time_steps(step, args.steps, args.warmup)
        recs[scheme] = (per, wall, launch)
        if scheme == "explicit":
            K = out.cpu().numpy()
    per, wall, launch = recs["explicit"]
    ms = wall * 1e3 / args.steps
    M, N = (L - 1) << lam, (L - 1) << lam
    cells = nx * ny * M * N
    ops = nx * ny * lifted_ops_per_pair(L - 1, L - 1, d, lam)
    avg_s = float(np.mean(per)) / 1e3
    rec = {
        "metric": "Goursat grid-cell updates/s, RBF-lifted Gram batch",
        "value": cells / (ms / 1e3), "unit": "cells/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": "RBF-lifted gram 128x128 pairs, 256-point paths, d=8+time, "
                               "dyadic order 1, sigma 0.5", "static_kernel": "exp(-|a-b|^2/2s^2)",
                   "pairs": nx * ny, "fine_cells_per_pair": M * N},
        "pairs_per_s": nx * ny / (ms / 1e3), "launch": launch,
        "implicit_ms_per_step": recs["implicit"][1] * 1e3 / args.steps,
        "roofline": {"bound": "alu", "achieved": ops / avg_s / 1e12, "peak": VALU_PEAK_TOPS,
                     "unit": "Tops/s", "frac": ops / avg_s / 1e12 / VALU_PEAK_TOPS,
                     "traffic": None,
                     "kernel": "lifted_sweep_kernel (events around the timed steps: nodes + sweep)",
                     "avg_launch_ms": avg_s * 1e3, "ops_per_pair": ops // (nx * ny),
                     "exp_ops": EXP_OPS},
    }
    if not args.no_cpu_baseline:
        import oracle
        threads = oracle.max_threads()
        n_s = args.cpu_sample_pairs or nx * ny
        rng = np.random.default_rng(1)
        idx = np.sort(rng.choice(nx * ny, size=n_s, replace=False))
        sx = [X[i // ny].astype(np.float64) for i in idx]
        sy = [Y[i % ny].astype(np.float64) for i in idx]
        oracle.lifted_rbf_pairs(sx[:8], sy[:8], lam, sigma)
        times = []
        for _ in range(3):
            t0 = time.perf_counter()
            ref = oracle.lifted_rbf_pairs(sx, sy, lam, sigma, nthreads=threads)
            times.append(time.perf_counter() - t0)
        dt = float(np.median(times))
        err = np.abs(K.reshape(-1)[idx] - ref) / np.maximum(1.0, np.abs(ref))
        what = (f"all {nx * ny} Gram pairs" if n_s == nx * ny
                else f"{n_s} of the {nx * ny} Gram pairs (seeded)")
        rec["cpu_baseline"] = {"value": n_s * M * N / dt, "unit": "cells/s", "cores": threads,
                               "kind": "oracle",
                               "sample": f"{what}, all host threads, median of 3 runs of "
                                         f"{dt:.2f} s",
                               "gpu_max_err_on_sample": float(err.max())}
    emit(rec)


FIG3_LENGTHS = (10, 20, 50, 100, 200, 500, 1000, 2000)
FIG3_DIMS = (2, 8, 32, 128, 512, 2048)


def bench_fig3(args):
    """The performance experiment of Figure 3: for N = 5 pairs of Brownian
    paths, the smallest dyadic order whose values lie within 1e-3 of the
    order-5 values (the P5 target) on every pair, and the time of the
    solve at that order -- on the GPU, and for the FP64 oracle on the host --
    against the length (d = 2) and against the channels (length 10).  The
    fitted exponents of time against length show how each side scales."""
    import torch
    import paper_2006_14794_amd as sk
    import workloads
    n_pairs, acc, target_order = 5, 1e-3, 5
    configs = [(L, 2) for L in FIG3_LENGTHS] + [(10, d) for d in FIG3_DIMS if d != 2]
    rows = []
    for L, d in configs:
        X, Y = workloads.fig3_pairs(L, d, n_pairs)
        Xt, Yt = torch.from_numpy(X).cuda(), torch.from_numpy(Y).cuda()
        target = sk.sigkernel_pair(Xt, Yt, target_order).cpu().numpy().astype(np.float64)
        lam = target_order
        for cand in range(target_order):
            v = sk.sigkernel_pair(Xt, Yt, cand).cpu().numpy().astype(np.float64)
            if np.all(np.abs(v - target) <= acc):
                lam = cand
                break
        graph, _ = sk.capture_pair(Xt, Yt, lam)
        reps = 20
        per, _ = time_steps(graph.replay, reps, 3)
        row = {"length": L, "dim": d, "order": lam, "gpu_ms": float(np.mean(per))}
        if not args.no_cpu_baseline:
            import oracle
            xs, ys = X.astype(np.float64), Y.astype(np.float64)
            oracle.pairs(xs[:1], ys[:1], 0)
            t0 = time.perf_counter()
            ref = oracle.pairs(xs, ys, lam, nthreads=oracle.max_threads())
            row["cpu_ms"] = (time.perf_counter() - t0) * 1e3
            got = sk.sigkernel_pair(Xt, Yt, lam).cpu().numpy()
            row["gpu_err_vs_oracle"] = float(np.max(np.abs(got - ref) / np.maximum(1, np.abs(ref))))
        rows.append(row)
        print(json.dumps(row), file=sys.stderr, flush=True)

    def exponent(key):
        pts = [(r["length"], r[key]) for r in rows if r["dim"] == 2 and r["length"] >= 100
               and key in r]
        if len(pts) < 2:
            return None
        lx = np.log([p[0] for p in pts])
        ly = np.log([p[1] for p in pts])
        return float(np.polyfit(lx, ly, 1)[0])

    longest = [r for r in rows if r["dim"] == 2][-1]
    rec = {
        "metric": "time to reach 1e-3 of the P5 target, 5 Brownian pairs (Figure 3 protocol)",
        "value": longest["gpu_ms"], "unit": "ms", "n_gpus": 1, "steps": 20, "warmup": 3,
        "ms_per_step": longest["gpu_ms"], "higher_is_better": False, "scaling": "strong",
        "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"Figure 3 protocol: 5 Brownian pairs; value at length "
                               f"{longest['length']}, d=2", "pairs": n_pairs,
                   "accuracy": acc, "target_order": target_order},
        "sweep": rows,
        "time_vs_length_exponent": {"gpu": exponent("gpu_ms"), "cpu_oracle": exponent("cpu_ms")},
    }
    if not args.no_cpu_baseline:
        rec["cpu_baseline"] = {"value": longest["cpu_ms"], "unit": "ms",
                               "cores": min(n_pairs, __import__("oracle").max_threads()),
                               "kind": "oracle",
                               "sample": f"the same 5 pairs at length {longest['length']}, "
                                         "OpenMP over the pairs"}
    emit(rec)


def bench_reduce(args):
    """The reduced-measure experiment: 30 fBM paths (Hurst exponent drawn from
    {0.2, 0.5, 0.8}, 50 points, time channel), their symmetric signature Gram
    at dyadic order 6, and the penalty of eq. (min_lasso) for a support of 6
    found by 40 bisection rounds of 3000 proximal-gradient iterations."""
    import torch
    import paper_2006_14794_amd as sk
    import workloads
    lam_order, support, iters, rounds = 6, 6, 3000, 40
    P, H = workloads.fbm_paths(n_points=50)
    Pt = torch.from_numpy(P).cuda()
    K = sk.sigkernel_gram(Pt, None, lam_order, symmetric=True)

    def gram_step():
        sk.sigkernel_gram(Pt, None, lam_order, symmetric=True, out=K)
    per_g, wall_g = time_steps(gram_step, args.steps, args.warmup)
    res = {}

    def search_step():
        res["r"] = sk.reduced_measure_support(K, support, iters, rounds)
    per_s, wall_s = time_steps(search_step, max(1, args.steps // 4), 1)
    beta, lam, step = res["r"]
    b = beta.cpu().numpy()
    nz = np.nonzero(b)[0]
    ms = (wall_g / args.steps + wall_s / max(1, args.steps // 4)) * 1e3
    total_iters = iters * rounds
    rec = {
        "metric": "reduced measure of 30 fBM paths: signature Gram + support search time",
        "value": ms, "unit": "ms", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": ms, "higher_is_better": False, "scaling": "strong", "vs_baseline": None,
        "dtype": "f64", "data": "synthetic",
        "config": {"workload": "30 fBM paths (H in {0.2,0.5,0.8}), 50 points + time, "
                               "dyadic order 6, support 6", "iters_per_round": iters,
                   "rounds": rounds},
        "gram_ms": float(np.mean(per_g)), "search_ms": float(np.mean(per_s)),
        "us_per_iteration": float(np.mean(per_s)) * 1e3 / total_iters,
        "selected": {"paths": nz.tolist(), "hurst": H[nz].tolist(),
                     "weights": b[nz].tolist(), "lam": lam.item(), "step": step.item()},
    }
    if not args.no_cpu_baseline:
        import oracle
        from oracle import reduced_measure as rm
        t0 = time.perf_counter()
        Kr = oracle.gram(P.astype(np.float64), P.astype(np.float64), lam_order,
                         nthreads=oracle.max_threads())
        tg = time.perf_counter() - t0
        t0 = time.perf_counter()
        rb, rl = rm.ista_support(Kr, np.full(30, 1.0 / 30), support, iters, rounds)
        ts = time.perf_counter() - t0
        rec["cpu_baseline"] = {"value": (tg + ts) * 1e3, "unit": "ms",
                               "cores": oracle.max_threads(), "kind": "oracle",
                               "sample": f"the whole experiment: Gram {tg * 1e3:.0f} ms (all "
                                         f"threads), search {ts * 1e3:.0f} ms (numpy)",
                               "selected_paths": np.nonzero(rb)[0].tolist(), "lam": rl}
    emit(rec)


def bench_increment_gram(args):
    """The coarse increment Gram G0 of the 128 x 128 Gram batch (255 x 255 per
    pair, d = 9) written to HBM row after row: bound by the 4-byte
    write per coarse cell.  Timed in the dense layout and with rows padded
    to 256 floats (1 KB); the bytes counted are G0's own (the padding column
    is not written) plus the points read."""
    import torch
    import paper_2006_14794_amd as sk
    import workloads
    X, Y = workloads.gram_batch()
    Xt, Yt = torch.from_numpy(X).cuda(), torch.from_numpy(Y).cuda()
    nx, L, d = X.shape
    n = L - 1
    ld_pad = (n + 3) // 4 * 4
    outs = {"padded": torch.empty((nx, Y.shape[0], n, ld_pad), dtype=torch.float32, device="cuda"),
            "dense": torch.empty((nx, Y.shape[0], n, n), dtype=torch.float32, device="cuda")}
    nbytes = nx * Y.shape[0] * n * n * 4 + (X.size + Y.size) * 4
    recs = {}
    for layout in ("padded", "dense"):
        for prec in ("f32", "bf16"):
            def step():
                sk.sigkernel_increment_gram(Xt, Yt, precision=prec, out=outs[layout],
                                            ld=ld_pad if layout == "padded" else None)
            per, wall = time_steps(step, args.steps, args.warmup)
            avg = float(np.mean(per)) / 1e3
            recs[f"{layout}_{prec}"] = {"ms": avg * 1e3, "hbm_GBps": nbytes / avg / 1e9,
                                        "frac_of_8TBps": nbytes / avg / 8e12}
    head = recs["dense_f32"]
    rec = {"metric": "increment Gram bytes written/s", "value": head["hbm_GBps"],
           "unit": "GB/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
           "ms_per_step": head["ms"], "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "f32", "data": "synthetic",
           "config": {"workload": "coarse Gram of 128 x 128 pairs, 255 x 255 each, d = 9"},
           "roofline": {"bound": "hbm", "achieved": head["hbm_GBps"], "peak": 8000.0,
                        "unit": "GB/s", "frac": head["frac_of_8TBps"], "traffic": None},
           "layouts": recs}
    if not args.no_cpu_baseline:
        import oracle
        # a sample of the pairs through the oracle's FP64 Gram on one host
        # thread, its entries counted at the 4 bytes the GPU writes; the
        # sample's entries are also compared with the GPU's dense float32 ones
        rng = np.random.default_rng(0)
        pick = rng.choice(nx * Y.shape[0], size=2048, replace=False)
        Xd, Yd = X.astype(np.float64), Y.astype(np.float64)
        t0 = time.perf_counter()
        refs = [oracle.increment_gram(Xd[k // Y.shape[0]], Yd[k % Y.shape[0]]) for k in pick]
        dt = time.perf_counter() - t0
        sk.sigkernel_increment_gram(Xt, Yt, out=outs["dense"])  # float32 inputs
        dense = outs["dense"].reshape(-1, n, n)
        err = max(float(np.abs(dense[int(k)].cpu().numpy() - r).max()) for k, r in
                  zip(pick[:64], refs[:64]))
        rec["cpu_baseline"] = {"value": len(pick) * n * n * 4 / dt / 1e9, "unit": "GB/s",
                               "cores": 1, "kind": "oracle",
                               "sample": f"{len(pick)} of the {nx * Y.shape[0]} pairs on one host "
                                         f"thread, {dt:.2f} s", **host_cpu()}
        rec["max_abs_err_vs_oracle_on_64_pairs"] = err
    emit(rec)


def bench_corrector(args):
    """65536 held-out pairs (256 points, R^8): the learned corrector (order-0
    features, network, device-side fallback to the plain order-3 solve)
    against the plain order-3 solve, both timed over whole batches."""
    import torch
    import paper_2006_14794_amd as sk
    import workloads
    from paper_2006_14794_amd import corrector as corr
    n = 65536
    X, Y = workloads.corrector_pairs(workloads.SEED_CORRECTOR_EVAL, n)
    Xc, Yc = torch.from_numpy(X).cuda(), torch.from_numpy(Y).cuda()
    del X, Y
    model = sk.Corrector.load(os.path.join(ROOT, "paper_2006_14794_amd", "corrector_weights.npz"))
    plain = torch.empty(n, dtype=torch.float32, device="cuda")

    def plain_step():
        sk.sigkernel_pair(Xc, Yc, 3, out=plain)
    res = {}

    def learned_step():
        res["out"] = model.predict(Xc, Yc, kappa=corr.KAPPA, tol=1e-3, chunk=n)
    # the non-learned alternative: the plain solves at orders 0 and 1,
    # extrapolated to order 3 under an error c 4^-lambda (c from k1 - k0)
    k0b = torch.empty(n, dtype=torch.float32, device="cuda")
    k1b = torch.empty(n, dtype=torch.float32, device="cuda")
    ext = torch.empty(n, dtype=torch.float64, device="cuda")

    def extrapolation_step():
        sk.sigkernel_pair(Xc, Yc, 0, out=k0b)
        sk.sigkernel_pair(Xc, Yc, 1, out=k1b)
        torch.add(k0b.double(), k1b.double() - k0b.double(), alpha=(63.0 / 64.0) * (4.0 / 3.0),
                  out=ext)
    per_p, wall_p = time_steps(plain_step, args.steps, args.warmup)
    per_l, wall_l = time_steps(learned_step, args.steps, args.warmup)
    per_x, wall_x = time_steps(extrapolation_step, args.steps, args.warmup)
    ms_p = wall_p * 1e3 / args.steps
    ms_l = wall_l * 1e3 / args.steps
    ms_x = wall_x * 1e3 / args.steps
    out, err, fb = res["out"]
    k3 = plain.cpu().numpy().astype(np.float64)
    e = np.abs(out.cpu().numpy() - k3) / np.abs(k3)
    ex = np.abs(ext.cpu().numpy() - k3) / np.abs(k3)
    cells3 = n * (255 << 3) ** 2
    # the network on the matrix cores: 3x3 convolutions, 32 output channels
    # (layer 1's 72 reduction terms padded to 80), plus the dense head
    macs = sum(o * o * 32 * k for o, k in ((32, 80), (16, 288), (8, 288), (4, 288))) + 2 * 512
    rec = {
        "metric": "order-3-equivalent grid-cell updates/s, learned corrector with fallback",
        "value": cells3 / (ms_l / 1e3), "unit": "cells/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms_l, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64+bf16", "data": "synthetic",
        "config": {"workload": "65536 held-out pairs, 256-point paths in R^8, std 0.3/16, "
                               f"order-0 input, order-3 target, kappa {corr.KAPPA}, tol 1e-3"},
        "plain_order3": {"ms_per_step": ms_p, "cells_per_s": cells3 / (ms_p / 1e3)},
        "speedup_vs_plain_order3": ms_p / ms_l,
        "fallback_fraction": float(fb.float().mean().item()),
        "rel_err_vs_order3": {"median": float(np.median(e)),
                              "p99": float(np.percentile(e, 99)), "max": float(e.max())},
        "extrapolation_orders_0_1": {
            "ms_per_step": ms_x,
            "rel_err_vs_order3": {"median": float(np.median(ex)), "p99": float(np.percentile(ex, 99)),
                                  "max": float(ex.max())},
            "note": "k0 + (63/64)(4/3)(k1 - k0), no learning: more accurate and faster than the "
                    "learned corrector on this workload"},
        "network_mfma": {"flop_per_pair": 2 * macs, "unit": "TFLOP/s",
                         "achieved_whole_call": 2 * macs * n / (ms_l / 1e3) / 1e12,
                         "peak": 2500.0,
                         "note": "whole predict call time; the fused network kernel's own "
                                 "duration is in profiles/"},
    }
    if not args.no_cpu_baseline:
        # the FP64 oracle's plain order-3 solve on 8192 seeded pairs of the
        # 65536 (about ten seconds on the host)
        import oracle
        idx = np.random.default_rng(2).choice(n, size=8192, replace=False)
        Xh, Yh = Xc.cpu().numpy(), Yc.cpu().numpy()
        xs = [Xh[i].astype(np.float64) for i in idx]
        ys = [Yh[i].astype(np.float64) for i in idx]
        threads = oracle.max_threads()
        oracle.pairs(xs[:4], ys[:4], 3)  # load + warm
        t0 = time.perf_counter()
        ref = oracle.pairs(xs, ys, 3, nthreads=threads)
        dt = time.perf_counter() - t0
        cells = len(idx) * (255 << 3) ** 2
        rec["cpu_baseline"] = {
            "value": cells / dt, "unit": "cells/s", "cores": threads, "kind": "oracle",
            "sample": f"plain order-3 solve of {len(idx)} of the 65536 pairs (seeded), all host threads, "
                      f"{dt:.2f} s; the metric's per-pair work at order 3, so the rate compares "
                      "with value directly",
            "gpu_plain_max_err_on_sample": float(np.max(np.abs(k3[idx] - ref) / np.abs(ref))),
            "extrapolated_whole_workload_s": dt * n / len(idx),
            "extrapolation": "by fine-cell count (every pair has the same cells)",
            **host_cpu()}
    emit(rec)


def bench_pair(args):
    """One pair of 32-point paths in R^2 (N(0, 1/32) increments), dyadic order
    0: the latency of a single sigkernel_pair call, eager and as a hipGraph
    replay, with the straight-segment pair against the closed form."""
    import torch
    import paper_2006_14794_amd as sk
    import workloads
    import oracle
    x, y, xs, ys = workloads.single_pair()
    dev = torch.device("cuda:0")
    xt, yt = torch.from_numpy(x[None]).to(dev), torch.from_numpy(y[None]).to(dev)
    out = torch.empty(1, dtype=torch.float32, device=dev)
    ws = torch.empty(sk.workspace_bytes(0, xt, yt, 0, 0), dtype=torch.uint8, device=dev)

    def call():
        sk.sigkernel_pair(xt, yt, 0, out=out, workspace=ws)
    graph, gout = sk.capture_pair(xt, yt, 0)
    per_e, wall_e = time_steps(call, args.steps, args.warmup)
    per_g, wall_g = time_steps(graph.replay, args.steps, args.warmup)
    us_e = wall_e * 1e6 / args.steps
    us_g = wall_g * 1e6 / args.steps
    # the value is the faster of the two ways to call it (on this runtime a
    # graph replay of its two small launches costs more than the eager call)
    us_best, best_path = (us_g, "hipgraph_replay") if us_g <= us_e else (us_e, "eager_call")
    ref = float(oracle.pairs([x.astype(np.float64)], [y.astype(np.float64)], 0)[0])
    k = float(gout.item())
    # the straight segments: the scheme converges to k = sum_k <a,b>^k / (k!)^2
    # under dyadic refinement (order 0 is a single cell, 1 + <a,b>)
    xsd, ysd = torch.from_numpy(xs[None]).to(dev), torch.from_numpy(ys[None]).to(dev)
    c = float(np.dot((xs[1] - xs[0]).astype(np.float64), (ys[1] - ys[0]).astype(np.float64)))
    closed = oracle.straight_segment_kernel(c)
    seg = {f"order_{o}": sk.sigkernel_pair(xsd, ysd, o).item() for o in (0, 2, 4, 6, 8)}
    rec = {
        "metric": "pairs/s of single-pair calls (latency), 32-point pair in R^2, order 0",
        "value": 1e6 / us_best, "unit": "pairs/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": us_best / 1e3, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": "one pair, 32 points in R^2, N(0, 1/32) increments from 0, "
                               "dyadic order 0; and one straight-segment pair"},
        "value_from": best_path,
        "us_per_pair": {"hipgraph_replay": us_g, "eager_call": us_e,
                        "gpu_event_per_launch": per_g[0] * 1e3},
        "rel_err_vs_oracle": abs(k - ref) / abs(ref),
        "straight_segment": {"inner_product": c, "closed_form": closed, "gpu": seg,
                             "rel_err": {k: abs(v - closed) / abs(closed) for k, v in seg.items()}},
    }
    if not args.no_cpu_baseline:
        xd, yd = [x.astype(np.float64)] * 100000, [y.astype(np.float64)] * 100000
        t0 = time.perf_counter()
        oracle.pairs(xd, yd, 0, nthreads=1)
        dt = time.perf_counter() - t0
        rec["cpu_baseline"] = {"value": len(xd) / dt, "unit": "pairs/s", "cores": 1,
                               "kind": "oracle",
                               "sample": f"the same pair solved {len(xd)} times on one host thread, "
                                         f"{dt:.2f} s", **host_cpu()}
    emit(rec)


def copy_calibration(args):
    """A plain device-to-device copy of 1 GiB, repeated: the reference
    dispatch for the HBM byte counters."""
    import torch
    n = (1 << 30) // 4
    a = torch.empty(n, dtype=torch.float32, device="cuda").fill_(1.0)
    b = torch.empty_like(a)
    for _ in range(max(1, args.steps)):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes_read": 4 * n, "copy_bytes_written": 4 * n,
                      "dispatches": max(1, args.steps)}), flush=True)


def main():
    args = parse()
    if args.copy_calibration:
        copy_calibration(args)
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only: --gpus {args.gpus} is not supported "
              "(the multi-GPU sharding is a design note, not built)", file=sys.stderr)
        sys.exit(2)
    if args.workload == "mmd":
        bench_mmd(args)
        return
    if args.workload == "ragged":
        bench_ragged(args)
        return
    if args.workload == "increment_gram":
        bench_increment_gram(args)
        return
    if args.workload == "corrector":
        bench_corrector(args)
        return
    if args.workload == "lifted":
        bench_lifted(args)
        return
    if args.workload == "fig3":
        bench_fig3(args)
        return
    if args.workload == "reduce":
        bench_reduce(args)
        return
    if args.workload == "pair":
        bench_pair(args)
        return

    import torch
    import paper_2006_14794_amd as sk
    import workloads

    lam = 1
    X, Y = workloads.gram_batch()
    nx, L, d = X.shape
    ny = Y.shape[0]
    dev = torch.device("cuda:0")
    Xt = torch.from_numpy(X).to(dev)
    Yt = torch.from_numpy(Y).to(dev)
    # launch tuning is set-up: timed candidates run before the warm-up
    scheme = args.scheme
    tune = None if args.no_autotune else sk.autotune("gram", Xt, Yt, lam, scheme=scheme)[0]
    out = torch.empty((nx, ny), dtype=torch.float32, device=dev)
    ws = torch.empty(sk.workspace_bytes(1, Xt, Yt, lam, 0), dtype=torch.uint8, device=dev)

    def call():
        sk.sigkernel_gram(Xt, Yt, lam, scheme=scheme, out=out, workspace=ws)

    graph = None
    if not args.eager:
        graph, out = sk.capture_gram(Xt, Yt, lam, scheme=scheme)
    step, launch = (call, "eager") if graph is None else (graph.replay, "hipGraph replay")
    # HIP events on the stream the step is launched on (torch's current stream)
    per_launch_ms, wall = time_steps(step, args.steps, args.warmup)
    ms_per_step = wall * 1e3 / args.steps

    M, N = (L - 1) << lam, (L - 1) << lam
    cells = nx * ny * M * N
    value = cells / (ms_per_step / 1e3)
    pairs_per_s = nx * ny / (ms_per_step / 1e3)

    avg_launch_s = float(np.mean(per_launch_ms)) / 1e3
    ops = cells * sweep_ops_per_cell(d, lam)
    achieved = ops / avg_launch_s / 1e12
    rec = {
        "metric": METRIC,
        "value": value,
        "unit": "cells/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "gram 128x128 pairs, 256-point paths, d=8+time, dyadic order 1",
                   "pairs": nx * ny, "fine_cells_per_pair": M * N, "sweep_state": "f64",
                   "scheme": scheme,
                   "increment_gram": "f32"},
        "pairs_per_s": pairs_per_s,
        "launch": launch,
        "tuning": tune,
        "roofline": {
            "bound": "alu",
            "achieved": achieved,
            "peak": VALU_PEAK_TOPS,
            "unit": "Tops/s",
            "frac": achieved / VALU_PEAK_TOPS,
            "traffic": measured_traffic(),
            "kernel": "sweep_kernel (events around the timed steps: increments + sweep)",
            "avg_launch_ms": avg_launch_s * 1e3,
            "ops_per_cell": sweep_ops_per_cell(d, lam),
        },
    }
    if not args.no_cpu_baseline:
        n_sample = args.cpu_sample_pairs
        rec["cpu_baseline"] = cpu_baseline(X, Y, lam, n_sample, out.cpu().numpy(),
                                          scheme=scheme)
    emit(rec)


if __name__ == "__main__":
    main()
