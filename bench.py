#!/usr/bin/env python
"""Benchmark: batched BDF-Newton cell-steps/s on one MI355X.

Workload (the timed "step"): one accepted step of the grouped BDF
integrator over 2^20 independent cells, each a 10-species random
mass-action network with 20 reactions (rates log-uniform in [1e-3, 1e8]
per cell, initial states uniform on the simplex), BDF order <= 5, Newton
with the FP64 10 x 10 block LU, rtol 1e-6, atol 1e-10.  Inputs are seeded
and synthetic and resident in HBM before timing starts.  value = cells x
accepted steps / wall time.

Also reported on the same GPU: the FP32-LU + FP64-refinement form on the
same workload, the fused N_Vector microbenchmark (2^26 FP64 vectors:
linear combination of 16, 8 dot products, WRMS norm; GB/s against the
8 TB/s HBM peak), the roofline of the dominant kernel (fused predictor,
factorisation and Newton iterations, timed with HIP events on the library's
stream) and the serial CPU oracle on a bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

HBM_PEAK_GBS = 8000.0
MAXCOR = 3


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def time_advance(b, t_end, steps, torch):
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    t, taken = b.advance(t_end, steps)
    torch.cuda.synchronize()
    return time.perf_counter() - t0, taken, t


def bdf_leg(G, W, torch, prob, dev, warmup, steps, linsol):
    b = G.Bdf.from_problem(prob, device=dev, mode=G.MODE_STREAM, attempts_per_sync=16,
                           linsol=linsol, maxcor=MAXCOR)
    b.advance(prob.t_end, warmup)
    s0 = b.stats()
    dt, taken, t = time_advance(b, prob.t_end, steps, torch)
    s1 = b.stats()
    return b, dt, taken, s0, s1


def fused_ops(G, W, torch, dev, n=1 << 26, warm=10, reps=50):
    """Microbenchmark of the fused operations, mean over `reps` calls
    (the paper's 50-repetition mean of its vector study)."""
    X = [W.torch_uniform_device(n, seed=1000 + j, device=dev) for j in range(16)]
    c = W.uniform_coefficients(16, seed=20242)
    z = torch.empty(n, dtype=torch.float64, device=dev)
    w = W.torch_uniform_device(n, seed=77, device=dev, lo=1e2, hi=1e8)
    out8 = torch.empty(8, dtype=torch.float64, device=dev)
    out1 = torch.empty(1, dtype=torch.float64, device=dev)
    ops = {
        "linear_combination_16": (lambda: G.nvec_linear_combination(c, X, z), 17 * 8 * n),
        "dot_prod_multi_1x8": (lambda: G.nvec_dot_prod_multi(X[0], X[1:9], out=out8), 9 * 8 * n),
        "wrms_norm": (lambda: G.nvec_wrms_norm(X[2], w, out=out1), 2 * 8 * n),
    }
    res = {}
    for name, (fn, nbytes) in ops.items():
        for _ in range(warm):
            fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / reps
        gbs = nbytes / (ms * 1e-3) / 1e9
        res[name] = {"GB_per_s": round(gbs, 1), "frac_of_hbm_peak": round(gbs / HBM_PEAK_GBS, 4),
                     "ms": round(ms, 4), "bytes": nbytes}
    del X, z, w
    torch.cuda.empty_cache()
    return res


def cpu_baseline(W, prob_full, ncells=1024, budget_s=12.0, max_steps=4000):
    """The serial oracle on the first `ncells` cells of the same workload,
    stepped from t = 0 until the time budget is spent."""
    import numpy as np

    import oracle
    n, R = 10, 20
    sub = W.Problem(dict(prob_full))
    sub["cell_topo"] = np.zeros(ncells, np.int32)
    sub["rates"] = np.ascontiguousarray(prob_full.rates[: ncells * R])
    sub["y0"] = np.ascontiguousarray(prob_full.y0[: ncells * n])
    b = oracle.Bdf(sub)
    t0 = time.perf_counter()
    steps = 0
    while steps < max_steps and time.perf_counter() - t0 < budget_s:
        if b.step(sub.t_end) != 0:
            break
        steps += 1
    dt = time.perf_counter() - t0
    return {"value": round(ncells * steps / dt, 1), "unit": "cell-steps/s", "cores": 1,
            "kind": "oracle",
            "sample": f"first {ncells} cells of the same 2^20-cell workload, {steps} steps "
                      f"from t=0 in {dt:.1f} s (serial C, FP64, FP64 LU)"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=400)
    ap.add_argument("--warmup", type=int, default=40)
    ap.add_argument("--cells", type=int, default=1 << 20)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-fused", action="store_true")
    ap.add_argument("--no-fp32", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only: this build has no multi-GPU path "
              f"(--gpus {args.gpus} requested)", file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_2011_12984_amd as G
    import workloads as W

    dev = torch.device("cuda:0")
    G.lib()
    log("generating workload")
    prob = W.random_network_batch(args.cells, n=10, seed=W.BASE_SEED + 3)
    n, R = 10, 20

    log("FP64 LU leg")
    b, dt, taken, s0, s1 = bdf_leg(G, W, torch, prob, dev, args.warmup, args.steps, G.LS_LU64)
    value = args.cells * taken / dt
    ms_per_step = 1e3 * dt / max(taken, 1)
    attempts = s1["nattempts"] - s0["nattempts"]
    niters = s1["nniters"] - s0["nniters"]

    log("profiling the dominant kernel")
    b.set_profiling(True)
    ps0 = b.stats()
    pdt, ptaken, _ = time_advance(b, prob.t_end, min(args.steps, 100), torch)
    ps1 = b.stats()
    kt = b.kernel_times()
    b.set_profiling(False)
    p_ms, p_cnt = kt["newton"]
    p_att = ps1["nattempts"] - ps0["nattempts"]
    q1 = (ps1["hist_reads"] - ps0["hist_reads"]) / max(p_att, 1)   # mean q + 1
    # fused predictor + Newton kernel, per cell: read q+1 history vectors
    # and R rates, write the iterate of each of the maxcor iterations
    bytes_per_launch = 8.0 * args.cells * (q1 * n + R + MAXCOR * n)
    avg_ms = p_ms / max(p_cnt, 1)
    achieved = bytes_per_launch / (avg_ms * 1e-3) / 1e9
    roofline = {"bound": "hbm",
                "kernel": "k_tpc_newton<10,0> (predictor, J, LU, 3 Newton iterations)",
                "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None,
                "avg_launch_ms": round(avg_ms, 4), "launches": p_cnt,
                "algorithmic_bytes_per_launch": int(bytes_per_launch),
                "mean_q_plus_1": round(q1, 3),
                "group_ms": {k: [round(v[0], 3), v[1]] for k, v in kt.items()}}
    t_after = b.stats()["t"]
    b.close()

    out_fp32 = None
    if not args.no_fp32:
        log("FP32 LU + refinement leg")
        b32, dt32, taken32, s320, s321 = bdf_leg(G, W, torch, prob, dev, args.warmup, args.steps,
                                                 G.LS_LU32REF)
        sweeps = s321["refine_sweeps"] - s320["refine_sweeps"]
        fb = s321["refine_fallbacks"] - s320["refine_fallbacks"]
        solves = (s321["nniters"] - s320["nniters"]) * args.cells
        out_fp32 = {"value": round(args.cells * taken32 / dt32, 1), "unit": "cell-steps/s",
                    "ms_per_step": round(1e3 * dt32 / max(taken32, 1), 4),
                    "refine_sweeps_per_block_solve": round(sweeps / max(solves, 1), 4),
                    "fp64_fallback_rate": round(fb / max(solves, 1), 6),
                    "attempts": s321["nattempts"] - s320["nattempts"]}
        b32.close()
        torch.cuda.empty_cache()

    fused = None
    if not args.no_fused:
        log("fused N_Vector microbenchmark")
        fused = fused_ops(G, W, torch, dev)

    cpu = None
    if not args.no_cpu:
        log("CPU oracle baseline")
        cpu = cpu_baseline(W, prob)

    line = {
        "metric": "cell-steps/s batched BDF-Newton + fused N_Vector GB/s; learned/FP32 vs FP64 LU",
        "value": round(value, 1), "unit": "cell-steps/s", "n_gpus": 1, "steps": taken,
        "warmup": args.warmup, "ms_per_step": round(ms_per_step, 4), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic (seeded numpy PCG64)",
        "config": {"workload": "2^20 cells x 10-species random mass-action network (20 reactions, "
                               "rates log-uniform 1e-3..1e8), BDF q<=5 + Newton + FP64 10x10 "
                               "block LU, rtol 1e-6 atol 1e-10, y>=0 projection",
                   "cells": args.cells, "species": n, "reactions": R,
                   "attempts_per_step": round(attempts / max(taken, 1), 4),
                   "newton_iters_per_step": round(niters / max(taken, 1), 4),
                   "t_reached": t_after},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "fp32_refined": out_fp32,
        "fused_ops": fused,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
