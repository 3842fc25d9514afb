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
HERE = os.path.dirname(os.path.abspath(__file__))
# Sources that define the fused Newton kernel the roofline times.
NEWTON_SOURCES = ("paper_2011_12984_amd/csrc/bdf_dev.hpp", "paper_2011_12984_amd/csrc/bdf_jit.hip",
                  "paper_2011_12984_amd/csrc/common.hpp")
# HBM bytes per launch of that kernel at 2^20 cells and order 5, from
# FETCH_SIZE / WRITE_SIZE counter runs scaled by a plain copy kernel (the
# traffic summary under profiles/), with the hash of NEWTON_SOURCES they
# were taken at: reported only while the sources still hash to it.
MEASURED_TRAFFIC = {"sha256_16": "f350373e5de32fdd", "bytes": 1430296658}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def sources_hash(paths):
    import hashlib
    h = hashlib.sha256()
    for p in paths:
        with open(os.path.join(HERE, p), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def host_cpu():
    """Host CPU model and the number of logical CPUs this process may use."""
    model = None
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
    return model, nproc


def time_advance(b, t_end, steps, torch):
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    t, taken = b.advance(t_end, steps)
    torch.cuda.synchronize()
    return time.perf_counter() - t0, taken, t


def bdf_leg(G, W, torch, prob, dev, warmup, steps, linsol, precond=None, jit=True, graph=False,
            defer=True, lazy=False):
    b = G.Bdf.from_problem(prob, device=dev, mode=G.MODE_GRAPH if graph else G.MODE_STREAM,
                           attempts_per_sync=16, linsol=linsol, maxcor=MAXCOR, precond=precond,
                           jit=jit, defer=defer, lazy=lazy)
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
        # a plain copy (nvec_scale by 1: one 16-byte unit per thread,
        # non-temporal): the streaming bandwidth this GPU reaches in practice,
        # for context beside the 8 TB/s peak; the runtime's own device copy
        # beside it
        "copy_reference": (lambda: G.nvec_scale(1.0, X[0], z), 2 * 8 * n),
        "runtime_copy": (lambda: z.copy_(X[0]), 2 * 8 * n),
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
    cp = res["copy_reference"]["GB_per_s"]
    for name in res:
        res[name]["frac_of_copy"] = round(res[name]["GB_per_s"] / cp, 4)
    del X, z, w
    torch.cuda.empty_cache()
    return res


def cpu_baseline(W, prob_full, ncells=1024, budget_s=12.0, max_steps=4000, robertson_reps=3):
    """The serial oracle on the first `ncells` cells of the same workload,
    stepped from t = 0 until the time budget is spent; and the whole
    1,000-cell Robertson BDF2 run to t = 10 (median of `robertson_reps`)."""
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
    model, nproc = host_cpu()
    out = {"value": round(ncells * steps / dt, 1), "unit": "cell-steps/s", "cores": 1,
           "kind": "oracle", "cpu_model": model, "host_logical_cpus": nproc,
           "sample": f"first {ncells} cells of the same 2^20-cell workload, {steps} steps "
                     f"from t=0 in {dt:.1f} s (serial C, FP64, FP64 LU, one thread)"}
    if robertson_reps:
        p = W.robertson_batch(1000)
        times = []
        for _ in range(robertson_reps):
            ob = oracle.Bdf(p)
            t0 = time.perf_counter()
            rc = ob.integrate(p.t_end)
            times.append(time.perf_counter() - t0)
            if rc != 0:
                break
        ws = float(np.median(times))
        st = ob.stats()["nsteps"]
        out["robertson_1000"] = {"whole_run_s": round(ws, 4), "steps": int(st),
                                 "value": round(1000 * st / ws, 1), "unit": "cell-steps/s",
                                 "runs": len(times)}
    return out

def wrms(a, b, rtol, atol):
    import numpy as np
    w = 1.0 / (rtol * np.abs(b) + atol)
    return float(np.sqrt(np.mean(((a - b) * w) ** 2)))


def accuracy_vs_fp64(G, W, torch, dev, make, t_end, **kw):
    """End-state difference (WRMS over all cells, and per cell: median and
    largest) between a run with the given linear solver and the FP64-LU run
    on the same problem to the same t_end; and each run's per-cell error
    against a tight-tolerance FP64 run (rtol and atol 1e-3 of the
    problem's), since two valid step sequences differ by their global
    errors."""
    import numpy as np
    prob = make()
    out = {}
    for name, k in (("fp64", {}), ("solver", kw),
                    ("tight", dict(rtol=prob.rtol * 1e-3, atol=prob.atol * 1e-3))):
        b = G.Bdf.from_problem(prob, device=dev, **k)
        b.integrate(t_end)
        out[name] = (b.y().cpu().numpy(), b.stats())
        b.close()
    yr, sr = out["fp64"]
    y, s = out["solver"]
    yt = out["tight"][0]
    n = prob.sizes[0]

    def per_cell(a, ref):
        return np.sqrt(np.mean((((a - ref) / (prob.rtol * np.abs(ref) + prob.atol)) ** 2)
                               .reshape(-1, n), 1))
    per = per_cell(y, yr)
    es, ef = per_cell(y, yt), per_cell(yr, yt)
    return {"cells": int(prob.ncells), "t_end": t_end,
            "wrms_diff": round(wrms(y, yr, prob.rtol, prob.atol), 6),
            "median_cell_wrms_diff": round(float(np.median(per)), 6),
            "max_cell_wrms_diff": round(float(per.max()), 6),
            "error_vs_tight_per_cell": {"solver": {"median": round(float(np.median(es)), 6),
                                                   "max": round(float(es.max()), 6)},
                                        "fp64_lu": {"median": round(float(np.median(ef)), 6),
                                                    "max": round(float(ef.max()), 6)}},
            "steps": [int(s["nsteps"]), int(sr["nsteps"])]}


def uneven_leg(G, W, torch, dev, warmup, steps, jit=True, linsol=None, lazy=False):
    """Blocks of 4..64 species (2^22 unknowns), FP32 LU + refinement (or
    another linsol, optionally with the lazy Newton matrix),
    hipGraph-captured attempts, launch mode and small-block mapping chosen
    by the library's autotuner."""
    prob = W.uneven_batch(1 << 22)
    t0 = time.perf_counter()
    b = G.Bdf.from_problem(prob, device=dev, mode=G.MODE_GRAPH, attempts_per_sync=16,
                           linsol=G.LS_LU32REF if linsol is None else linsol,
                           launch=G.LAUNCH_AUTO, maxcor=MAXCOR, jit=jit, lazy=lazy)
    torch.cuda.synchronize()
    t_tune = time.perf_counter() - t0
    tu = b.tuning()
    b.advance(prob.t_end, warmup)
    s0 = b.stats()
    dt, taken, t = time_advance(b, prob.t_end, steps, torch)
    s1 = b.stats()
    b.close()
    names = {(0, 0): "per_class_tpc", (0, 1): "per_class_spc16", (1, 0): "one_launch_tpc",
             (1, 1): "one_launch_spc16"}
    # The step's bound: max(algorithmic bytes at 8 TB/s, LU flops at the
    # vector peak of the factorisation's type).  Bytes per cell-step
    # 8 (2 (q+1) n + R) (history read and written once, rates read once, the
    # run's mean q + 1); flops per factorisation n(n-1)/2 + (n-1)n(2n-1)/3,
    # times factorisations (set-ups) per step.
    import numpy as np
    ct = np.asarray(prob.cell_topo)
    n_c = np.array([nu.shape[1] for nu, _ in prob.topologies], np.float64)[ct]
    r_c = np.array([nu.shape[0] for nu, _ in prob.topologies], np.float64)[ct]
    att = max(s1["nattempts"] - s0["nattempts"], 1)
    q1 = (s1["hist_reads"] - s0["hist_reads"]) / att
    step_bytes = 8.0 * float(np.sum(2.0 * q1 * n_c + r_c))
    setups = (s1["nsetups"] - s0["nsetups"]) / max(taken, 1)
    lu_flops = float(np.sum(n_c * (n_c - 1) / 2 + (n_c - 1) * n_c * (2 * n_c - 1) / 3)) * setups
    fp32 = (G.LS_LU32REF if linsol is None else linsol) == G.LS_LU32REF
    t_hbm = step_bytes / (HBM_PEAK_GBS * 1e9) * 1e3
    t_alu = lu_flops / ((157.3e12 if fp32 else 78.6e12)) * 1e3
    ms_step = 1e3 * dt / max(taken, 1)
    roof = {"bound": "hbm" if t_hbm >= t_alu else "alu", "bound_ms_per_step": round(max(t_hbm, t_alu), 4),
            "algorithmic_bytes_per_step": int(step_bytes), "lu_flops_per_step": int(lu_flops),
            "mean_q_plus_1": round(q1, 3), "frac": round(max(t_hbm, t_alu) / ms_step, 4),
            "peaks": "8 TB/s; FP32 157.3 / FP64 78.6 TFLOP/s vector"}
    return {"cells": prob.ncells, "unknowns": prob.N, "value": round(prob.ncells * taken / dt, 1),
            "roofline": roof,
            "unit": "cell-steps/s", "ms_per_step": round(1e3 * dt / max(taken, 1), 4),
            "chosen": names[(tu["launch"], tu["map_small"])],
            "candidates_ms_per_step": {names[k]: round(v, 4) for k, v in tu["ms_per_step"].items()},
            "create_and_tune_s": round(t_tune, 2),
            "attempts_per_step": round((s1["nattempts"] - s0["nattempts"]) / max(taken, 1), 4),
            "setups_per_attempt": round((s1["nsetups"] - s0["nsetups"]) /
                                        max(s1["nattempts"] - s0["nattempts"], 1), 4),
            "newton_iters_per_step": round((s1["nniters"] - s0["nniters"]) / max(taken, 1), 4),
            "refine_sweeps": s1["refine_sweeps"] - s0["refine_sweeps"],
            "refine_fallbacks": s1["refine_fallbacks"] - s0["refine_fallbacks"]}


def uneven_variants(G):
    """The uneven batch with other block solves: FP64 LU and the
    Gauss-Jordan inverse, each factored every attempt and with the lazy
    Newton matrix (factors or inverse stored and reused over steps)."""
    return (("fp64_lu", {"linsol": G.LS_LU64}),
            ("fp64_lu_lazy", {"linsol": G.LS_LU64, "lazy": True}),
            ("gauss_jordan", {"linsol": G.LS_GJ}),
            ("gauss_jordan_lazy", {"linsol": G.LS_GJ, "lazy": True}))


def learned_leg(G, W, torch, dev, cells, warmup, steps, epochs, nblocks):
    """cfg: 2^20 cells x 21 species (one network and rate vector, cells differ
    in their state); MLP trained on `nblocks` blocks captured from the plain
    solver; learned modified Newton vs plain FP64 LU on the same GPU."""
    n = 21
    prob = W.learned_batch(cells, n=n)
    t0 = time.perf_counter()
    plain = G.Bdf.from_problem(prob, device=dev, attempts_per_sync=16)
    X, M = G.capture_training_set(plain, n, nblocks, per_capture=8192, steps_between=8,
                                  t_end=prob.t_end)
    plain.close()
    t_cap = time.perf_counter() - t0
    pc = G.Precond(n, batch_cap=1024)
    pc.set_params(W.mlp_init(n, out_scale=0.02))
    t0 = time.perf_counter()
    hist = G.train_precond(pc, X, M, epochs=epochs, batch=1024, lr=1e-3, seed=20246)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    del X, M
    torch.cuda.empty_cache()
    out = {"cells": cells, "species": n, "training_blocks": int(nblocks), "epochs": epochs,
           "capture_s": round(t_cap, 2), "train_s": round(t_train, 2),
           "val_loss": [round(hist["val0"], 6), round(hist["val"][-1], 6)]}
    for name, kw in (("plain_lu", {}), ("learned", {"linsol": G.LS_LEARNED, "precond": pc}),
                     ("gauss_jordan_lazy", {"linsol": G.LS_GJ, "lazy": True})):
        b, dt, taken, s0, s1 = bdf_leg(G, W, torch, prob, dev, warmup, steps,
                                       kw.get("linsol", G.LS_LU64), precond=kw.get("precond"),
                                       lazy=kw.get("lazy", False))
        d = {k: s1[k] - s0[k] for k in ("nsteps", "nattempts", "nniters", "lp_cell_solves",
                                        "lp_fallback_cells", "lp_step_fallbacks")}
        out[name] = {"value": round(cells * taken / dt, 1), "unit": "cell-steps/s",
                     "ms_per_step": round(1e3 * dt / max(taken, 1), 4),
                     "newton_iters_per_step": round(d["nniters"] / max(taken, 1), 4),
                     "attempts_per_step": round(d["nattempts"] / max(taken, 1), 4)}
        if name == "learned":
            out[name]["cell_fallback_rate"] = round(d["lp_fallback_cells"] / max(d["lp_cell_solves"], 1), 6)
            out[name]["attempt_lu_retries"] = int(d["lp_step_fallbacks"])
        b.close()
    out["accuracy_vs_fp64"] = accuracy_vs_fp64(
        G, W, torch, dev, lambda: W.learned_batch(1 << 14, n=n), 1e-2,
        linsol=G.LS_LEARNED, precond=pc)
    pc.close()
    return out


def robertson_leg(G, W, torch, dev, reps=3):
    """1,000 Robertson-type cells (3 species), BDF2, whole run to t = 10:
    far below the vector length where a GPU pays off, so launch and
    synchronisation latency bound it.  Median of `reps` whole runs, each on
    a fresh handle with its inputs already in HBM (creation not timed)."""
    import numpy as np
    p = W.robertson_batch(1000)
    out = {}
    for name, kw in (("stream", {"mode": G.MODE_STREAM}), ("graph", {"mode": G.MODE_GRAPH})):
        times, steps = [], None
        for _ in range(reps):
            b = G.Bdf.from_problem(p, device=dev, attempts_per_sync=16, jit=True, **kw)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            t = b.integrate(p.t_end)
            torch.cuda.synchronize()
            times.append(time.perf_counter() - t0)
            steps = b.stats()["nsteps"]
            b.close()
            assert t == p.t_end
        ws = float(np.median(times))
        out[name] = {"whole_run_s": round(ws, 4), "steps": int(steps),
                     "value": round(1000 * steps / ws, 1), "unit": "cell-steps/s"}
    return out


def krylov_leg(G, W, torch, prob, dev, warmup, steps):
    """The benchmark workload with Newton-Krylov (GMRES over all cells,
    block-Jacobi preconditioner from the batched LU): a fresh preconditioner
    every attempt (one Krylov iteration per solve) and the lazy one (reused
    over steps, several Krylov iterations).  The host drives the Krylov
    iteration with one synchronising reduction per inner-product pass."""
    out = {}
    for name, kw in (("gmres_fresh_preconditioner", dict()),
                     ("gmres_lazy_preconditioner", dict(lazy=True))):
        b = G.Bdf.from_problem(prob, device=dev, mode=G.MODE_STREAM, linsol=G.LS_GMRES,
                               maxcor=MAXCOR, **kw)
        b.advance(prob.t_end, warmup)
        s0 = b.stats()
        dt, taken, _ = time_advance(b, prob.t_end, steps, torch)
        s1 = b.stats()
        b.close()
        nit = s1["nniters"] - s0["nniters"]
        out[name] = {"value": round(prob.ncells * taken / dt, 1), "unit": "cell-steps/s",
                     "ms_per_step": round(1e3 * dt / max(taken, 1), 4),
                     "newton_iters_per_step": round(nit / max(taken, 1), 4),
                     "krylov_iters_per_newton_iter":
                         round((s1["nliters"] - s0["nliters"]) / max(nit, 1), 4),
                     "setups_per_attempt": round((s1["nsetups"] - s0["nsetups"]) /
                                                 max(s1["nattempts"] - s0["nattempts"], 1), 4)}
    return out


def brusselator_leg(G, W, torch, dev, ncells=1 << 20):
    """The demonstration reaction of Section 7 (3 species per cell, the
    1-D Gaussian profile over ncells cells), whole run from t = 0 to 10 on a
    fresh handle (creation not timed): grouped stepping with the FP64 LU or
    the explicit Gauss-Jordan block inverse, and per-cell stepping with the
    inverse.  value = accepted cell-steps / wall time."""
    p = W.brusselator_batch(ncells)
    out = {"cells": ncells, "species": 3, "t_end": p.t_end}
    for name, kw in (("grouped_lu", dict(linsol=G.LS_LU64, jit=True, attempts_per_sync=16)),
                     ("grouped_gauss_jordan", dict(linsol=G.LS_GJ, jit=True,
                                                   attempts_per_sync=16)),
                     ("per_cell_gauss_jordan", dict(linsol=G.LS_GJ, per_cell=True))):
        b = G.Bdf.from_problem(p, device=dev, **kw)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        t = b.integrate(p.t_end)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        s = b.stats()
        b.close()
        cell_steps = s["nsteps"] if kw.get("per_cell") else s["nsteps"] * ncells
        out[name] = {"whole_run_s": round(dt, 4), "reached": t == p.t_end,
                     "steps": int(s["nsteps"]) if not kw.get("per_cell") else None,
                     "cell_steps": int(cell_steps), "value": round(cell_steps / dt, 1),
                     "unit": "cell-steps/s",
                     "attempts_per_step": round(s["nattempts"] / max(s["nsteps"], 1), 4)}
    return out


def per_cell_leg(G, W, torch, prob, dev, max_steps=2000000):
    """The benchmark workload with per-cell adaptive stepping (every cell its
    own step size and order), integrated from t = 0 to t_end = 10 on a fresh
    handle; creation not timed.  value = total accepted cell-steps / wall
    time; the per-cell step distribution shows what bounds the wall time."""
    import numpy as np
    b = G.Bdf.from_problem(prob, device=dev, per_cell=True, max_steps=max_steps)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    try:
        t = b.integrate(prob.t_end)
        err = None
    except G.BdfGpuError as e:
        t, err = None, str(e)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    counts, tc = b.cell_stats()
    s = b.stats()
    b.close()
    st = counts[:, 0]
    return {"t_end": prob.t_end, "reached_all": t == prob.t_end, "error": err,
            "wall_s": round(dt, 3), "cell_steps": int(s["nsteps"]),
            "value": round(s["nsteps"] / dt, 1), "unit": "cell-steps/s",
            "attempts_per_step": round(s["nattempts"] / max(s["nsteps"], 1), 4),
            "per_cell_steps": {"min": int(st.min()), "median": float(np.median(st)),
                               "p99": float(np.quantile(st, 0.99)), "max": int(st.max())},
            "cells_over_10k_steps": int((st > 10000).sum())}


def long_run_leg(G, W, torch, prob, dev, jit=True, max_steps=20000, **kw):
    """The benchmark workload integrated from t = 0 for max_steps accepted
    steps (or to t_end) on a fresh handle, creation and the starting step
    not timed: the step mix of a long run (orders, retries, Newton
    iterations) beside the short timed window of the headline.  kw: extra
    handle options (variable coefficients, lazy Newton matrix)."""
    b = G.Bdf.from_problem(prob, device=dev, mode=G.MODE_STREAM, attempts_per_sync=16,
                           linsol=G.LS_LU64, maxcor=MAXCOR, jit=jit, **kw)
    b.advance(prob.t_end, 1)
    s0 = b.stats()
    dt, taken, t = time_advance(b, prob.t_end, max_steps, torch)
    s1 = b.stats()
    b.close()
    return {"t_end": prob.t_end, "t_reached": t, "steps": taken + 1, "timed_steps": taken,
            "wall_s": round(dt, 3), "value": round(prob.ncells * taken / dt, 1),
            "unit": "cell-steps/s", "ms_per_step": round(1e3 * dt / max(taken, 1), 4),
            "attempts_per_step": round((s1["nattempts"] - s0["nattempts"]) / max(taken, 1), 4),
            "newton_iters_per_step": round((s1["nniters"] - s0["nniters"]) / max(taken, 1), 4),
            "setups_per_attempt": round((s1["nsetups"] - s0["nsetups"]) /
                                        max(s1["nattempts"] - s0["nattempts"], 1), 4),
            "order_hist": [a - b_ for a, b_ in zip(s1["order_hist"], s0["order_hist"])]}


def vc_lazy_leg(G, W, torch, prob, dev, warmup, steps, long_steps, jit=True):
    """The benchmark workload with variable coefficients, the lazy Newton
    matrix, and both: the headline's window (warmup, then `steps` timed
    steps) and, for both together, the long run from t = 0."""
    out = {}
    for name, kw in (("vc", dict(vc=True)), ("lazy", dict(lazy=True)),
                     ("vc_lazy", dict(vc=True, lazy=True))):
        b = G.Bdf.from_problem(prob, device=dev, mode=G.MODE_STREAM, attempts_per_sync=16,
                               linsol=G.LS_LU64, maxcor=MAXCOR, jit=jit, **kw)
        b.advance(prob.t_end, warmup)
        s0 = b.stats()
        dt, taken, _ = time_advance(b, prob.t_end, steps, torch)
        s1 = b.stats()
        b.close()
        att = s1["nattempts"] - s0["nattempts"]
        out[name] = {"value": round(prob.ncells * taken / dt, 1), "unit": "cell-steps/s",
                     "ms_per_step": round(1e3 * dt / max(taken, 1), 4),
                     "attempts_per_step": round(att / max(taken, 1), 4),
                     "newton_iters_per_step": round((s1["nniters"] - s0["nniters"]) /
                                                    max(taken, 1), 4),
                     "setups_per_attempt": round((s1["nsetups"] - s0["nsetups"]) / max(att, 1), 4),
                     "stale_retries": s1["nstale_retries"] - s0["nstale_retries"]}
    if long_steps > 0:
        out["vc_lazy_long_run"] = long_run_leg(G, W, torch, prob, dev, jit=jit,
                                               max_steps=long_steps, vc=True, lazy=True)
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=400)
    ap.add_argument("--warmup", type=int, default=40)
    ap.add_argument("--cells", type=int, default=1 << 20)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-fused", action="store_true")
    ap.add_argument("--no-fp32", action="store_true")
    ap.add_argument("--no-learned", action="store_true")
    ap.add_argument("--no-uneven", action="store_true")
    ap.add_argument("--no-robertson", action="store_true")
    ap.add_argument("--no-krylov", action="store_true",
                    help="skip the Newton-Krylov (GMRES) legs")
    ap.add_argument("--no-vc-lazy", action="store_true",
                    help="skip the variable-coefficient / lazy Newton matrix legs")
    ap.add_argument("--no-brusselator", action="store_true",
                    help="skip the demonstration reaction's whole runs")
    ap.add_argument("--no-per-cell", action="store_true",
                    help="skip the per-cell adaptive stepping run to t = 10")
    ap.add_argument("--long-steps", type=int, default=20000,
                    help="accepted steps of the long run from t = 0 (0 skips it)")
    ap.add_argument("--profile-warmup", type=int, default=60,
                    help="steps before the kernel-timing window (order 5 is reached by then)")
    ap.add_argument("--graph", action="store_true")
    ap.add_argument("--no-defer", action="store_true",
                    help="separate history-update kernel instead of the deferred update")
    ap.add_argument("--no-jit", action="store_true",
                    help="generic table-driven Newton kernels instead of network-specialised ones")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run nvec_scale (a plain copy, 512 MiB in and out) 5 times: "
                         "the reference for HBM byte counters")
    ap.add_argument("--profile-uneven", type=int, default=0, metavar="STEPS",
                    help="only advance the uneven batch (per-class launches, FP32-refined LU, "
                         "stream mode) STEPS steps: the workload of the segment-kernel profiles")
    ap.add_argument("--profile-lazy", action="store_true",
                    help="with --profile-uneven: the lazy Newton matrix (FP64 LU, or the "
                         "Gauss-Jordan inverse with --profile-gj)")
    ap.add_argument("--profile-gj", action="store_true",
                    help="with --profile-uneven: the Gauss-Jordan inverse")
    ap.add_argument("--only-uneven", action="store_true",
                    help="only run the uneven-batch legs (FP32-refined, FP64, FP64 lazy) and "
                         "print their results")
    ap.add_argument("--profile-mlp", action="store_true",
                    help="only run the learned preconditioner's MFMA forward pass on 2^20 random "
                         "inputs (2 warm-up + 5 timed calls): the workload of the MLP profiles")
    ap.add_argument("--learned-epochs", type=int, default=30)
    ap.add_argument("--learned-blocks", type=int, default=1 << 18)
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
    if args.copy_calibration:
        x = W.torch_uniform_device(1 << 26, seed=5, device=dev)
        z = torch.empty_like(x)
        for _ in range(5):
            G.nvec_scale(1.0, x, z)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calibration": {"kernel": "k_scale2", "bytes_read": 8 << 26,
                                               "bytes_written": 8 << 26, "launches": 5}}))
        return
    if args.profile_uneven > 0:
        p = W.uneven_batch(1 << 22)
        b = G.Bdf.from_problem(p, device=dev, mode=G.MODE_STREAM, attempts_per_sync=1,
                               linsol=(G.LS_GJ if args.profile_gj else
                                       G.LS_LU64 if args.profile_lazy else G.LS_LU32REF),
                               lazy=args.profile_lazy, launch=G.LAUNCH_PER_CLASS, maxcor=MAXCOR,
                               jit=True)
        b.advance(p.t_end, args.profile_uneven)
        torch.cuda.synchronize()
        s = b.stats()
        print(json.dumps({"profile_uneven": {"steps": s["nsteps"], "attempts": s["nattempts"],
                                             "setups": s["nsetups"]}}))
        return
    if args.only_uneven:
        out = uneven_leg(G, W, torch, dev, args.warmup, min(args.steps, 200), jit=not args.no_jit)
        for name, kw in uneven_variants(G):
            out[name] = uneven_leg(G, W, torch, dev, args.warmup, min(args.steps, 200),
                                   jit=not args.no_jit, **kw)
        print(json.dumps({"uneven": out}))
        return
    if args.profile_mlp:
        n, B = 21, 1 << 20
        pc = G.Precond(n, batch_cap=1024)
        pc.set_params(W.mlp_init(n, out_scale=0.02))
        X = W.torch_uniform_device(B * (n + 1), seed=7, device=dev).view(B, n + 1)
        pc.fit_normalization(X)
        for _ in range(2):
            pc.forward(X)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(5):
            pc.forward(X)
        torch.cuda.synchronize()
        ms = 1e3 * (time.perf_counter() - t0) / 5
        flops = 2.0 * B * ((n + 1) * 256 + 256 * 256 + 256 * n * n)
        print(json.dumps({"profile_mlp": {"samples": B, "ms": round(ms, 4),
                                          "TFLOP_per_s": round(flops / ms / 1e9, 1)}}))
        return
    log("generating workload")
    prob = W.random_network_batch(args.cells, n=10, seed=W.BASE_SEED + 3)
    n, R = 10, 20

    log("FP64 LU leg")
    b, dt, taken, s0, s1 = bdf_leg(G, W, torch, prob, dev, args.warmup, args.steps, G.LS_LU64,
                                   jit=not args.no_jit, graph=args.graph, defer=not args.no_defer)
    value = args.cells * taken / dt
    ms_per_step = 1e3 * dt / max(taken, 1)
    attempts = s1["nattempts"] - s0["nattempts"]
    niters = s1["nniters"] - s0["nniters"]

    t_after = b.stats()["t"]
    hist_reads = s1["hist_reads"] - s0["hist_reads"]
    b.close()

    log("profiling the dominant kernel")
    # A stream-mode handle of the same workload that reads the controller
    # after every attempt, so that every timed launch does work (with several
    # attempts per status read, launches enqueued after the step limit return
    # at once); advanced past the order ramp before the timing window.
    pb = G.Bdf.from_problem(prob, device=dev, mode=G.MODE_STREAM, attempts_per_sync=1,
                            linsol=G.LS_LU64, maxcor=MAXCOR, jit=not args.no_jit,
                            defer=not args.no_defer)
    pb.advance(prob.t_end, args.profile_warmup)
    pb.set_profiling(True)
    ps0 = pb.stats()
    pdt, ptaken, _ = time_advance(pb, prob.t_end, min(args.steps, 100), torch)
    ps1 = pb.stats()
    kt = pb.kernel_times()
    pb.set_profiling(False)
    pb.close()
    p_ms, p_cnt = kt["newton"]
    p_att = ps1["nattempts"] - ps0["nattempts"]
    # a launch runs two Newton iterations; an attempt the replay of those
    # leaves undecided takes a continuation launch
    p_cont = ps1["ncont"] - ps0["ncont"]
    if p_cnt != p_att + p_cont:
        raise RuntimeError(f"timed {p_cnt} Newton launches for {p_att} attempts and "
                           f"{p_cont} continuations")
    q1 = (ps1["hist_reads"] - ps0["hist_reads"]) / max(p_att, 1)   # mean q + 1
    # The step's algorithmic bytes per cell are 8 (2 (q+1) n + R): the
    # history read and written once and the rates read once.  With the
    # deferred update the Newton kernel does all of it (the history write of
    # an accepted step happens in the next attempt's kernel): per launch,
    # the step bytes times accepted steps per launch.  With a separate
    # history update the Newton kernel's share is the read half,
    # 8 ((q+1) n + R), and the update's the write half.
    deferred = kt["accept"][1] == 0
    if deferred:
        bytes_per_launch = 8.0 * args.cells * (2 * q1 * n + R) * ptaken / max(p_cnt, 1)
        alg = "8 * cells * (2 (q+1) n + R) per accepted step (history read and written, rates " \
              "read), times accepted steps per launch"
    else:
        bytes_per_launch = 8.0 * args.cells * (q1 * n + R)
        alg = "8 * cells * ((q+1) * n + R): history read + rates"
    avg_ms = p_ms / max(p_cnt, 1)
    achieved = bytes_per_launch / (avg_ms * 1e-3) / 1e9
    sha = sources_hash(NEWTON_SOURCES)
    traffic = (MEASURED_TRAFFIC["bytes"]
               if (sha == MEASURED_TRAFFIC["sha256_16"] and args.cells == 1 << 20
                   and not args.no_jit) else None)
    # whole step against the step's algorithmic bytes, over the headline run
    q1_main = hist_reads / max(attempts, 1)
    step_bytes = 8.0 * args.cells * (2 * q1_main * n + R)
    step_gbs = step_bytes / (ms_per_step * 1e-3) / 1e9
    roofline = {"bound": "hbm",
                "kernel": ("k_tpc_newton<10,0>" if args.no_jit else
                           "bdf_newton_net_np10_ls0 (k_tpc_newton<10,0> specialised to the network)")
                          + (" (history update of the previous step, predictor, J, LU, 3 Newton "
                             "iterations)" if deferred else " (predictor, J, LU, 3 Newton iterations)"),
                "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4),
                "traffic": traffic, "newton_sources_sha256_16": sha,
                "avg_launch_ms": round(avg_ms, 4), "launches": p_cnt, "attempts": p_att,
                "continuations": p_cont,
                "algorithmic_bytes_per_launch": int(bytes_per_launch),
                "algorithmic_bytes": alg, "deferred_history_update": deferred,
                "mean_q_plus_1": round(q1, 3),
                "group_ms": {k: [round(v[0], 3), v[1]] for k, v in kt.items()},
                "step": {"algorithmic_bytes_per_step": int(step_bytes),
                         "algorithmic_bytes": "8 * cells * (2 (q+1) n + R)",
                         "mean_q_plus_1": round(q1_main, 3),
                         "achieved": round(step_gbs, 1),
                         "frac": round(step_gbs / HBM_PEAK_GBS, 4)}}

    out_fp32 = None
    if not args.no_fp32:
        log("FP32 LU + refinement leg")
        b32, dt32, taken32, s320, s321 = bdf_leg(G, W, torch, prob, dev, args.warmup, args.steps,
                                                 G.LS_LU32REF, jit=not args.no_jit)
        sweeps = s321["refine_sweeps"] - s320["refine_sweeps"]
        fb = s321["refine_fallbacks"] - s320["refine_fallbacks"]
        solves = (s321["nniters"] - s320["nniters"]) * args.cells
        out_fp32 = {"value": round(args.cells * taken32 / dt32, 1), "unit": "cell-steps/s",
                    "ms_per_step": round(1e3 * dt32 / max(taken32, 1), 4),
                    "refine_sweeps_per_block_solve": round(sweeps / max(solves, 1), 4),
                    "fp64_fallback_rate": round(fb / max(solves, 1), 6),
                    "attempts": s321["nattempts"] - s320["nattempts"]}
        b32.close()
        out_fp32["accuracy_vs_fp64"] = accuracy_vs_fp64(
            G, W, torch, dev, lambda: W.random_network_batch(1 << 16, n=10, seed=W.BASE_SEED + 3),
            1e-3, linsol=G.LS_LU32REF)
        torch.cuda.empty_cache()

    long_run = None
    if args.long_steps > 0:
        log(f"long run: {args.long_steps} steps from t = 0")
        long_run = long_run_leg(G, W, torch, prob, dev, jit=not args.no_jit,
                                max_steps=args.long_steps)

    vc_lazy = None
    if not args.no_vc_lazy:
        log("variable coefficients and lazy Newton matrix")
        vc_lazy = vc_lazy_leg(G, W, torch, prob, dev, args.warmup, args.steps, args.long_steps,
                              jit=not args.no_jit)

    krylov = None
    if not args.no_krylov:
        log("Newton-Krylov (GMRES, block-Jacobi preconditioner)")
        krylov = krylov_leg(G, W, torch, prob, dev, args.warmup, min(args.steps, 100))

    per_cell = None
    if not args.no_per_cell:
        log("per-cell adaptive stepping, whole run to t = 10")
        per_cell = per_cell_leg(G, W, torch, prob, dev)

    robertson = None
    if not args.no_robertson:
        log("1,000-cell Robertson BDF2 whole runs")
        robertson = robertson_leg(G, W, torch, dev)

    brusselator = None
    if not args.no_brusselator:
        log("demonstration reaction (3 species, order-3 reaction), whole runs to t = 10")
        brusselator = brusselator_leg(G, W, torch, dev)

    fused = None
    if not args.no_fused:
        log("fused N_Vector microbenchmark")
        fused = fused_ops(G, W, torch, dev)

    uneven = None
    if not args.no_uneven:
        log("uneven batch leg (autotuned launch, hipGraph, FP32-refined LU)")
        uneven = uneven_leg(G, W, torch, dev, args.warmup, min(args.steps, 200), jit=not args.no_jit)
        for name, kw in uneven_variants(G):
            uneven[name] = uneven_leg(G, W, torch, dev, args.warmup, min(args.steps, 200),
                                      jit=not args.no_jit, **kw)

    learned = None
    if not args.no_learned:
        log("learned preconditioner leg (capture, training, learned vs plain LU)")
        learned = learned_leg(G, W, torch, dev, args.cells, args.warmup, min(args.steps, 200),
                              args.learned_epochs, args.learned_blocks)

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
                   "network_specialised_kernels": not args.no_jit,
                   "t_reached": t_after},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "long_run": long_run,
        "variable_coefficients_lazy": vc_lazy,
        "newton_krylov": krylov,
        "per_cell_whole_run": per_cell,
        "robertson_1000_bdf2": robertson,
        "brusselator_2p20": brusselator,
        "fp32_refined": out_fp32,
        "fused_ops": fused,
        "uneven": uneven,
        "learned": learned,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
