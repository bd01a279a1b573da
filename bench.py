"""Benchmark: surrogate-stencil operator apply on the 288-macro shell, level 7.

One step = one full application y = L~ x of the two-scale operator (Sec. 3.4
eq. ts): surrogate volume rows of all 288 macros plus the element-wise rows of
the lower primitives, on the shell r in [0.55, 1] refined to N = 128 intervals
per macro edge (100,270,590 unknowns, FP64).  Inputs are seeded, synthetic
and resident in HBM before timing starts.

Printed JSON line (one): metric / value (GDoF/s of the whole operator), the
roofline of the dominant kernel (surrogate volume kernel, HBM-bound: 16
algorithmic bytes per interior node, x read once and y written once), the
IFEM apply on the same GPU, the q = 4 surrogate, a Gauss-Seidel sweep, and
the CPU oracle timed on a bounded sample of the same rows.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu]
       [--level 7] [--mesh shell288] [--only-volume]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def time_events(fn, reps, stream):
    """Average duration (ms) of fn() with HIP events on `stream`."""
    import torch
    start = torch.cuda.Event(enable_timing=True)
    stop = torch.cuda.Event(enable_timing=True)
    start.record(stream)
    for _ in range(reps):
        fn()
    stop.record(stream)
    stop.synchronize()
    return start.elapsed_time(stop) / reps


def cpu_baseline(vtx, tet, lam, q, coeffs, x_canon, n_free_total, budget_s=12.0):
    """The oracle's surrogate operator on a random sample of the workload's
    rows (all unique free nodes equally likely), scaled to GDoF/s."""
    import numpy as np

    import oracle
    O = oracle.Mesh(vtx, tet)
    N = 2 ** lam
    mask = O.dirichlet_mask(N)
    free = np.flatnonzero(~mask)
    rng = np.random.default_rng(123)
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    n = 20000
    sample = free[np.unique(rng.integers(0, len(free), size=n))]
    t0 = time.perf_counter()
    O.apply_rows(N, x_canon, sample, kind=oracle.LSQP, q=q, coeffs=coeffs)
    dt = time.perf_counter() - t0
    n2 = int(min(len(free), max(n, n * budget_s / max(dt, 1e-6))))
    sample = free[np.unique(rng.integers(0, len(free), size=n2))]
    n2 = len(sample)
    t0 = time.perf_counter()
    O.apply_rows(N, x_canon, sample, kind=oracle.LSQP, q=q, coeffs=coeffs)
    dt = time.perf_counter() - t0
    return {"value": round(n2 / dt / 1e9, 6), "unit": "GDoF/s", "cores": threads,
            "kind": "oracle",
            "sample": "%d of %d free rows (uniform random, seed 123) of the same operator and "
                      "input, oracle surrogate rows (Horner-free direct polynomial evaluation) "
                      "and element-wise lower-primitive rows; %.1f s wall" % (n2, n_free_total, dt)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--level", type=int, default=7)
    ap.add_argument("--mesh", default="shell288", choices=["shell288", "shell36", "single"])
    ap.add_argument("--q", type=int, default=2)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--only-volume", action="store_true",
                    help="time only the surrogate volume kernel (profiling runs)")
    ap.add_argument("--copy-calib", action="store_true",
                    help="run a plain 1 GiB device copy (counter calibration) and exit")
    args = ap.parse_args()

    if args.gpus != 1:
        print("bench.py runs on one GPU only (this build has no multi-GPU path); "
              "got --gpus %d" % args.gpus, file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_1608_06473_amd as ts
    from paper_1608_06473_amd import inputs

    torch.cuda.set_device(0)
    stream = torch.cuda.current_stream()

    if args.copy_calib:
        a = torch.ones(2 ** 27, dtype=torch.float64, device="cuda")  # 1 GiB
        b = torch.empty_like(a)
        for _ in range(5):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_each_way": a.numel() * 8, "copies": 5}))
        return

    lam, q = args.level, args.q
    vtx, tet = {"shell288": inputs.shell288, "shell36": inputs.shell36,
                "single": inputs.single_macro}[args.mesh]()
    G = ts.Mesh(vtx, tet)
    info = G.layout(lam)
    log("mesh %s level %d: %d macros, %d free dof, %d volume dof, block vector %d"
        % (args.mesh, lam, info.n_macros, info.n_free, info.n_volume, info.vec_len))
    t0 = time.perf_counter()
    op = ts.Operator(G, lam, method=ts.TS_LSQP, q=q, sample_j=2)
    torch.cuda.synchronize()
    t_setup = time.perf_counter() - t0
    log("setup (sampling + normal equations, levels 3..%d): %.3f s" % (lam, t_setup))

    x_canon = inputs.uniform(info.n_unique, 0)
    xb = G.to_block(lam, x_canon)
    yb = G.zeros(lam)

    def step():
        ts.ts_apply(op.h, lam, ts.TS_F64, xb, yb, stream)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    ms = dt / args.steps * 1e3
    value = info.n_free * args.steps / dt / 1e9
    log("full apply: %.3f ms/step, %.1f GDoF/s" % (ms, value))

    # dominant kernel: the surrogate volume kernel, HIP events on its stream
    reps = max(5, args.steps)
    vol_ms = time_events(lambda: ts.ts_apply_volume(op.h, lam, ts.TS_F64, xb, yb, stream),
                         reps, stream)
    alg_bytes = 16.0 * info.n_volume
    achieved = alg_bytes / (vol_ms / 1e3) / 1e9
    log("volume kernel: %.3f ms, %.1f GB/s algorithmic (%.1f GDoF/s)"
        % (vol_ms, achieved, info.n_volume / vol_ms / 1e6))
    if args.only_volume:
        return

    extra = {}
    # IFEM apply (comparison path)
    opI = ts.Operator(G, lam, method=ts.TS_IFEM)
    ts.ts_apply(opI.h, lam, ts.TS_F64, xb, yb, stream)
    ifem_ms = time_events(lambda: ts.ts_apply(opI.h, lam, ts.TS_F64, xb, yb, stream), 3, stream)
    extra["ifem_apply"] = {"ms": round(ifem_ms, 4),
                           "gdofs": round(info.n_free / ifem_ms / 1e6, 3),
                           "surrogate_speedup": round(ifem_ms / ms, 2)}
    log("IFEM apply: %.3f ms (%.2f GDoF/s)" % (ifem_ms, info.n_free / ifem_ms / 1e6))
    del opI
    # q = 4 surrogate
    op4 = ts.Operator(G, lam, method=ts.TS_LSQP, q=4, sample_j=2)
    ts.ts_apply(op4.h, lam, ts.TS_F64, xb, yb, stream)
    q4_ms = time_events(lambda: ts.ts_apply(op4.h, lam, ts.TS_F64, xb, yb, stream), reps, stream)
    q4_vol = time_events(lambda: ts.ts_apply_volume(op4.h, lam, ts.TS_F64, xb, yb, stream),
                         reps, stream)
    extra["q4_apply"] = {"ms": round(q4_ms, 4), "gdofs": round(info.n_free / q4_ms / 1e6, 3),
                         "volume_ms": round(q4_vol, 4),
                         "volume_gbs": round(alg_bytes / (q4_vol / 1e3) / 1e9, 1)}
    log("q=4 apply: %.3f ms (volume %.3f ms)" % (q4_ms, q4_vol))
    del op4
    # FP32 apply and one Gauss-Seidel sweep (FP64)
    x32 = xb.float()
    y32 = torch.zeros_like(x32)
    ts.ts_apply(op.h, lam, ts.TS_F32, x32, y32, stream)
    f32_ms = time_events(lambda: ts.ts_apply(op.h, lam, ts.TS_F32, x32, y32, stream), reps, stream)
    extra["fp32_apply"] = {"ms": round(f32_ms, 4), "gdofs": round(info.n_free / f32_ms / 1e6, 3)}
    del x32, y32
    fb = G.rhs(lam, ts.TS_RHS_MANUFACTURED, [0.55, 1.0])
    ub = torch.zeros_like(fb)
    gs_ms = time_events(lambda: ts.ts_smooth(op.h, lam, ts.TS_F64, fb, ub, 1, stream), 3, stream)
    extra["gs_sweep"] = {"ms": round(gs_ms, 4), "gdofs": round(info.n_free / gs_ms / 1e6, 3)}
    log("FP32 apply %.3f ms; GS sweep %.3f ms" % (f32_ms, gs_ms))

    cpu = None
    if not args.no_cpu:
        log("cpu baseline (oracle on host cores)...")
        cpu = cpu_baseline(vtx, tet, lam, q, op.coeffs(lam), x_canon, info.n_free)
        log("cpu baseline: %s" % cpu)

    line = {
        "metric": "GDoF/s surrogate stencil apply (FP64, whole operator)",
        "value": round(value, 3),
        "unit": "GDoF/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic: x ~ U[-1,1] (PCG64 seed 0) on the cubed-sphere shell",
        "config": {"workload": "%s level %d (N=%d) LSQP q=%d j=2 surrogate apply, FP64"
                               % (args.mesh, lam, 2 ** lam, q),
                   "macros": int(info.n_macros), "free_dof": int(info.n_free),
                   "volume_dof": int(info.n_volume), "setup_s": round(t_setup, 3)},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": None, "kernel": "k_surrogate<2,double,double,0,0>",
                     "kernel_ms": round(vol_ms, 4),
                     "algorithmic_bytes": int(alg_bytes)},
        "cpu_baseline": cpu,
    }
    line.update(extra)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
