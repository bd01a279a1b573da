"""Benchmark: surrogate-stencil operator apply on the 288-macro shell, level 7.

One step = one full application y = L~ x of the two-scale operator (Sec. 3.4
eq. ts): surrogate volume rows of all 288 macros plus the element-wise rows of
the lower primitives, on the shell r in [0.55, 1] refined to N = 128 intervals
per macro edge (100,270,590 unknowns, FP64).  Inputs are seeded, synthetic
and resident in HBM before timing starts.

Printed JSON line (one): metric / value (GDoF/s of the whole operator), the
roofline of the step's dominant kernel (the surrogate volume kernel launched
with the interior-face rows fused in, HBM-bound: 16 algorithmic bytes per
row, x read once and y written once; traffic from the committed rocprofv3
counter record of the same kernel source) and of its volume rows alone, the
IFEM apply on the same GPU, q = 4, FP32 and FP16-weight applies, the residual,
Gauss-Seidel sweeps, V(3,3) solves to 1e-10 in FP64 and with FP32 / FP16-weight
cycles under FP64 refinement, the single-macro latency and the 36-macro
shell's apply, sweep and solves, a bounded run of the serve loop, and the CPU
oracle timed on the free rows of the same operator.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu]
       [--level 7] [--mesh shell288] [--only-volume] [--only-gs] [--no-solve] [--no-serve]
       [--no-small] [--serve-requests 30] [--serve-sustained 60]
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
FP64_PEAK_TFS = 78.6   # MI355X FP64 vector
# the paper's count for one IFEM update: 24 element matrices, edge sums and
# the central weight (1,353 FLOP) plus the 29 FLOP of the application
IFEM_FLOP_PER_NODE = 1353 + 29


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


# the kernel and what fixes its access pattern (tiles, face-row copy order)
KERNEL_SOURCES = ["paper_1608_06473_amd/csrc/ts_surrogate.h",
                  "paper_1608_06473_amd/csrc/ts_face.h",
                  "paper_1608_06473_amd/csrc/k_surr_inst.hip",
                  "paper_1608_06473_amd/csrc/ts_topology.cpp"]
PMC_RECORD = "profiles/pmc_k_surr_lds_q2_shell288_l7.md"


def kernel_source_hash():
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def pmc_traffic(key="record"):
    """HBM bytes per launch from the committed counter summary (its `record:`
    line for the volume-only launch, `record_whole:` for the whole-operator
    launch: FETCH_SIZE and WRITE_SIZE in KiB per dispatch, scaled by the
    factors measured on a plain device copy), or None when the summary is
    missing or was taken on another version of the kernel source."""
    path = os.path.join(ROOT, PMC_RECORD)
    if not os.path.exists(path):
        return None
    rec = None
    tag = key + ": "
    with open(path) as fh:
        for ln in fh:
            if ln.startswith(tag):
                rec = json.loads(ln[len(tag):])
    if rec is None:
        return None
    if rec.get("kernel_source_hash") != kernel_source_hash():
        return None
    return int((rec["fetch_kib"] * rec["fetch_scale"] + rec["write_kib"] * rec["write_scale"])
               * 1024)


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for ln in fh:
                if ln.startswith("model name"):
                    return ln.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _omp_set_threads(n):
    """Thread count of the oracle's OpenMP regions (libgomp's ICV of this
    thread), or None if libgomp cannot be reached."""
    import ctypes
    try:
        gomp = ctypes.CDLL("libgomp.so.1")
    except OSError:
        return None
    gomp.omp_get_max_threads.restype = ctypes.c_int
    old = gomp.omp_get_max_threads()
    gomp.omp_set_num_threads(int(n))
    return old


def cpu_baseline(vtx, tet, lam, q, x_canon, n_free_total, solutions=None, log=print):
    """The CPU leg: the oracle (test infrastructure, plain C built here with
    -O3 -march=native for this host) timed on the same operator and input, and
    the oracle's measurement of the GPU solutions' residuals.

    Timing mirrors the paper's "minimum of several runs": one warm-up pass,
    then the best of 3 passes over all free rows on all host cores, and the
    best of 2 passes over every 64th free row on one core.  solutions: name ->
    (f, u, coefficients) canonical host arrays of GPU solves; the oracle
    evaluates ||f - L~u||_2 / ||f||_2 over the free rows with the same
    coefficients, row by row and independently of the GPU."""
    import numpy as np

    os.environ["TS_ORACLE_NATIVE"] = "1"
    import oracle
    O = oracle.Mesh(vtx, tet)
    N = 2 ** lam
    coeffs = O.fit(N, oracle.LSQP, q, 2)
    free = np.flatnonzero(~O.dirichlet_mask(N))
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))

    def best(rows, passes):
        O.apply_rows(N, x_canon, rows, kind=oracle.LSQP, q=q, coeffs=coeffs)  # warm-up
        b = float("inf")
        for _ in range(passes):
            t0 = time.perf_counter()
            O.apply_rows(N, x_canon, rows, kind=oracle.LSQP, q=q, coeffs=coeffs)
            b = min(b, time.perf_counter() - t0)
        return b

    t_all = best(free, 3)
    sub = free[::64]
    old = _omp_set_threads(1)
    t_one = best(sub, 2) if old is not None else None
    if old is not None:
        _omp_set_threads(old)
    out = {"value": round(len(free) / t_all / 1e9, 6), "unit": "GDoF/s", "cores": threads,
           "kind": "oracle",
           "sample": "all %d free rows of the same operator and input (oracle surrogate rows by "
                     "direct evaluation of the 3D polynomials, element-wise lower-primitive "
                     "rows), best of 3 passes after one warm-up, %d threads; oracle built with "
                     "gcc -O3 -march=native on this host" % (n_free_total, threads),
           "cpu_model": _cpu_model(), "nproc": os.cpu_count(),
           "best_pass_s": round(t_all, 3)}
    if t_one is not None:
        out["single_core"] = {"value": round(len(sub) / t_one / 1e9, 6), "unit": "GDoF/s",
                              "sample": "every 64th free row (%d rows), best of 2 passes after "
                                        "one warm-up, 1 thread" % len(sub)}
    log("cpu baseline: %s" % out)
    res = {}
    for name, (f, u, c) in (solutions or {}).items():
        r = O.residual(N, f, u, kind=oracle.LSQP, q=q, coeffs=c)
        res[name] = O.norm_free(N, r) / O.norm_free(N, f)
        log("oracle relative residual of the %s solution: %.3e" % (name, res[name]))
    return out, res


def solve_bench(ts, G, lam, op, log, keep=None):
    """V(3,3) solves of the manufactured problem to 1e-10 in three precisions,
    and the FP64 double-discretisation solve (surrogate smoothing, IFEM
    residuals, stopped at a relative update of 1e-10).  The first solve of each
    creates the solver and is not timed.  keep (a dict): the canonical host
    copies (f, u, coefficients) of the three surrogate solutions, for the
    oracle's residual check in the CPU leg."""
    import torch
    fb = G.rhs(lam, ts.TS_RHS_MANUFACTURED, [0.55, 1.0])
    out = {}
    u64 = None
    fc = G.to_canon(lam, fb).cpu().numpy() if keep is not None else None
    coef = op.coeffs(lam) if keep is not None else None
    for prec, name, dd in ((ts.TS_F64, "fp64", False), (ts.TS_F32, "fp32_ir", False),
                           (ts.TS_F16W, "fp16w_ir", False), (ts.TS_F64, "fp64_dd", True)):
        sv = ts.Solver(op, lam, precision=prec, rtol=1e-10, max_cycles=100, dd=dd)
        u, rc, info = sv.solve(fb, raise_on_fail=False)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        u, rc, info = sv.solve(fb, raise_on_fail=False)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        rec = {"ms": round(dt * 1e3, 2), "cycles": info.cycles, "status": rc,
               "rel_update" if dd else "rel_residual": info.rel_residual,
               "ms_per_cycle": round(dt * 1e3 / max(info.cycles, 1), 3)}
        if u64 is None:
            u64 = u
        else:
            rec["max_rel_diff_vs_fp64_solve"] = float((u - u64).abs().max() / u64.abs().max())
        out[name] = rec
        log("solve %s: %s" % (name, rec))
        if keep is not None and not dd:
            keep[name] = (fc, G.to_canon(lam, u).cpu().numpy(), coef)
        del sv
    out["fp32_ir_speedup_vs_fp64"] = round(out["fp64"]["ms"] / out["fp32_ir"]["ms"], 3)
    # the coarser levels evaluating the finest level's polynomials (remark in
    # Sec. 3.4): set-up time and the FP64 solve's cycles against one fit per
    # level
    t0 = time.perf_counter()
    opf = ts.Operator(G, lam, method=op.method, q=op.q)
    torch.cuda.synchronize()
    setup_each = time.perf_counter() - t0
    del opf
    t0 = time.perf_counter()
    opc = ts.Operator(G, lam, method=op.method, q=op.q, coarse_from_finest=True)
    torch.cuda.synchronize()
    setup = time.perf_counter() - t0
    sv = ts.Solver(opc, lam, rtol=1e-10, max_cycles=100)
    u, rc, info = sv.solve(fb, raise_on_fail=False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    u, rc, info = sv.solve(fb, raise_on_fail=False)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    rec = {"ms": round(dt * 1e3, 2), "cycles": info.cycles, "status": rc,
           "rel_residual": info.rel_residual, "ms_per_cycle": round(dt * 1e3 / max(info.cycles, 1), 3),
           "operator_setup_ms": round(setup * 1e3, 2),
           "operator_setup_ms_one_fit_per_level": round(setup_each * 1e3, 2),
           "max_rel_diff_vs_fp64_solve": float((u - u64).abs().max() / u64.abs().max())}
    out["fp64_coarse_from_finest"] = rec
    log("solve fp64_coarse_from_finest: %s" % rec)
    del sv, opc
    return out


def small_configs(ts, log, stream):
    """The two small workloads: one FP64 y = Ax on a single macro at level 5
    (6,545 nodes; IFEM vs LSQP q = 2 latency), and the 36-macro shell at
    level 6 (apply, Gauss-Seidel sweep, V(3,3) solves of the manufactured
    problem to 1e-10 with the pure q = 2 surrogate, with the selective
    surrogate that keeps IFEM rows on macros whose fit fails its check, and
    with IFEM)."""
    import torch

    from paper_1608_06473_amd import inputs, study
    out = {}
    v, t = inputs.single_macro()
    M = ts.Mesh(v, t)
    lam = 5
    info = M.layout(lam)
    x = M.to_block(lam, inputs.uniform(info.n_unique, 0))
    res = {"workload": "single macro of the shell r in [0.55, 1], level 5, %d nodes, FP64 y = Ax"
                       % info.n_unique}
    ys = {}
    for name, kw in (("ifem", dict(method=ts.TS_IFEM)), ("lsqp_q2", dict(method=ts.TS_LSQP, q=2))):
        op = ts.Operator(M, lam, sample_j=2, **kw)
        y = M.zeros(lam)
        ts.ts_apply(op.h, lam, ts.TS_F64, x, y, stream)
        us = time_events(lambda: ts.ts_apply(op.h, lam, ts.TS_F64, x, y, stream), 50, stream) * 1e3
        torch.cuda.synchronize()
        ys[name] = y
        res[name + "_us"] = round(us, 2)
        del op
    res["max_rel_diff"] = float((ys["lsqp_q2"] - ys["ifem"]).abs().max() / ys["ifem"].abs().max())
    out["single_macro_l5"] = res
    log("single macro level 5: IFEM %.1f us, LSQP q=2 %.1f us" % (res["ifem_us"], res["lsqp_q2_us"]))

    v, t = inputs.shell36(study.R1, study.R2)
    M = ts.Mesh(v, t)
    lam = 6
    info = M.layout(lam)
    x = M.to_block(lam, inputs.uniform(info.n_unique, 0))
    f = M.rhs(lam, ts.TS_RHS_MANUFACTURED, [study.R1, study.R2])
    res = {"workload": "36-macro shell r in [0.55, 1], level 6, %d free DoF, q = 2, manufactured "
                       "u = sin(pi (r - 0.55) / 0.45) x y z, FP64 V(3,3) to 1e-10" % info.n_free}
    op = ts.Operator(M, lam, method=ts.TS_LSQP, q=2, sample_j=2)
    y = M.zeros(lam)
    ts.ts_apply(op.h, lam, ts.TS_F64, x, y, stream)
    ms = time_events(lambda: ts.ts_apply(op.h, lam, ts.TS_F64, x, y, stream), 20, stream)
    u = x.clone()
    gs = time_events(lambda: ts.ts_smooth(op.h, lam, ts.TS_F64, f, u, 1, stream), 5, stream)
    res["apply_ms"] = round(ms, 4)
    res["apply_gdofs"] = round(info.n_free / ms / 1e6, 2)
    res["gs_sweep_ms"] = round(gs, 4)
    del op, y, u
    for name, kw in (("lsqp_q2", dict(method=ts.TS_LSQP, q=2)),
                     ("lsqp_q2_selective", dict(method=ts.TS_LSQP, q=2, fallback_tol=0.25)),
                     ("ifem", dict(method=ts.TS_IFEM))):
        op = ts.Operator(M, lam, sample_j=2, **kw)
        sv = ts.Solver(op, lam, precision=ts.TS_F64, rtol=1e-10, max_cycles=100)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        u, rc, si = sv.solve(f, raise_on_fail=False)
        torch.cuda.synchronize()
        r = {"status": int(rc), "cycles": int(si.cycles),
             "ms": round((time.perf_counter() - t0) * 1e3, 1),
             "rel_residual": float(si.rel_residual)}
        if rc == ts.TS_OK:
            r["error"] = study.error_norm(M, lam, u)
        if kw.get("fallback_tol"):
            r["ifem_macros_by_level"] = {l: int(op.macro_flags(l).sum()) for l in range(3, lam + 1)}
        res[name] = r
        log("36-macro shell level 6, %s: %s" % (name, json.dumps(r)))
        del sv, op
    out["shell36_l6"] = res
    return out


def serve_bench(n_requests, log, sustained=60):
    """The serve loop on the 288-macro topology: the first n_requests of the
    Poisson(50/s) trace (a burst over the GPU's capacity: latency is
    queueing), and `sustained` requests at 4/s, a rate one GPU keeps up with
    (latency without a queue)."""
    from paper_1608_06473_amd import inputs
    from paper_1608_06473_amd.serve import Server
    out = {}
    for key, n, rate in (("burst", n_requests, 50.0), ("sustained", sustained, 4.0)):
        if n <= 0:
            continue
        trace = inputs.serving_trace(n, rate=rate, seed=0)
        srv = Server(topology="shell288", max_active=32, warm_levels=(4, 5, 6, 7))
        try:
            _, summ = srv.run(trace)
        finally:
            srv.close()
        summ["trace"] = ("first %d requests of the Poisson(%g/s) trace, levels 4-7, r_in ~ "
                         "U[0.4, 0.7], 8 Gaussian bumps, FP32 V(3,3) + FP64 refinement to 1e-8, "
                         "288-macro shell topology; the layout's level data are built at server "
                         "start-up, outside the latencies" % (n, rate))
        log("serving (%s): %s" % (key, json.dumps(summ)))
        out[key] = summ
    return out


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
    ap.add_argument("--only-gs", action="store_true",
                    help="time only the FP64 Gauss-Seidel sweep (profiling runs)")
    ap.add_argument("--only-ifem", action="store_true",
                    help="time only the IFEM volume rows, FP64 apply (profiling runs)")
    ap.add_argument("--copy-calib", action="store_true",
                    help="run a plain 1 GiB device copy (counter calibration) and exit")
    ap.add_argument("--no-solve", action="store_true")
    ap.add_argument("--no-serve", action="store_true")
    ap.add_argument("--no-small", action="store_true",
                    help="skip the single-macro and 36-macro workloads")
    ap.add_argument("--serve-requests", type=int, default=30)
    ap.add_argument("--serve-sustained", type=int, default=60,
                    help="requests of the 4/s serving leg (0: skip)")
    args = ap.parse_args()

    if args.gpus != 1:
        print("bench.py runs on one GPU only (the library has no multi-GPU path); "
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
    # the whole-operator launch (volume rows with the face rows fused in, edge
    # and vertex rows beside it on the operator's side stream), HIP events on
    # the caller's stream, which joins the side stream
    whole_ms = time_events(step, max(5, args.steps), stream)
    # rows of the fused launch: the volume rows and the free nodes of the
    # interior faces (faces shared by two macros), (N-1)(N-2)/2 per face
    tri = np.sort(np.asarray(tet, dtype=np.int64)[:, [[1, 2, 3], [0, 2, 3], [0, 1, 3], [0, 1, 2]]],
                  axis=2).reshape(-1, 3)
    _, cnt = np.unique(tri, axis=0, return_counts=True)
    n_face = int((cnt == 2).sum()) * (2 ** lam - 1) * (2 ** lam - 2) // 2
    fused_alg = 16.0 * (info.n_volume + n_face)

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
    if args.only_gs:
        fb = G.rhs(lam, ts.TS_RHS_MANUFACTURED, [0.55, 1.0])
        ub = xb.clone()
        gs_ms = time_events(lambda: ts.ts_smooth(op.h, lam, ts.TS_F64, fb, ub, 1, stream), 3,
                            stream)
        log("GS sweep (FP64): %.3f ms" % gs_ms)
        return

    extra = {}
    # IFEM apply (comparison path): whole operator, and its volume rows
    # against the FP64 vector peak with the paper's count of 1,353 FLOP per
    # stencil assembly plus 29 per application (Tab. flops)
    opI = ts.Operator(G, lam, method=ts.TS_IFEM)
    ts.ts_apply(opI.h, lam, ts.TS_F64, xb, yb, stream)
    if args.only_ifem:
        iv = time_events(lambda: ts.ts_apply_volume(opI.h, lam, ts.TS_F64, xb, yb, stream), 3,
                         stream)
        log("IFEM volume rows (FP64): %.3f ms" % iv)
        return
    ifem_ms = time_events(lambda: ts.ts_apply(opI.h, lam, ts.TS_F64, xb, yb, stream), 3, stream)
    ifem_vol = time_events(lambda: ts.ts_apply_volume(opI.h, lam, ts.TS_F64, xb, yb, stream), 3,
                           stream)
    ifem_tf = IFEM_FLOP_PER_NODE * info.n_volume / (ifem_vol / 1e3) / 1e12
    extra["ifem_apply"] = {"ms": round(ifem_ms, 4),
                           "gdofs": round(info.n_free / ifem_ms / 1e6, 3),
                           "surrogate_speedup": round(ifem_ms / ms, 2),
                           "volume_ms": round(ifem_vol, 4),
                           "roofline": {"bound": "alu", "achieved": round(ifem_tf, 2),
                                        "peak": FP64_PEAK_TFS, "unit": "TFLOP/s",
                                        "frac": round(ifem_tf / FP64_PEAK_TFS, 4),
                                        "flop_per_node": IFEM_FLOP_PER_NODE,
                                        "kernel": "k_ifem_lds, FP64 apply, volume rows"}}
    log("IFEM apply: %.3f ms (%.2f GDoF/s), volume rows %.3f ms (%.1f TFLOP/s)"
        % (ifem_ms, info.n_free / ifem_ms / 1e6, ifem_vol, ifem_tf))
    # one FP64 V(3,3) cycle with IFEM rows and with the q = 2 surrogate (the
    # paper compares the two methods by their cycle times)
    fI = G.rhs(lam, ts.TS_RHS_MANUFACTURED, [0.55, 1.0])
    cyc = {}
    for name, o in (("ifem", opI), ("lsqp_q2", op)):
        svc = ts.Solver(o, lam, precision=ts.TS_F64, rtol=1e-10)
        uI = G.zeros(lam)
        ts.ts_vcycle(svc.h, ts.TS_F64, fI, uI, stream)
        cyc[name] = time_events(lambda: ts.ts_vcycle(svc.h, ts.TS_F64, fI, uI, stream), 2, stream)
        del svc, uI
    extra["ifem_apply"]["vcycle_ms"] = round(cyc["ifem"], 2)
    extra["ifem_apply"]["surrogate_vcycle_ms"] = round(cyc["lsqp_q2"], 2)
    extra["ifem_apply"]["vcycle_ratio"] = round(cyc["ifem"] / cyc["lsqp_q2"], 2)
    log("FP64 V(3,3) cycle: IFEM %.1f ms, LSQP q=2 %.1f ms" % (cyc["ifem"], cyc["lsqp_q2"]))
    del opI, fI
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
    # the constant stencil of the unmapped macros (the paper's 29-FLOP lower
    # bound): apply, volume kernel, residual and a Gauss-Seidel sweep
    opC = ts.Operator(G, lam, method=ts.TS_CONS)
    ts.ts_apply(opC.h, lam, ts.TS_F64, xb, yb, stream)
    c_ms = time_events(lambda: ts.ts_apply(opC.h, lam, ts.TS_F64, xb, yb, stream), reps, stream)
    c_vol = time_events(lambda: ts.ts_apply_volume(opC.h, lam, ts.TS_F64, xb, yb, stream), reps,
                        stream)
    rC = G.zeros(lam)
    c_res = time_events(lambda: ts.ts_residual(opC.h, lam, ts.TS_F64, xb, xb, rC, stream), reps,
                        stream)
    uC = xb.clone()
    c_gs = time_events(lambda: ts.ts_smooth(opC.h, lam, ts.TS_F64, xb, uC, 1, stream), 3, stream)
    extra["cons_apply"] = {"ms": round(c_ms, 4), "gdofs": round(info.n_free / c_ms / 1e6, 3),
                           "volume_ms": round(c_vol, 4),
                           "volume_gbs": round(alg_bytes / (c_vol / 1e3) / 1e9, 1),
                           "residual_ms": round(c_res, 4), "gs_sweep_ms": round(c_gs, 4),
                           "surrogate_q2_over_cons": round(ms / c_ms, 3)}
    log("constant-stencil apply: %.3f ms (volume %.3f ms), residual %.3f ms, GS sweep %.3f ms"
        % (c_ms, c_vol, c_res, c_gs))
    del opC, rC, uC
    # the symmetric surrogate (edge polynomials at the midpoints, centre from
    # the row sum): the same volume kernel in its row-sum mode
    opS = ts.Operator(G, lam, method=ts.TS_LSQP_SYM, q=q, sample_j=2)
    ts.ts_apply(opS.h, lam, ts.TS_F64, xb, yb, stream)
    sym_ms = time_events(lambda: ts.ts_apply(opS.h, lam, ts.TS_F64, xb, yb, stream), reps, stream)
    extra["sym_apply"] = {"ms": round(sym_ms, 4), "gdofs": round(info.n_free / sym_ms / 1e6, 3)}
    log("symmetric surrogate apply: %.3f ms (%.2f GDoF/s)" % (sym_ms, info.n_free / sym_ms / 1e6))
    del opS
    # q = 2 with surrogate rows on the interior faces as well (FP64 apply,
    # residual and Gauss-Seidel sweep); its largest relative deviation from
    # the operator with exact face rows on this x
    opF = ts.Operator(G, lam, method=ts.TS_LSQP, q=q, sample_j=2, face_surrogate=True)
    yF = torch.zeros_like(xb)
    ts.ts_apply(opF.h, lam, ts.TS_F64, xb, yF, stream)
    fs_ms = time_events(lambda: ts.ts_apply(opF.h, lam, ts.TS_F64, xb, yF, stream), reps, stream)
    ts.ts_apply(op.h, lam, ts.TS_F64, xb, yb, stream)
    torch.cuda.synchronize()
    fs_dev = float((yF - yb).abs().max() / yb.abs().max())
    rF = torch.zeros_like(xb)
    fs_res = time_events(lambda: ts.ts_residual(opF.h, lam, ts.TS_F64, xb, xb, rF, stream), reps,
                         stream)
    uF = xb.clone()
    fs_gs = time_events(lambda: ts.ts_smooth(opF.h, lam, ts.TS_F64, xb, uF, 1, stream), 5, stream)
    extra["face_surrogate_apply"] = {
        "ms": round(fs_ms, 4), "gdofs": round(info.n_free / fs_ms / 1e6, 3),
        "residual_ms": round(fs_res, 4), "gs_sweep_ms": round(fs_gs, 4),
        "max_rel_dev_vs_exact_face_rows": fs_dev}
    log("face-surrogate apply: %.3f ms (%.2f GDoF/s), residual %.3f ms, GS sweep %.3f ms, "
        "deviation %.2e" % (fs_ms, info.n_free / fs_ms / 1e6, fs_res, fs_gs, fs_dev))
    del opF, yF, rF, uF
    # FP32 and FP16-weight applies, residual, Gauss-Seidel sweeps
    x32 = xb.float()
    y32 = torch.zeros_like(x32)
    ts.ts_apply(op.h, lam, ts.TS_F32, x32, y32, stream)
    f32_ms = time_events(lambda: ts.ts_apply(op.h, lam, ts.TS_F32, x32, y32, stream), reps, stream)
    extra["fp32_apply"] = {"ms": round(f32_ms, 4), "gdofs": round(info.n_free / f32_ms / 1e6, 3)}
    ts.ts_apply(op.h, lam, ts.TS_F16W, x32, y32, stream)
    f16_ms = time_events(lambda: ts.ts_apply(op.h, lam, ts.TS_F16W, x32, y32, stream), reps, stream)
    extra["fp16w_apply"] = {"ms": round(f16_ms, 4), "gdofs": round(info.n_free / f16_ms / 1e6, 3)}
    fb = G.rhs(lam, ts.TS_RHS_MANUFACTURED, [0.55, 1.0])
    ub = xb.clone()
    rb = G.zeros(lam)
    res_ms = time_events(lambda: ts.ts_residual(op.h, lam, ts.TS_F64, fb, ub, rb, stream), reps,
                         stream)
    extra["residual"] = {"ms": round(res_ms, 4), "gdofs": round(info.n_free / res_ms / 1e6, 3)}
    gs_ms = time_events(lambda: ts.ts_smooth(op.h, lam, ts.TS_F64, fb, ub, 1, stream), 3, stream)
    f32b, u32 = fb.float(), ub.float()
    gs32_ms = time_events(lambda: ts.ts_smooth(op.h, lam, ts.TS_F32, f32b, u32, 1, stream), 3,
                          stream)
    extra["gs_sweep"] = {"ms": round(gs_ms, 4), "gdofs": round(info.n_free / gs_ms / 1e6, 3),
                         "fp32_ms": round(gs32_ms, 4)}
    log("FP32 apply %.3f ms, FP16W apply %.3f ms, residual %.3f ms, GS sweep %.3f ms (FP32 %.3f)"
        % (f32_ms, f16_ms, res_ms, gs_ms, gs32_ms))
    del x32, y32, f32b, u32, ub, rb, fb
    solutions = {} if not args.no_cpu else None
    if not args.no_solve:
        extra["solve"] = solve_bench(ts, G, lam, op, log, keep=solutions)
    if not args.no_small:
        extra["small_configs"] = small_configs(ts, log, stream)
    if not args.no_serve:
        extra["serving"] = serve_bench(args.serve_requests, log, args.serve_sustained)

    cpu = None
    if not args.no_cpu:
        log("cpu baseline (oracle on host cores)...")
        cpu, ores = cpu_baseline(vtx, tet, lam, q, x_canon, info.n_free, solutions, log)
        for name, v in ores.items():
            extra["solve"][name]["oracle_rel_residual"] = v

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
        "roofline": {
            "bound": "hbm", "achieved": round(fused_alg / (whole_ms / 1e3) / 1e9, 1),
            "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(fused_alg / (whole_ms / 1e3) / 1e9 / HBM_PEAK_GBS, 4),
            "traffic": pmc_traffic("record_whole"),
            "kernel": "k_surr_lds, FP64 apply, the step's launch: volume rows with the "
                      "interior-face rows fused in (timed as ts_apply on its stream, which "
                      "also zeroes the Dirichlet rows and joins the side stream's edge and "
                      "vertex rows)",
            "kernel_ms": round(whole_ms, 4), "algorithmic_bytes": int(fused_alg),
            "rows": int(info.n_volume + n_face),
            "kernel_source_hash": kernel_source_hash()},
        "roofline_volume_rows": {
            "bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
            "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": pmc_traffic(),
            "kernel": "k_surr_lds, FP64 apply, volume rows only (ts_apply_volume)",
            "kernel_ms": round(vol_ms, 4), "algorithmic_bytes": int(alg_bytes)},
        "cpu_baseline": cpu,
    }
    line.update(extra)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
