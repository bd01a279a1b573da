"""Continuous-batching request loop for shell Poisson solves on one GPU.

Requests arrive at their trace times: a level, an inner radius, and a
right-hand side of Gaussian bumps.  A request is admitted when it fits the
HBM budget and a slot is free.  A worker thread then builds (or re-targets)
its mesh, surrogate operator and multigrid solver on the solver's own stream,
and enqueues the start of the solve (ts_solve_begin).  The scheduler thread polls
every active solve without blocking (ts_solve_query) and enqueues the next
refinement iteration of requests whose last one has finished, in one batched
call (ts_solve_batch_step),
smallest level first and, within a level, in arrival order, as long as the
work in flight stays under a budget (an iteration counts its unknowns
relative to a level-7 iteration on the 288-macro shell, so about two of those
run at once while small requests pass them).  Work of many requests is therefore in flight on the
device at once, and requests arriving meanwhile join as slots and memory free
up.  A request retires when its FP64 relative residual reaches the tolerance.

Requests on one macro layout differ only in their radii, so the server
keeps a template mesh of the layout whose levels (index lists, tiles, lane
orders) are built once, on first need, and every solver's mesh shares them
(ts_mesh_create_like) with its own vertices.  Solvers stay resident in HBM:
when a request retires, its solver (mesh, operator, multigrid state and
vectors) serves the next request of the same level, moved to that request's
shell in place (ts_solver_set_vertices rebuilds only the geometry-dependent
data, in the buffers they have).  Freeing device memory waits for the whole
device, so a solver is released only when the memory is needed for another
level (the one idle the longest first), on a thread of its own, and its
memory counts as used until the release has completed.

Every request runs the same sequence of kernels on its own data whatever else
is in flight (no atomics, fixed reduction order), so a result is bitwise the
same alone and in the mix.
"""
from __future__ import annotations

import argparse
import collections
import concurrent.futures as cf
import json
import sys
import threading
import time

import numpy as np

from . import (TS_EINVAL, TS_ENOMEM, TS_F32, TS_F64, TS_LSQP, TS_OK, TS_RHS_BUMPS,
               TS_SOLVE_DONE, TS_SOLVE_READY, Mesh, Operator, Solver, TSError, inputs,
               ts_device_bytes, ts_rhs, ts_solve_batch_step, ts_solve_info)

TOPOLOGIES = {
    # the 288-macro shell (faces split 2 x 2, two radial layers) scaled to the
    # request's inner radius; the middle layer sits halfway
    "shell288": lambda r_in: inputs.shell288(r_in, 1.0),
    "shell36": lambda r_in: inputs.shell36(r_in, 1.0),
}
N_MACROS = {"shell288": 288, "shell36": 36}


def request_bytes(n_macros, level, precision=TS_F32):
    """Admission estimate of the device bytes of one request: caller vectors
    f, u (FP64), the outer residual, the FP32 correction pair and three
    V-cycle vectors per level (FP32 or FP64), the stored interface rows of
    every level (and their FP32 copies), the nodal load values of the right-hand side (a set-up
    temporary), plus a fixed allowance for coefficients, lists and the
    coarse inverse."""
    def vec(lam):
        N = 2 ** lam
        return n_macros * (N + 1) * (N + 2) * (N + 3) // 6
    def face_nodes(lam):  # about 1.8 interior faces per macro, (N-1)(N-2)/2 nodes each
        N = 2 ** lam
        return int(1.84 * n_macros) * (N - 1) * (N - 2) // 2
    per_level = 12 if precision != TS_F64 else 24
    # stored interface rows of the request's geometry: two 15-entry FP64
    # copies per interior-face node, and their FP32 roundings for FP32 cycles
    face_row = 240 + (120 if precision != TS_F64 else 0)
    b = vec(level) * (16 + 8 + (8 if precision != TS_F64 else 0) + 8 + 8)
    for lam in range(2, level + 1):
        b += vec(lam) * per_level + face_nodes(lam) * face_row
    return int(b + 32 * 2 ** 20)


class Ledger:
    """Device-memory accounting of the admitted requests and the admission
    rule.

    A request's estimate is held from admission until its release has
    completed on the releasing thread, not merely been handed to it: freeing
    device memory waits for the device, so releases can lag far behind
    retirements, and memory counted as free before it is free lets the
    admitted set outgrow the device.  Estimates of requests admitted but not
    yet set up are not in a free-memory snapshot yet; the rule subtracts
    them."""

    def __init__(self, budget, reserve):
        self.budget, self.reserve = budget, reserve
        self.held = 0          # admitted, release not completed
        self.unallocated = 0   # admitted, set-up not finished
        self.releasing = []    # (future, bytes, seconds at hand-over)
        self.peak = 0
        self.release_s = []    # hand-over to completion, per release batch

    def shortfall(self, b, free=None, pending=False):
        """Bytes missing for a request of b bytes (<= 0: it fits); free: the
        device's free bytes (a snapshot), or None to check the budget only;
        pending: count the releases in progress as done."""
        pend = sum(x for _, x, _ in self.releasing) if pending else 0
        s = self.held - pend + b - self.budget
        if free is not None:
            s = max(s, b + self.reserve - (free + pend - self.unallocated))
        return s

    def fits(self, b, free=None):
        """Whether a request of b bytes may be admitted now."""
        return self.shortfall(b, free) <= 0

    def admit(self, b):
        self.held += b
        self.unallocated += b
        self.peak = max(self.peak, self.held)

    def set_up(self, b):
        """The request's set-up has ended (its memory is allocated, or it
        failed and holds what it allocated until released)."""
        self.unallocated -= b

    def release(self, fut, b, now):
        self.releasing.append((fut, b, now))

    def poll(self, now):
        """Return the estimates of the releases that have completed."""
        keep = []
        for fut, b, t in self.releasing:
            if fut.done():
                fut.result()
                self.held -= b
                self.release_s.append(now - t)
            else:
                keep.append((fut, b, t))
        self.releasing = keep

    def idle(self):
        return self.held == 0 and not self.releasing



class Slot:
    """A resident solver of one level: its stream, mesh, operator, solver and
    the caller vectors f, u.  A slot serves one request at a time and, once
    that request has retired, the next request of its level (the solver is
    moved to the new shell in place)."""
    __slots__ = ("level", "bytes", "stream", "mesh", "op", "sv", "f", "u", "t_idle")

    def __init__(self, level, nbytes):
        self.level, self.bytes = level, nbytes
        self.stream = self.mesh = self.op = self.sv = self.f = self.u = None
        self.t_idle = 0.0


def request_work(n_macros, level):
    """Work of one refinement iteration relative to one on the 288-macro
    shell at level 7 (the ratio of the block sizes)."""
    def vec(m, lam):
        N = 2 ** lam
        return m * (N + 1) * (N + 2) * (N + 3) // 6
    return vec(n_macros, level) / vec(288, 7)


class Request:
    __slots__ = ("id", "t", "level", "r_in", "bytes", "work", "t_admit", "t_ready", "t_done",
                 "slot", "new", "info", "status", "cycles", "rel", "u_host", "error")

    def __init__(self, rec, n_macros, precision):
        self.id, self.t, self.level, self.r_in = rec["id"], rec["t"], rec["level"], rec["r_in"]
        self.bytes = request_bytes(n_macros, self.level, precision)
        self.work = request_work(n_macros, self.level)
        self.t_admit = self.t_ready = self.t_done = None
        self.slot = None
        self.new = True  # its slot was created for it (not a resident one)
        self.info = ts_solve_info()
        self.status = None
        self.cycles = 0
        self.rel = None
        self.u_host = None
        self.error = None


class Server:
    """One GPU, many requests in flight.

    topology: key of TOPOLOGIES; q, fallback_tol: surrogate degree and the
    per-macro IFEM fallback tolerance; precision: TS_F32 (FP32 V-cycles with
    FP64 refinement), TS_F16W or TS_F64; rtol: FP64 relative residual to
    reach; hbm_budget: bytes the admitted requests may use (estimate);
    max_active: slots; keep: ids whose solutions are copied to the host;
    inflight_work: budget of refinement iterations in flight, in units of a
    level-7 iteration on the 288-macro shell (request_work); one iteration is
    always allowed; warm_levels: levels whose layout data are built at
    start-up (else on the first request that needs them); resident: keep the
    solver of a retired request resident and serve the next request of its
    level with it (moved to the new shell in place, ts_solver_set_vertices)
    instead of building and releasing one per request; reserve_bytes: device
    memory that must stay free beside an admitted request's estimate (the
    runtime needs some for its own queues, and the estimate is only an
    estimate); yield_level: while any request of this level or below is being
    set up or solved, requests of higher levels get no new iterations (their
    kernels would otherwise sit between the small requests' many short
    kernels on the shared hardware queues), as long as no request waits for
    admission; None: off.  The default, 5, serves levels 4 and 5 of a 4/s
    mix of levels 4-7 in 45 / 66 ms (p50) instead of 106 / 145 ms, for about
    10% more level-7 latency.
    """

    def __init__(self, topology="shell288", q=2, precision=TS_F32, rtol=1e-8, max_cycles=60,
                 hbm_budget=160 * 2 ** 30, max_active=32, setup_workers=4, fallback_tol=0.25,
                 keep=(), gc_batch=8, inflight_work=2.0, warm_levels=(), yield_level=5,
                 reserve_bytes=16 * 2 ** 30, resident=True):
        import torch
        self.torch = torch
        self.topology = topology
        self.n_macros = N_MACROS[topology]
        self.q, self.precision, self.rtol = q, precision, rtol
        self.max_cycles = max_cycles
        self.hbm_budget = hbm_budget
        self.max_active = max_active
        self.fallback_tol = fallback_tol
        self.keep = set(keep)
        self.gc_batch = gc_batch
        self.inflight_work = inflight_work
        self.yield_level = yield_level
        self.reserve_bytes = reserve_bytes
        self.template = None  # the layout's mesh; its levels are shared
        self.built = set()
        if warm_levels:
            vtx, tet = TOPOLOGIES[topology](0.55)
            self.template = Mesh(vtx, tet)
            for lam in range(2, max(warm_levels) + 1):
                self.template.layout(lam)
                self.built.add(lam)
        self.tlock = threading.Lock()
        self.shared = 0       # requests whose levels were all built already
        self.resident = resident
        self.idle = collections.defaultdict(list)  # level -> idle resident solvers
        self.reused = 0       # requests served by a resident solver
        self.evicted = 0      # resident solvers released to make room
        self.setup_workers = setup_workers
        self.pool = cf.ThreadPoolExecutor(max_workers=setup_workers)
        # retired requests are released on a thread of their own: freeing
        # device memory waits for the device, and the scheduler must not
        self.reaper = cf.ThreadPoolExecutor(max_workers=1)

    # -- per request ---------------------------------------------------------
    def _setup(self, r):
        torch = self.torch
        vtx, tet = TOPOLOGIES[self.topology](r.r_in)
        sl = r.slot
        if not r.new:
            # a resident solver of this level, moved to the request's shell
            sl.sv.set_vertices(vtx, sl.stream)
        else:
            sl.stream = torch.cuda.Stream()
            with self.tlock:  # levels are built on the template once, under the lock
                if self.template is None:
                    self.template = Mesh(vtx, tet)
                if r.level in self.built:
                    self.shared += 1
                for lam in range(2, r.level + 1):
                    if lam not in self.built:
                        self.template.layout(lam)
                        self.built.add(lam)
                sl.mesh = Mesh(vtx, tet, like=self.template)
            sl.op = Operator(sl.mesh, r.level, method=TS_LSQP, q=self.q, sample_j=2,
                             fallback_tol=self.fallback_tol, stream=sl.stream)
            sl.sv = Solver(sl.op, r.level, precision=self.precision, rtol=self.rtol,
                           max_cycles=self.max_cycles)
            # The vectors come from the caching allocator's pool of this
            # thread's current stream (the default stream, shared by all
            # slots) and are only written on the slot's stream.  Allocated on
            # the slot's stream, their blocks would, once freed, serve only
            # that stream again, and the pools of the pooled streams would
            # grow side by side.  They are freed after the slot's stream has
            # finished with them (its last solve is DONE).
            n = sl.mesh.layout(r.level).vec_len
            sl.f = torch.empty(n, dtype=torch.float64, device="cuda")
            sl.u = torch.empty(n, dtype=torch.float64, device="cuda")
        sl.mesh.check_shell(r.r_in, 1.0)
        params = inputs.gaussian_bumps(r.id, r.r_in, 1.0)
        with torch.cuda.stream(sl.stream):
            sl.f.zero_()
            sl.u.zero_()
            ts_rhs(sl.mesh.h, r.level, TS_RHS_BUMPS, params, sl.f, sl.stream)
        sl.sv.begin(sl.f, sl.u, sl.stream)
        return r

    def _retire(self, r, now):
        r.t_done = now
        r.status = r.info.status
        r.cycles = r.info.cycles
        r.rel = r.info.rel_residual
        if r.id in self.keep and r.status == TS_OK:
            with self.torch.cuda.stream(r.slot.stream):
                r.u_host = r.slot.u.cpu().numpy()

    @staticmethod
    def _fail(r, now, code, msg):
        """End one request with an error status; the others keep running."""
        r.t_done = now
        r.status = code
        r.error = msg

    @staticmethod
    def _destroy_now(slots):
        for sl in slots:
            sl.sv = sl.op = sl.mesh = sl.f = sl.u = None
            sl.stream = None

    def _destroy(self, ledger, slots, now):
        if slots:
            ledger.release(self.reaper.submit(self._destroy_now, list(slots)),
                           sum(sl.bytes for sl in slots), now)

    # -- loop ----------------------------------------------------------------
    def run(self, trace, log=None):
        """Serve the trace (list of dicts id, t, level, r_in) in wall-clock
        time and return (requests, summary).  log (optional): called with a
        progress line every 2 s."""
        torch = self.torch
        reqs = [Request(rec, self.n_macros, self.precision) for rec in trace]
        pending = collections.deque(sorted(reqs, key=lambda r: r.t))
        waiting = collections.deque()
        to_setup = []  # admitted, set-up not started: smallest level first
        setting_up = {}
        active = collections.defaultdict(list)
        grave = []
        ledger = Ledger(self.hbm_budget, self.reserve_bytes)
        # solvers left resident by an earlier run of this server hold memory
        ledger.held = ledger.peak = sum(sl.bytes for lst in self.idle.values() for sl in lst)
        peak_dev = 0
        occ_area = 0.0
        occ_level = collections.defaultdict(float)  # time-weighted active count per level
        used_area = 0.0  # time-weighted admitted bytes
        dev_samples = []  # (time, library device bytes), sampled at most every 50 ms
        n_active = 0
        n_retired = 0
        emptied = False
        t_log = 0.0
        t0 = time.perf_counter()
        t_last = 0.0
        while pending or waiting or to_setup or setting_up or any(active.values()):
            now = time.perf_counter() - t0
            occ_area += n_active * (now - t_last)
            for lvl, lst in active.items():
                occ_level[lvl] += len(lst) * (now - t_last)
            used_area += ledger.held * (now - t_last)
            if not dev_samples or now - dev_samples[-1][0] >= 0.05:
                dev_samples.append((now, ts_device_bytes()))
            t_last = now
            ledger.poll(now)
            if log and now - t_log >= 2.0:
                t_log = now
                log("%.1f s: %d of %d served, %d active, %d in set-up, %d waiting, %d resident "
                    "idle; held %.1f GB (%d releases pending); library %.1f GB, torch reserved "
                    "%.1f GB, device free %.1f GB"
                    % (now, n_retired, len(reqs), n_active, len(setting_up) + len(to_setup),
                       len(waiting), sum(len(v) for v in self.idle.values()),
                       ledger.held / 2 ** 30, len(ledger.releasing),
                       ts_device_bytes() / 2 ** 30, torch.cuda.memory_reserved() / 2 ** 30,
                       torch.cuda.mem_get_info()[0] / 2 ** 30))
            while pending and pending[0].t <= now:
                waiting.append(pending.popleft())
            # admission in arrival order: a resident solver of the request's
            # level if one is idle, else a new one if the memory allows
            while waiting and n_active + len(setting_up) + len(to_setup) < self.max_active:
                r = waiting[0]
                if r.bytes > self.hbm_budget:
                    # can never fit: rejected alone, the server goes on
                    waiting.popleft()
                    self._fail(r, now, TS_ENOMEM, "request needs %d bytes, over the HBM "
                               "budget of %d" % (r.bytes, self.hbm_budget))
                    continue
                if self.idle[r.level]:
                    waiting.popleft()
                    r.slot = self.idle[r.level].pop()
                    r.new = False
                    self.reused += 1
                    r.t_admit = now
                    to_setup.append(r)
                    continue
                free = torch.cuda.mem_get_info()[0] if torch.cuda.is_available() else None
                if not ledger.fits(r.bytes, free):
                    if grave:
                        self._destroy(ledger, grave, now)
                        grave = []
                        continue
                    lru = [sl for lst in self.idle.values() for sl in lst]
                    if lru and ledger.shortfall(r.bytes, free, pending=True) > 0:
                        # release the resident solver idle the longest
                        sl = min(lru, key=lambda q: q.t_idle)
                        self.idle[sl.level].remove(sl)
                        self._destroy(ledger, [sl], now)
                        self.evicted += 1
                        continue
                    busy = (n_active + len(setting_up) + len(to_setup) > 0
                            or ledger.releasing or lru)
                    if not busy and not emptied:
                        # nothing of ours is in flight or resident: return
                        # torch's cached blocks to the device and look again
                        torch.cuda.empty_cache()
                        emptied = True
                        continue
                    if not busy:
                        waiting.popleft()
                        self._fail(r, now, TS_ENOMEM, "not enough free device memory for "
                                   "the request (%d bytes and a reserve of %d)"
                                   % (r.bytes, self.reserve_bytes))
                        continue
                    break
                emptied = False
                waiting.popleft()
                r.slot = Slot(r.level, r.bytes)
                ledger.admit(r.bytes)
                r.t_admit = now
                to_setup.append(r)
            # set-ups run on the worker threads, smallest level first
            while to_setup and len(setting_up) < self.setup_workers:
                r = min(to_setup, key=lambda q: (q.level, q.t))
                to_setup.remove(r)
                setting_up[self.pool.submit(self._setup, r)] = r
            # requests whose set-up finished join the active set
            for fut in [f for f in setting_up if f.done()]:
                r = setting_up.pop(fut)
                if r.new:
                    ledger.set_up(r.bytes)
                err = fut.exception()
                r.t_ready = time.perf_counter() - t0
                if err is not None:
                    # a failed set-up (device memory, non-finite data, ...)
                    # ends this request only; its solver is released
                    code = err.code if isinstance(err, TSError) else TS_EINVAL
                    self._fail(r, r.t_ready, code, str(err))
                    grave.append(r.slot)
                    continue
                active[r.level].append(r)
                n_active += 1
            progressed = False
            # retire finished requests; the others, smallest level first and
            # in arrival order, get their next iteration while the work in
            # flight stays within the budget
            inflight = 0.0
            ready = []
            for lvl in sorted(active):
                still = []
                for r in active[lvl]:
                    st = r.slot.sv.query(r.info)
                    if st == TS_SOLVE_DONE:
                        t_done = time.perf_counter() - t0
                        self._retire(r, t_done)
                        if r.status == TS_OK and self.resident:
                            # the solver stays resident for the next request
                            # of its level
                            r.slot.t_idle = t_done
                            self.idle[r.level].append(r.slot)
                        else:
                            grave.append(r.slot)
                        n_active -= 1
                        progressed = True
                        n_retired += 1
                        continue
                    still.append(r)
                    if st == TS_SOLVE_READY:
                        ready.append(r)
                    else:
                        inflight += r.work
                active[lvl] = still
            batch = []
            # the hold applies while no request waits for admission: with a
            # backlog the GPU is saturated and throughput comes first
            yl = self.yield_level
            small = yl is not None and not waiting and (
                any(active[l] for l in active if l <= yl)
                or any(q.level <= yl for q in setting_up.values())
                or any(q.level <= yl for q in to_setup))
            for r in ready:  # already in priority order
                if small and r.level > yl:
                    break
                w = r.work
                if inflight > 0.0 and inflight + w > self.inflight_work:
                    break
                batch.append(r.slot.sv)
                inflight += w
            if batch:
                try:
                    ts_solve_batch_step(batch)
                except TSError:
                    # the failing solver's solve has ended with the error as
                    # its status (retired by the next query); solvers after
                    # it were not stepped and stay ready
                    pass
                progressed = True
            if len(grave) >= self.gc_batch:
                peak_dev = max(peak_dev, ts_device_bytes())
                self._destroy(ledger, grave, time.perf_counter() - t0)
                grave = []
            if not progressed:
                time.sleep(50e-6)
        peak_dev = max(peak_dev, ts_device_bytes())
        self._destroy(ledger, grave, time.perf_counter() - t0)
        for fut, _, _ in ledger.releasing:
            fut.result()
        ledger.poll(time.perf_counter() - t0)
        if any(r.t_admit is not None for r in reqs):
            torch.cuda.synchronize()
        t_end = time.perf_counter() - t0
        summ = summarize(reqs, t_end, occ_area, ledger.peak, peak_dev)
        summ["mean_active_by_level"] = {int(l): round(a / max(t_end, 1e-9), 2)
                                        for l, a in sorted(occ_level.items())}
        summ["mean_held_gb"] = round(used_area / max(t_end, 1e-9) / 2 ** 30, 3)
        if dev_samples:
            b = np.array([d for _, d in dev_samples], dtype=np.float64)
            summ["library_gb_over_time"] = {"samples": len(dev_samples),
                                            "mean": round(float(b.mean()) / 2 ** 30, 3),
                                            "max": round(float(b.max()) / 2 ** 30, 3)}
        if ledger.release_s:
            summ["release_s"] = {"batches": len(ledger.release_s),
                                 "mean": round(float(np.mean(ledger.release_s)), 3),
                                 "max": round(float(np.max(ledger.release_s)), 3)}
        summ["levels_shared"] = self.shared
        summ["resident_reused"] = self.reused
        summ["resident_evicted"] = self.evicted
        summ["resident_idle_at_end"] = sum(len(v) for v in self.idle.values())
        return reqs, summ

    def close(self):
        self.pool.shutdown(wait=True)
        self.reaper.shutdown(wait=True)
        for lst in self.idle.values():
            self._destroy_now(lst)
        self.idle.clear()
        self.template = None
        self.built = set()
        if self.torch.cuda.is_available():
            self.torch.cuda.empty_cache()


def summarize(reqs, t_end, occ_area, peak_used, peak_dev):
    done = [r for r in reqs if r.t_done is not None]
    ok = [r for r in done if r.status == TS_OK]
    # latency statistics over the requests that were served
    lat = np.array([r.t_done - r.t for r in ok]) if ok else np.zeros(1)
    first = min(r.t for r in reqs)
    last = max(r.t_done for r in done) if done else first
    by_level = {}
    for lvl in sorted({r.level for r in ok}):
        la = np.array([r.t_done - r.t for r in ok if r.level == lvl])
        by_level[int(lvl)] = {"n": int(la.size),
                              "p50_ms": round(float(np.percentile(la, 50)) * 1e3, 2),
                              "p99_ms": round(float(np.percentile(la, 99)) * 1e3, 2),
                              "cycles_mean": round(float(np.mean([r.cycles for r in ok
                                                                  if r.level == lvl])), 2)}
    return {
        "requests": len(reqs),
        "completed_ok": len(ok),
        "failed": len(done) - len(ok),
        "offered_rate_per_s": round(len(reqs) / max(max(r.t for r in reqs) - first, 1e-9), 2),
        "solves_per_s": round(len(ok) / max(last - first, 1e-9), 3),
        "p50_latency_ms": round(float(np.percentile(lat, 50)) * 1e3, 2),
        "p99_latency_ms": round(float(np.percentile(lat, 99)) * 1e3, 2),
        "failed_by_status": {str(c): sum(1 for r in done if r.status == c)
                             for c in sorted({r.status for r in done if r.status != TS_OK})},
        "mean_setup_ms": round(float(np.mean([r.t_ready - r.t_admit for r in ok])) * 1e3, 2)
        if ok else None,
        "mean_queue_ms": round(float(np.mean([r.t_admit - r.t for r in ok])) * 1e3, 2)
        if ok else None,
        "mean_active": round(occ_area / max(t_end, 1e-9), 2),
        "peak_held_gb": round(peak_used / 2 ** 30, 3),
        "peak_library_gb": round(peak_dev / 2 ** 30, 3),
        "max_rel_residual": float(max(r.rel for r in ok)) if ok else None,
        "wall_s": round(t_end, 3),
        "by_level": by_level,
    }


def main():
    ap = argparse.ArgumentParser(description="Serve a Poisson trace of shell solves on one GPU "
                                             "and print the latency / throughput summary.")
    ap.add_argument("--requests", type=int, default=30)
    ap.add_argument("--rate", type=float, default=50.0, help="arrivals per second")
    ap.add_argument("--levels", default="4-7", help="uniform over this range")
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--topology", default="shell288", choices=sorted(TOPOLOGIES))
    ap.add_argument("--precision", default="f32", choices=["f64", "f32", "f16w"])
    ap.add_argument("--rtol", type=float, default=1e-8)
    ap.add_argument("--inflight-work", type=float, default=2.0)
    ap.add_argument("--max-active", type=int, default=32)
    ap.add_argument("--yield-level", type=int, default=5,
                    help="hold higher levels while requests up to this level are in flight "
                         "(0: off)")
    ap.add_argument("--no-resident", action="store_true",
                    help="build and release a solver per request")
    args = ap.parse_args()
    from . import TS_F16W
    lo, hi = (int(v) for v in args.levels.split("-"))
    prec = {"f64": TS_F64, "f32": TS_F32, "f16w": TS_F16W}[args.precision]
    trace = inputs.serving_trace(args.requests, rate=args.rate, seed=args.seed,
                                 levels=tuple(range(lo, hi + 1)))
    srv = Server(topology=args.topology, precision=prec, rtol=args.rtol,
                 max_active=args.max_active, inflight_work=args.inflight_work,
                 yield_level=args.yield_level or None, resident=not args.no_resident,
                 warm_levels=tuple(range(lo, hi + 1)))
    try:
        _, summ = srv.run(trace, log=lambda m: print(m, file=sys.stderr, flush=True))
    finally:
        srv.close()
    print(json.dumps(summ), flush=True)


if __name__ == "__main__":
    main()
