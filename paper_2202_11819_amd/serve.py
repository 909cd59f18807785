"""Request loop for the served form, its serial baseline, and their benchmarks.

Serving here is continuous batching: requests that arrive while others run
are admitted as soon as a slot and enough of the HBM budget are free, their
grids stay resident, and every round advances all running requests together
(one fused launch per sweep over all of their tiles).  Finished requests are
copied to page-locked host memory while later rounds run.  Latency is
measured from a request's arrival to its result being in host memory.

The baseline serves the same arrival trace one request at a time in arrival
order with the plain solver (a solver per request, graph mode); its latencies
follow from the measured service times: finish_i = max(arrival_i,
finish_{i-1}) + service_i.
"""
from __future__ import annotations

import collections
import json
import math
import sys
import time

import numpy as np
import torch

from . import j3d
from . import workloads as W
from .api import Batch, Pool, Solver


def nearest_rank(values, q):
    """Nearest-rank percentile (q in (0, 100])."""
    v = sorted(values)
    if not v:
        return float("nan")
    k = max(1, math.ceil(q / 100.0 * len(v)))
    return v[k - 1]


def serve_pool(trace, budget_bytes, max_slots=256, round_sweeps=50, check_every=50, tol=0.0,
               keep_results=False, log=None, fill_cells=None, tune=None, backlog_share=None, two_sweep=False):
    """Serve `trace` (list of workloads.Request) in real time; per-request records.
    fill_cells, backlog_share: round policy, tune: (variant, zchunk) of the
    rounds (None keeps the library defaults), two_sweep: two sweeps per launch."""
    pool = Pool(budget_bytes, max_slots=max_slots)
    if two_sweep:
        pool.set_two_sweep(True)
    if fill_cells is not None or backlog_share is not None:
        pool.set_policy(1 << 25 if fill_cells is None else fill_cells, 32, 2 if backlog_share is None else backlog_share)
    if tune is not None:
        pool.set_tune(*tune)
    problems = [W.to_problem(r.spec) for r in trace]
    pending = collections.deque(range(len(trace)))
    waiting = collections.deque()
    active = {}
    recs = [None] * len(trace)
    done = 0
    busy = False
    t0 = time.perf_counter()
    rounds = 0
    try:
        while done < len(trace):
            now = time.perf_counter() - t0
            while pending and trace[pending[0]].arrival <= now:
                waiting.append(pending.popleft())
            finished, busy = pool.poll()
            now = time.perf_counter() - t0
            for slot in finished:
                i = active.pop(slot)
                u, res, it = pool.result(slot)
                recs[i] = {"i": i, "arrival": trace[i].arrival, "done": now, "latency": now - trace[i].arrival,
                           "residual": res, "iters": it, "cells": problems[i].cells}
                if keep_results:
                    recs[i]["u"] = u.copy()
                pool.release(slot)
                done += 1
                if log and done % 100 == 0:
                    log(f"[serve] {done}/{len(trace)} done at {now:.1f} s, {len(active)} running")
            while waiting:
                i = waiting[0]
                slot = pool.try_admit(problems[i], trace[i].spec.iters, tol=tol, check_every=check_every)
                if slot is None:
                    if not active and not busy:
                        raise RuntimeError(f"request {i} ({problems[i].n}) does not fit an empty pool")
                    break
                waiting.popleft()
                active[slot] = i
            if not busy and active:
                busy = pool.step(round_sweeps)
                rounds += busy
                if not busy:  # every admitted request has finished: their result copies are in flight
                    time.sleep(0.0002)
            elif not active and not waiting and pending:
                # idle until the next arrival
                gap = trace[pending[0]].arrival - (time.perf_counter() - t0)
                if gap > 0:
                    time.sleep(min(gap, 0.001))
    finally:
        pool.close()
    return recs, rounds


def serve_serial(trace, log=None, keep_results=False, tol=0.0, check_every=50, mode="graph"):
    """The same trace, one plain solve at a time in arrival order.  With tol > 0
    a solve runs in pieces of check_every sweeps (the last one shorter), reads
    the residual after each and stops at the first r <= tol, the same rule the
    pool applies."""
    recs = []
    finish = 0.0
    for i, r in enumerate(trace):
        t0 = time.perf_counter()
        s = Solver(r.spec.n, nblk=r.spec.nblk, bc=r.spec.bc, seed=r.spec.seed, pid=r.spec.pid)
        if tol > 0:
            done = 0
            while True:
                k = min(check_every, r.spec.iters - done)
                res = s.run(k, mode=mode, residual=True)
                done += k
                if res <= tol or done >= r.spec.iters:
                    break
        else:
            res = s.run(r.spec.iters, mode=mode, residual=True)
            done = r.spec.iters
        u = s.get_interior()
        s.close()
        service = time.perf_counter() - t0
        start = max(r.arrival, finish)
        finish = start + service
        rec = {"i": i, "arrival": r.arrival, "done": finish, "latency": finish - r.arrival, "service": service,
               "residual": res, "iters": done, "cells": int(np.prod(r.spec.n))}
        if keep_results:
            rec["u"] = u
        recs.append(rec)
        if log and (i + 1) % 100 == 0:
            log(f"[serial] {i + 1}/{len(trace)}")
    return recs


def summarize(recs, warmup):
    m = [r for r in recs if r["i"] >= warmup]
    lat = [r["latency"] for r in m]
    span = max(r["done"] for r in m) - min(r["arrival"] for r in m)
    lups = sum(r["cells"] * r["iters"] for r in m)
    return {"solves_per_s": round(len(m) / span, 3), "p50_ms": round(1e3 * nearest_rank(lat, 50), 2),
            "p99_ms": round(1e3 * nearest_rank(lat, 99), 2), "mean_ms": round(1e3 * float(np.mean(lat)), 2),
            "GLUPs": round(lups / span / 1e9, 2), "requests": len(m), "span_s": round(span, 2)}


def _log(*a):
    print(*a, file=sys.stderr, flush=True)


def serve_bench(count=1100, load=0.8, tol=0.0, fill_cells=None, backlog_share=None, pool_tune=None,
                pool_two_sweep=False, serial_two_sweep=False, dump="", log=_log):
    """Served workload: Poisson arrivals at `load` x the serial capacity, served
    by the pool and, on the same trace, one request at a time by plain solves.
    Returns the benchmark record (a dict)."""
    warmup = min(100, count // 10)
    base = W.serve_trace(count=count, rate=1.0)
    smode = "two_sweep" if serial_two_sweep else "graph"
    # serial capacity from a sample of the same request mix, after a few
    # untimed solves (first-call costs are not part of the service time)
    serve_serial(W.rescale_arrivals(base[-5:], 1e9), mode=smode)
    sample = base[: min(40, count)]
    t0 = time.perf_counter()
    serve_serial(W.rescale_arrivals(sample, 1e9), mode=smode)
    mean_service = (time.perf_counter() - t0) / len(sample)
    rate = load / mean_service
    trace = W.rescale_arrivals(base, rate)
    log(f"[serve] mean serial service {mean_service * 1e3:.1f} ms -> arrival rate {rate:.2f}/s ({load} x capacity)")
    free = torch.cuda.mem_get_info()[0]
    budget = int(min(200e9, 0.85 * free))
    recs, rounds = serve_pool(trace, budget, log=log, fill_cells=fill_cells, tune=pool_tune,
                              backlog_share=backlog_share, tol=tol, two_sweep=pool_two_sweep)
    pool_sum = summarize(recs, warmup)
    srecs = serve_serial(trace, log=log, tol=tol, mode=smode)
    serial_sum = summarize(srecs, warmup)
    # every request served in the mix against the same request solved alone:
    # the last sweep's residual (bit pattern) and the sweep count must agree
    same_res = sum(1 for a, b in zip(recs, srecs)
                   if np.float64(a["residual"]).tobytes() == np.float64(b["residual"]).tobytes())
    same_it = sum(1 for a, b in zip(recs, srecs) if a["iters"] == b["iters"])
    early = sum(1 for a, r in zip(recs, trace) if a["iters"] < r.spec.iters)
    if dump:
        with open(dump, "w") as f:
            json.dump({"rate": rate, "pool": recs, "serial": srecs,
                       "specs": [[list(r.spec.n), r.spec.iters] for r in trace]}, f)
    return {"metric": "served solves/s and p50/p99 latency (arrival to result on host)",
            "value": pool_sum["solves_per_s"], "unit": "solves/s", "higher_is_better": True,
            "pool": pool_sum, "serial_plain": serial_sum, "rounds": rounds,
            "p99_vs_serial": round(serial_sum["p99_ms"] / pool_sum["p99_ms"], 3),
            "mix_vs_alone": {"requests": len(recs), "residual_bit_identical": same_res,
                             "sweeps_identical": same_it, "stopped_early": early},
            "pool_two_sweep": pool_two_sweep, "serial_mode": smode,
            "pool_tune": list(pool_tune) if pool_tune else None,
            "config": {"workload": f"{count} Jacobi3D solve requests, Poisson arrivals at {rate:.2f}/s "
                                   f"({load} x serial capacity), per-axis size U{{32..384}}, 50..2000 sweeps, "
                                   f"residual every 50, tol {tol:g}, budget {budget / 1e9:.0f} GB, "
                                   f"first {warmup} discarded", "dtype": "f64"}}


def bench_serve(args):
    fill = int(getattr(args, "fill_cells", -1))
    share = int(getattr(args, "backlog_share", -1))
    ptune = getattr(args, "pool_tune", "")
    out = serve_bench(count=int(getattr(args, "requests", 0) or 1100), load=float(getattr(args, "load", 0.8) or 0.8),
                      tol=float(getattr(args, "tol", 0.0) or 0.0), fill_cells=None if fill < 0 else fill,
                      backlog_share=None if share < 0 else share,
                      pool_tune=tuple(int(v) for v in ptune.split(",")) if ptune else None,
                      pool_two_sweep=bool(getattr(args, "pool_two_sweep", False)),
                      serial_two_sweep=bool(getattr(args, "serial_two_sweep", False)),
                      dump=getattr(args, "serve_dump", ""))
    print(json.dumps(out), flush=True)


def batch_bench(tune=None, retune=False, batch_only=False, two_sweep=False, loop=True, log=_log):
    """Batched workload: 256 problems in one launch per sweep (autotuned shape,
    or `tune`) against the same problems solved one after another with the
    plain solver.  Returns the benchmark record (a dict)."""
    from .autotune import tune_batch

    specs = W.batch()
    problems = [W.to_problem(s) for s in specs]
    iters = [s.iters for s in specs]
    lups = sum(p.cells * it for p, it in zip(problems, iters))
    search = None
    if tune is None:
        t0 = time.perf_counter()
        tune, searched = tune_batch(problems, iters, log=log, force=retune, report=True)
        search = {"candidates": searched, "seconds": round(time.perf_counter() - t0, 2)}
    tune = tuple(tune)
    log(f"[batch] tune {tune} ({j3d.variants()[tune[0]]})")

    def timed_batch(t, two=False):
        b = Batch(problems, iters, tune=t)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(b.stream)
        b.run(residuals=False, two_sweep=two)
        e1.record(b.stream)
        e1.synchronize()
        b.close()
        return e0.elapsed_time(e1) * 1e-3

    timed_batch(tune)
    tb = min(timed_batch(tune) for _ in range(2))
    out = {"metric": "batched FP64 Jacobi3D GLUP/s (256 problems, one launch per sweep)",
           "value": round(lups / tb / 1e9, 2), "unit": "GLUP/s", "higher_is_better": True,
           "batched_s": round(tb, 4), "tune": list(tune), "tile": list(j3d.variants()[tune[0]]),
           "autotune": search,
           "config": {"workload": f"256 independent problems, per-axis size log-uniform in [32, 256], "
                                  f"per-face bc U[-1,1], 100..1000 sweeps, {lups / 1e9:.1f} GLUP in total",
                      "dtype": "f64"}}
    if batch_only:
        return out
    if two_sweep:
        # the same batch with two sweeps per launch (all problems are undivided)
        timed_batch(tune, True)
        t2 = min(timed_batch(tune, True) for _ in range(2))
        out["two_sweep_batched_s"] = round(t2, 4)
        out["two_sweep_GLUPs"] = round(lups / t2 / 1e9, 2)
    if loop:
        # per-problem loop: each problem solved on its own with the plain solver
        run_s = 0.0
        wall0 = time.perf_counter()
        for s in specs:
            sol = Solver(s.n, bc=s.bc, seed=s.seed, pid=s.pid)
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(sol.stream)
            sol.run(s.iters, mode="graph")
            e1.record(sol.stream)
            e1.synchronize()
            run_s += e0.elapsed_time(e1) * 1e-3
            sol.close()
        wall = time.perf_counter() - wall0
        out.update({"per_problem_loop_s": round(run_s, 4), "per_problem_loop_GLUPs": round(lups / run_s / 1e9, 2),
                    "per_problem_loop_wall_s": round(wall, 2), "speedup_vs_loop": round(run_s / tb, 3)})
    return out


def bench_batch(args):
    fixed = getattr(args, "tune", "")
    out = batch_bench(tune=tuple(int(v) for v in fixed.split(",")) if fixed else None,
                      retune=getattr(args, "retune", False), batch_only=getattr(args, "batch_only", False),
                      two_sweep=getattr(args, "batch_two_sweep", False))
    print(json.dumps(out), flush=True)
