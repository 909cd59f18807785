#!/usr/bin/env python3
"""Benchmark of the FP64 Jacobi3D hot path on one MI355X.

Default workload (one JSON line): a 512^3 FP64 grid over-decomposed into
8x8x8 blocks of 64^3, zero Dirichlet boundary, seeded U[0,1) interior.  One
step is a whole solve: reset the interior from a copy resident in HBM, then
1000 sweeps (each packs, exchanges and unpacks all halos and updates every
block, fused into one kernel and replayed from a HIP graph) with the residual
of the last sweep.  value = interior cells x sweeps / step time (GLUP/s).

The same line carries the rest of the metric under "configs", one compact
record per workload: the 512^3 grid in the unfused and fused modes, the
1024^3 grid at four decompositions, the batched form (256 problems) against
a per-problem loop, and the served form (Poisson arrivals) against serial
plain solves with p50/p99 latency (--headline-only skips them).

Other workloads (--workload): modes, sweep (1024^3 decompositions), batch,
serve, odf, hostex, twostep; each prints its own JSON lines.  Multi-GPU runs
are not part of the library: --gpus above 1 exits with a message.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "FP64 Jacobi3D GLUP/s + % HBM peak; served solves/s, p50/p99 latency"
HBM_PEAK_GBPS = 8000.0   # MI355X HBM3E, published
FP64_PEAK_TFLOPS = 78.6  # MI355X FP64 vector, published


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def sweep_bytes(problem) -> int:
    """Algorithmic bytes of one fused sweep over all blocks of a problem.

    Per block: read and write every interior cell once (16 B/cell), read the
    six halo faces (8 B/cell, global-boundary faces included: y and z halos
    are the neighbours' own boundary rows / planes), and write each x face
    that has a neighbour into that neighbour's x-halo array (8 B/cell).
    """
    from paper_2202_11819_amd import j3d
    nb, ext = j3d.j3d_block_extents(problem)
    total = 0
    for bz, ez in enumerate(ext[2]):
        for by, ey in enumerate(ext[1]):
            for bx, ex in enumerate(ext[0]):
                faces = [ey * ez, ey * ez, ex * ez, ex * ez, ex * ey, ex * ey]
                has = [bx > 0, bx + 1 < nb[0], by > 0, by + 1 < nb[1], bz > 0, bz + 1 < nb[2]]
                total += 16 * ex * ey * ez + 8 * sum(faces) + 8 * sum(f for f, h in zip(faces[:2], has[:2]) if h)
    return total


def measured_traffic(edge, blocks):
    """HBM bytes per sweep launch from the committed rocprofv3 counter runs, if the
    kernel source is unchanged since they were taken (else None)."""
    import hashlib
    path = os.path.join(ROOT, "profiles", f"sweep_kernel_{edge}cubed_{blocks}x{blocks}x{blocks}_blocks.traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f)
    with open(os.path.join(ROOT, rec["kernel_source"]), "rb") as f:
        if hashlib.sha256(f.read()).hexdigest() != rec["kernel_source_sha256"]:
            return None
    return rec["fetch_bytes_per_launch"] + rec["write_bytes_per_launch"]


def copy_bandwidth(nbytes=2 << 30, reps=10, runtime=False):
    """Measured streaming copy (read + write bytes per second), GB/s: the
    library's copy kernel, and with runtime=True also the HIP runtime's own
    device-to-device copy (hipMemcpyAsync, through torch's copy_) as a pair."""
    import torch
    from paper_2202_11819_amd import j3d
    src = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    dst = torch.empty_like(src)
    st = torch.cuda.current_stream()

    def timed(fn):
        fn()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(st)
        for _ in range(reps):
            fn()
        e1.record(st)
        e1.synchronize()
        return 2 * nbytes / (e0.elapsed_time(e1) / reps * 1e-3) / 1e9

    lib = timed(lambda: j3d.j3d_device_copy(dst.data_ptr(), src.data_ptr(), nbytes, st.cuda_stream))
    rt = timed(lambda: dst.copy_(src)) if runtime else None
    del src, dst
    torch.cuda.empty_cache()
    return (lib, rt) if runtime else lib


def cpu_baseline(n, target_seconds=15.0):
    """The oracle as it stands, on this host's cores, over a bounded sample.

    The timed copy is the oracle's source built -O3 -march=native on this
    host (the parity build is portable; a CPU test checks that both give the
    same bits).  The oracle's set-up (ghost fill, seeded interior) and
    copy-out are timed separately by a 1-sweep run and subtracted, so the
    rate is per sweep."""
    from oracle import oracle
    omp = os.environ.get("OMP_NUM_THREADS", "")
    threads = int(omp or 0) or len(os.sched_getaffinity(0))
    threads = max(1, min(threads, 64))
    cells = n[0] * n[1] * n[2]

    def rate(threads_, seconds):
        def timed(t):
            t0 = time.perf_counter()
            oracle.jacobi(n, t, seed=1, nthreads=threads_, native=True)
            return time.perf_counter() - t0

        t1 = timed(1)
        per = max((timed(3) - t1) / 2, 1e-4)
        k = max(1, min(2000, int(seconds / per)))
        dt = max(timed(1 + k) - t1, 1e-6)
        return cells * k / dt / 1e9, k, dt

    value, k, dt = rate(threads, target_seconds)
    one, k1, dt1 = rate(1, target_seconds / 3)
    return {"value": round(value, 4), "unit": "GLUP/s", "cores": threads, "kind": "oracle",
            "sample": f"{n[0]}x{n[1]}x{n[2]} seeded grid (the benchmark's problem), {k} sweeps taking "
                      f"{dt:.1f} s on {threads} threads, set-up and copy-out of a 1-sweep run subtracted",
            "build": " ".join(["gcc"] + oracle.NATIVE_CFLAGS),
            "one_thread_value": round(one, 4), "one_thread_sample": f"{k1} sweeps taking {dt1:.1f} s",
            "cpu_model": cpu_model(), "omp_num_threads": omp or None, "host_cpus": os.cpu_count(),
            "affinity_cpus": len(os.sched_getaffinity(0))}


def cpu_model():
    """lscpu's model name (with vendor and family when the name is generic)."""
    import subprocess
    fields = {}
    try:
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
        for line in out.splitlines():
            if ":" in line:
                k, v = line.split(":", 1)
                fields[k.strip()] = v.strip()
    except (OSError, subprocess.SubprocessError):
        pass
    name = fields.get("Model name", "")
    if not name:
        try:
            with open("/proc/cpuinfo") as f:
                for line in f:
                    if line.startswith("model name"):
                        name = line.split(":", 1)[1].strip()
                        break
        except OSError:
            pass
    extra = [f"{k} {fields[k]}" for k in ("Vendor ID", "CPU family", "Model", "Stepping", "Socket(s)",
                                          "Core(s) per socket", "Thread(s) per core") if k in fields]
    return f"{name or 'unknown'} ({', '.join(extra)})" if extra else (name or "unknown")


def bench_overdecomposed(args):
    import torch
    from paper_2202_11819_amd import api, j3d
    from paper_2202_11819_amd import workloads as W

    spec = W.overdecomposed(nb=args.blocks, edge=args.edge, iters=args.sweeps)
    n, sweeps = spec.n, spec.iters
    cells = n[0] * n[1] * n[2]
    log(f"[bench] workload {n} as {spec.nblk} blocks, {sweeps} sweeps/step, mode {args.mode}")
    s = api.Solver(n, nblk=spec.nblk, seed=spec.seed)
    if args.tune:
        v, zc, bpc = (int(x) for x in args.tune.split(","))
        s.set_tune(v, zc, bpc)
    tune = s.get_tune()                   # (variant, zchunk, blocks_per_cu)
    u0 = s.get_interior_device()          # the seeded interior, kept resident in HBM
    stream = torch.cuda.current_stream()
    per_launch = sweep_bytes(s.problem)

    def step(timing=None):
        s.set_interior(u0)
        if timing is not None:
            timing[0].record(stream)
        s.run(sweeps - 1, mode=args.mode)
        if timing is not None:
            timing[1].record(stream)
        return s.run(1, mode="fused", residual=True)

    for w in range(args.warmup):
        step()
        log(f"[bench] warmup {w + 1}/{args.warmup} done")
    torch.cuda.synchronize()
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
           for _ in range(args.steps)]
    t_start, t_end = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    wall0 = time.perf_counter()
    t_start.record(stream)
    res = None
    for k in range(args.steps):
        res = step(evs[k])
        log(f"[bench] step {k + 1}/{args.steps} done")
    t_end.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - wall0
    ms_total = t_start.elapsed_time(t_end)
    ms_step = ms_total / args.steps
    # each step's sweep time; a step also resets the interior and takes one checked sweep
    ms_steps = [a.elapsed_time(b) for a, b in evs]
    kernel_ms = sum(a.elapsed_time(b) for a, b in evs) / (args.steps * (sweeps - 1))
    glups = cells * sweeps / (ms_step * 1e-3) / 1e9
    achieved = per_launch / (kernel_ms * 1e-3) / 1e9
    traffic_bytes = measured_traffic(args.edge, args.blocks) if args.mode == "graph" and not args.tune else None
    out = {
        "metric": METRIC, "value": round(glups, 3), "unit": "GLUP/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_step, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"{n[0]}^3 FP64 grid as {spec.nblk[0]}x{spec.nblk[1]}x{spec.nblk[2]} blocks of "
                               f"{n[0] // spec.nblk[0]}^3, zero Dirichlet boundary, seeded U[0,1) interior, "
                               f"{sweeps} sweeps per step (pack+exchange+unpack+update fused, {args.mode})",
                   "grid": list(n), "blocks": list(spec.nblk), "sweeps": sweeps, "mode": args.mode,
                   "tune": list(tune), "tile": list(j3d.variants()[tune[0]])},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBPS, 4),
                     "traffic": (round(traffic_bytes / (kernel_ms * 1e-3) / 1e9, 1) if traffic_bytes else None),
                     "kernel": "sweep_kernel", "bytes_per_launch": per_launch,
                     "traffic_bytes_per_launch": traffic_bytes,
                     "avg_launch_ms": round(kernel_ms, 4)},
        "residual": res,
        "wall_s": round(wall, 3),
        "sweep_ms_per_step": {"mean": round(sum(ms_steps) / len(ms_steps), 3), "min": round(min(ms_steps), 3),
                              "max": round(max(ms_steps), 3)},
    }
    s.close()
    del u0
    torch.cuda.empty_cache()
    if not args.headline_only:
        out["configs"] = side_configs(args, spec)
    if not args.no_copy:
        lib_copy, rt_copy = copy_bandwidth(runtime=True)
        out["copy_GBps"] = round(lib_copy, 1)
        out["runtime_copy_GBps"] = round(rt_copy, 1)
        out["roofline"]["frac_of_copy"] = round(achieved / out["copy_GBps"], 4)
    if not args.no_cpu_baseline:
        log("[bench] cpu baseline (oracle) ...")
        out["cpu_baseline"] = cpu_baseline(n, args.cpu_seconds)
    print(json.dumps(out), flush=True)


def side_configs(args, spec):
    """The rest of the metric, one compact record per configuration: the same
    512^3 grid in the unfused and fused modes (and bit-identical to the
    undivided run), the 1024^3 decomposition sweep, the batched form against a
    per-problem loop, and the served form against serial plain solves."""
    out = {}
    log("[bench] config: modes of the overdecomposed grid")
    out["overdecomposed_modes"] = modes_side(spec)
    log("[bench] config: 1024^3 decompositions")
    out["decompositions_1024"] = {"workload": "1024^3 FP64 grid, 500 sweeps (graph) per decomposition",
                                  "runs": sweep_records(iters=args.sweep_iters)}
    from paper_2202_11819_amd import serve
    log("[bench] config: batched form")
    b = serve.batch_bench(log=log)
    out["batched"] = {k: b[k] for k in ("value", "unit", "batched_s", "tune", "tile", "autotune",
                                       "per_problem_loop_s", "per_problem_loop_GLUPs", "speedup_vs_loop", "config")}
    out["batched"]["hbm_frac"] = round(b["value"] * batch_bytes_per_lup() / HBM_PEAK_GBPS, 4)
    log("[bench] config: served form")
    sv = serve.serve_bench(count=args.requests, load=args.load, log=log)
    out["served"] = {k: sv[k] for k in ("value", "unit", "pool", "serial_plain", "p99_vs_serial", "mix_vs_alone",
                                       "config")}
    return out


def batch_bytes_per_lup():
    """Algorithmic bytes per cell update of the batched workload (interior read
    and write plus the Dirichlet halo reads, weighted by sweeps)."""
    from paper_2202_11819_amd import workloads as W
    lups = byts = 0
    for s in W.batch():
        nx, ny, nz = s.n
        c = nx * ny * nz
        lups += c * s.iters
        byts += s.iters * (16 * c + 16 * (ny * nz + nx * nz + nx * ny))
    return byts / lups


def modes_side(spec):
    """ms per sweep of the overdecomposed grid in the unfused modes (per block
    and per phase), fused and graph; and whether the graph run equals the
    undivided grid's bit for bit after the full sweep count."""
    import torch
    from paper_2202_11819_amd import api
    n, sweeps = spec.n, spec.iters
    cells = n[0] * n[1] * n[2]
    res = {"workload": f"{n[0]}^3 as {spec.nblk[0]}x{spec.nblk[1]}x{spec.nblk[2]} blocks", "ms_per_sweep": {}}
    for mode, iters in (("unfused_block", 6), ("unfused_phase", 100), ("fused", sweeps), ("graph", sweeps)):
        with api.Solver(n, nblk=spec.nblk, seed=spec.seed) as s:
            s.run(2, mode=mode)
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(s.stream)
            s.run(iters, mode=mode)
            e1.record(s.stream)
            e1.synchronize()
            ms = e0.elapsed_time(e1) / iters
            res["ms_per_sweep"][mode] = round(ms, 4)
            res.setdefault("GLUPs", {})[mode] = round(cells / ms / 1e6, 2)
    with api.Solver(n, nblk=spec.nblk, seed=spec.seed) as a, api.Solver(n, seed=spec.seed) as b:
        a.run(sweeps, mode="graph")
        b.run(sweeps, mode="graph")
        ua, ub = a.get_interior_device(), b.get_interior_device()
        res["graph_equals_undivided_bitwise"] = bool(torch.equal(ua.view(torch.int64), ub.view(torch.int64)))
        del ua, ub
    torch.cuda.empty_cache()
    return res


def bench_modes(args):
    """The same grid in every mode: per-block streams under each fusion strategy, the
    host-staged exchange with and without overlap, per-phase, fused and graph."""
    import torch
    from paper_2202_11819_amd import api
    from paper_2202_11819_amd import workloads as W

    spec = W.overdecomposed(nb=args.blocks, edge=args.edge, iters=args.sweeps)
    n = spec.n
    cells = n[0] * n[1] * n[2]
    for mode, iters in [("unfused_block", 10), ("unfused_block+graph", 10), ("block_a", 10), ("block_b", 10),
                        ("block_c", 20), ("block_c+graph", 20), ("host_staged", 10), ("host_overlap", 10),
                        ("unfused_phase", 100), ("fused", args.sweeps), ("graph", args.sweeps)]:
        s2 = api.Solver(n, nblk=spec.nblk, seed=spec.seed)
        s2.run(2, mode=mode)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        s2.run(iters, mode=mode)
        e1.record()
        e1.synchronize()
        ms = e0.elapsed_time(e1)
        out = {"metric": "FP64 Jacobi3D GLUP/s by execution mode", "value": round(cells * iters / ms / 1e6, 3),
               "unit": "GLUP/s", "mode": mode, "sweeps": iters, "ms_per_sweep": round(ms / iters, 4),
               "config": {"workload": f"{n[0]}^3 as {spec.nblk} blocks"}}
        print(json.dumps(out), flush=True)
        s2.close()
        torch.cuda.empty_cache()


def sweep_records(iters=500):
    """1024^3 at several decompositions: GLUP/s and algorithmic GB/s vs block count."""
    import torch
    from paper_2202_11819_amd import api, j3d
    from paper_2202_11819_amd import workloads as W

    recs = []
    for label, spec in W.block_sweep(iters=iters):
        n = spec.n
        cells = n[0] * n[1] * n[2]
        s = api.Solver(n, nblk=spec.nblk, split=spec.split, seed=spec.seed)
        s.run(10, mode="graph")
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(s.stream)
        s.run(spec.iters, mode="graph")
        e1.record(s.stream)
        e1.synchronize()
        ms = e0.elapsed_time(e1)
        per = sweep_bytes(s.problem)
        gbps = per * spec.iters / (ms * 1e-3) / 1e9
        nblocks = spec.nblk[0] * spec.nblk[1] * spec.nblk[2]
        recs.append({"workload": label, "blocks": nblocks, "value": round(cells * spec.iters / ms / 1e6, 3),
                     "unit": "GLUP/s", "GBps": round(gbps, 1), "hbm_frac": round(gbps / HBM_PEAK_GBPS, 4),
                     "B_per_LUP": round(per / cells, 3), "sweeps": spec.iters,
                     "ms_per_sweep": round(ms / spec.iters, 4), "tune": list(s.get_tune()),
                     "tile": list(j3d.variants()[s.get_tune()[0]])})
        s.close()
        torch.cuda.empty_cache()
    return recs


def bench_sweep(args):
    for r in sweep_records(iters=args.sweep_iters):
        r["metric"] = "FP64 Jacobi3D GLUP/s vs decomposition"
        print(json.dumps(r), flush=True)
    if not args.no_copy:  # the copy kernel of known size also calibrates counter runs of this workload
        print(json.dumps({"metric": "streaming copy, 2 GiB", "copy_GBps": round(copy_bandwidth(), 1)}), flush=True)


def bench_odf(args):
    """Fusion strategies and graphs vs overdecomposition (the shape of Fig. 7 and 8 on one GPU).

    A fixed grid is split into 1, 8, 64 and 512 blocks; every block runs its
    own stream of GPU operations under no fusion, strategy A, B or C, each
    launched directly or replayed from HIP graphs; the all-block fused sweep
    is the reference.  Time per iteration shows where launches dominate."""
    import torch
    from paper_2202_11819_amd import api

    edge = args.odf_edge
    n = (edge,) * 3
    cells = edge ** 3
    modes = ["unfused_block", "block_a", "block_b", "block_c", "host_staged", "host_overlap", "fused"]
    for nb in (1, 2, 4, 8):
        with api.Solver(n, nblk=(nb,) * 3, seed=1) as s:
            for m in modes:
                for cap in (False, True):
                    mode = m + ("+graph" if cap else "")
                    sweeps = args.odf_sweeps
                    s.run(2, mode=mode)  # warm-up, captures the graphs
                    torch.cuda.synchronize()
                    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                    w0 = time.perf_counter()
                    e0.record()
                    s.run(sweeps, mode=mode)
                    e1.record()
                    e1.synchronize()
                    wall = time.perf_counter() - w0
                    ms = e0.elapsed_time(e1) / sweeps
                    print(json.dumps({"metric": "time per iteration vs overdecomposition", "grid": list(n),
                                      "blocks": nb ** 3, "block_edge": edge // nb, "mode": mode,
                                      "ms_per_iter": round(ms, 4), "host_ms_per_iter": round(1e3 * wall / sweeps, 4),
                                      "GLUPs": round(cells / ms / 1e6, 2), "sweeps": sweeps}), flush=True)
        torch.cuda.empty_cache()


def bench_hostex(args):
    """Host-staged exchange with and without overlap (Fig. 1's computation-communication
    overlap) on 1024^3 at 2^3 and 4^3 blocks, beside the fused device-resident sweep."""
    import torch
    from paper_2202_11819_amd import api

    n = (1024,) * 3
    for nb in (2, 4):
        with api.Solver(n, nblk=(nb,) * 3, seed=1) as s:
            for mode in ("fused", "host_staged", "host_overlap", "host_staged+graph", "host_overlap+graph"):
                s.run(2, mode=mode)
                torch.cuda.synchronize()
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                e0.record()
                s.run(args.odf_sweeps, mode=mode)
                e1.record()
                e1.synchronize()
                ms = e0.elapsed_time(e1) / args.odf_sweeps
                print(json.dumps({"metric": "time per iteration, host-staged exchange", "grid": list(n),
                                  "blocks": nb ** 3, "mode": mode, "ms_per_iter": round(ms, 4),
                                  "GLUPs": round(1024 ** 3 / ms / 1e6, 2), "sweeps": args.odf_sweeps}), flush=True)
        torch.cuda.empty_cache()


def bench_twostep(args):
    """Two sweeps per launch against one, on the same grid left undivided (--edge, --sweeps)."""
    import torch
    from paper_2202_11819_amd import api

    n = (args.edge,) * 3
    cells = args.edge ** 3
    sweeps = args.sweeps - args.sweeps % 2
    with api.Solver(n, seed=1) as s:
        u0 = s.get_interior_device()
        for mode in ("graph", "two_sweep"):
            s.set_interior(u0)
            s.run(10, mode=mode)
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            s.run(sweeps, mode=mode)
            e1.record()
            e1.synchronize()
            ms = e0.elapsed_time(e1)
            per_launch = 2 if mode == "two_sweep" else 1
            launches = sweeps // per_launch
            # algorithmic bytes per launch: each cell read and written once, plus the boundary layer read
            nbytes = 16 * cells + 16 * 3 * args.edge ** 2
            gbps = nbytes * launches / (ms * 1e-3) / 1e9
            print(json.dumps({"metric": "FP64 Jacobi3D GLUP/s, one vs two sweeps per launch", "grid": list(n),
                              "blocks": [1, 1, 1], "mode": mode, "sweeps": sweeps,
                              "value": round(cells * sweeps / ms / 1e6, 2), "unit": "GLUP/s",
                              "ms_per_sweep": round(ms / sweeps, 4), "sweeps_per_launch": per_launch,
                              "launch_ms": round(ms / launches, 4), "bytes_per_launch": nbytes,
                              "GBps": round(gbps, 1), "hbm_frac": round(gbps / HBM_PEAK_GBPS, 4)}), flush=True)
        del u0
    torch.cuda.empty_cache()


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="overdecomposed",
                    choices=["overdecomposed", "modes", "sweep", "batch", "serve", "odf", "hostex", "twostep"])
    ap.add_argument("--mode", default="graph", choices=["graph", "fused", "unfused_phase", "unfused_block"])
    ap.add_argument("--edge", type=int, default=512)
    ap.add_argument("--blocks", type=int, default=8)
    ap.add_argument("--sweeps", type=int, default=1000)
    ap.add_argument("--sweep-iters", type=int, default=500)
    ap.add_argument("--tune", default="", help="variant,zchunk,blocks_per_cu")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-copy", action="store_true")
    ap.add_argument("--headline-only", action="store_true",
                    help="default workload: only the 512^3 line (no modes, decompositions, batched or served records)")
    ap.add_argument("--batch-two-sweep", action="store_true", help="batch workload: also two sweeps per launch")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--requests", type=int, default=1100, help="serve workload: number of requests")
    ap.add_argument("--serve-dump", default="", help="serve workload: write per-request records here")
    ap.add_argument("--retune", action="store_true", help="batch workload: ignore the tuning cache")
    ap.add_argument("--batch-only", action="store_true",
                    help="batch workload: time only the batched runs (with --tune: no autotuning in the process)")
    ap.add_argument("--copy-calib", action="store_true",
                    help="also run the 2 GiB copy kernel once (counter calibration in profiled runs)")
    ap.add_argument("--load", type=float, default=0.8, help="serve workload: arrival rate / serial capacity")
    ap.add_argument("--tol", type=float, default=0.0,
                    help="serve workload: stop a request at the first residual check with r <= tol (0: never)")
    ap.add_argument("--fill-cells", type=int, default=-1, help="serve workload: pool round policy (-1: default)")
    ap.add_argument("--pool-tune", default="", help="serve workload: variant,zchunk of the pool's rounds")
    ap.add_argument("--pool-two-sweep", action="store_true", help="serve workload: two sweeps per launch in the pool")
    ap.add_argument("--serial-two-sweep", action="store_true",
                    help="serve workload: the serial baseline solves with two sweeps per launch")
    ap.add_argument("--backlog-share", type=int, default=-1,
                    help="serve workload: rounds hold at least 1/k of the running cells (-1: default)")
    ap.add_argument("--odf-edge", type=int, default=256, help="odf workload: grid edge")
    ap.add_argument("--odf-sweeps", type=int, default=20, help="odf workload: timed sweeps per mode")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py runs on one GPU only: the library has no multi-GPU path "
              "(every block of the decomposition sits on one MI355X).", file=sys.stderr)
        sys.exit(2)
    import torch
    torch.cuda.set_device(0)
    if args.workload == "overdecomposed":
        bench_overdecomposed(args)
    elif args.workload == "modes":
        bench_modes(args)
    elif args.workload == "sweep":
        bench_sweep(args)
    elif args.workload == "batch":
        from paper_2202_11819_amd import serve
        serve.bench_batch(args)
        if args.copy_calib:
            copy_bandwidth(reps=1)
    elif args.workload == "serve":
        from paper_2202_11819_amd import serve
        serve.bench_serve(args)
    elif args.workload == "odf":
        bench_odf(args)
    elif args.workload == "hostex":
        bench_hostex(args)
    elif args.workload == "twostep":
        bench_twostep(args)


if __name__ == "__main__":
    main()
