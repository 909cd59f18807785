"""Tile-shape / schedule search for the batched form.

The batched form advances many independent problems with one launch per
sweep; the kernel shape (tile variant, z-chunk) and the schedule (one
workgroup per tile, or a persistent grid of blocks_per_cu workgroups per
compute unit taking tiles from per-XCD queues) are chosen here by timing
short batched runs of the actual problem mix on the device.  Results are
cached in a JSON file keyed by the device architecture and a size class of
the mix, so a later batch of the same class reuses the choice.
"""
from __future__ import annotations

import hashlib
import json
import math
import os
import time

import torch

from . import j3d
from .api import Batch

DEFAULT_CACHE = os.path.join(os.path.expanduser("~"), ".cache", "j3d", "tune.json")


def size_class(problems) -> str:
    """Size class of a problem mix: count, largest and median block shape (powers of two)."""
    cells = sorted(p.cells for p in problems)
    med = cells[len(cells) // 2]
    mx = max(max(p.n) for p in problems)
    return (f"count{2 ** math.ceil(math.log2(max(1, len(problems))))}"
            f"-max{2 ** math.ceil(math.log2(mx))}-med{2 ** round(math.log2(med))}")


def device_arch() -> str:
    return torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]


def candidates(problems):
    """Stage 1: every tile shape that suits the mix's widths, z-chunk 32, one
    workgroup per tile."""
    widest = max(p.n[0] for p in problems)
    return [(v, 32, 0) for v, (tx, ty, threads) in enumerate(j3d.variants()) if tx <= max(64, 2 * widest)]


def refinements(best_shapes):
    """Stage 2: the best shapes of stage 1 crossed with z-chunks and schedules."""
    out = []
    for v in best_shapes:
        for zc in (0, 16, 24, 32, 48, 64):
            for bpc in (0, 2):
                out.append((v, zc, bpc))
    return out


def time_batch(problems, iters, tune, stream=None) -> float:
    """Seconds for one batched run (after creation) of `problems` with `tune`."""
    b = Batch(problems, iters, tune=tune, stream=stream)
    try:
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        b.run(residuals=False)
        e1.record()
        e1.synchronize()
        return e0.elapsed_time(e1) * 1e-3
    finally:
        b.close()


def tune_batch(problems, iters, sample_sweeps=24, cache_path=DEFAULT_CACHE, log=None, force=False,
               report=False, keep=3):
    """Best (variant, zchunk, blocks_per_cu) for this mix; cached per (arch, size class).
    Two stages on a shortened copy of the mix: every suitable tile shape at
    z-chunk 32, then the `keep` best shapes over z-chunks and schedules.
    report=True returns (tune, candidates timed), 0 timed for a cache hit."""
    # the key names the library build and its tile table, so a cache written
    # by another build (whose variant indices may mean other shapes) is not used
    table = hashlib.sha256(repr(j3d.variants()).encode()).hexdigest()[:12]
    key = f"{device_arch()}|{j3d.j3d_version()}|{table}|batch|{size_class(problems)}"
    cache = {}
    if cache_path and os.path.exists(cache_path):
        with open(cache_path) as f:
            cache = json.load(f)
    if not force and key in cache:
        best = tuple(cache[key]["tune"])
        return (best, 0) if report else best
    # a shortened copy of the mix keeps the same tiles and the same
    # relative iteration counts
    top = max(iters) if iters else 1
    short = [max(1, round(sample_sweeps * it / top)) if it > 0 else 0 for it in iters]
    t0 = time.perf_counter()

    def run(cands):
        res = []
        for cand in cands:
            try:
                dt = time_batch(problems, short, cand)
            except j3d.J3DError:
                continue
            res.append((dt, cand))
            if log:
                log(f"[autotune] variant {cand[0]} {j3d.variants()[cand[0]]} zchunk {cand[1]} "
                    f"blocks/CU {cand[2]}: {dt * 1e3:.2f} ms")
        return sorted(res)

    stage1 = run(candidates(problems))
    shapes = [c[0] for _, c in stage1[:keep]]
    stage2 = run([c for c in refinements(shapes) if c[1] != 32 or c[2] != 0])
    results = sorted(stage1 + stage2)
    best = results[0][1]
    cache[key] = {"tune": list(best), "seconds": results[0][0], "searched": len(results),
                  "search_s": round(time.perf_counter() - t0, 2)}
    if cache_path:
        os.makedirs(os.path.dirname(cache_path), exist_ok=True)
        with open(cache_path, "w") as f:
            json.dump(cache, f, indent=1, sort_keys=True)
    return (best, len(results)) if report else best
