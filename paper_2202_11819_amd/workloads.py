"""Seeded synthetic inputs for Jacobi3D runs.

Input generators only: problem shapes, decompositions, boundary values,
iteration counts and arrival times, drawn from numpy's PCG64 with a fixed
seed.  Nothing here computes any part of the method; the same generated
inputs feed both the HIP library and the CPU oracle in the tests.

The paper's runs use synthetic grids only (Sec. IV): no dataset is involved.
Workloads:
  small          64^3, one block, zero boundary, 100 sweeps
  overdecomposed 512^3 as 8x8x8 blocks of 64^3, zero boundary, 1000 sweeps
  block sweep    1024^3 as 4^3, 8^3, 16^3 blocks and an uneven split with
                 100..160 cells per block per axis, 500 sweeps
  batch          256 problems, per-axis size log-uniform in [32, 256],
                 per-face boundary U[-1, 1], 100..1000 sweeps each
  serve          Poisson arrivals, per-axis size U{32..384}, 50..2000 sweeps
"""
from __future__ import annotations

import dataclasses

import numpy as np

SEED = 1


@dataclasses.dataclass
class Spec:
    n: tuple
    nblk: tuple = (1, 1, 1)
    split: tuple | None = None
    bc: tuple = (0.0,) * 6
    seed: int = SEED
    pid: int = 0
    iters: int = 0


def small():
    return Spec(n=(64, 64, 64), iters=100)


def overdecomposed(nb=8, edge=512, iters=1000):
    return Spec(n=(edge,) * 3, nblk=(nb,) * 3, iters=iters)


def uneven_split(n: int, lo: int, hi: int, rng: np.random.Generator):
    """Extents of p blocks along one axis, each in [lo, hi], summing to n.

    p is drawn uniformly from the feasible counts (lo*p <= n <= hi*p); every
    block starts at lo and the remaining cells go one at a time to blocks
    drawn uniformly among those still below hi.
    """
    feasible = [p for p in range(1, n + 1) if lo * p <= n <= hi * p]
    if not feasible:
        raise ValueError(f"no split of {n} into blocks of {lo}..{hi}")
    p = int(rng.choice(feasible))
    ext = [lo] * p
    rest = n - lo * p
    while rest > 0:
        open_ = [i for i in range(p) if ext[i] < hi]
        ext[int(rng.choice(open_))] += 1
        rest -= 1
    return ext


def block_sweep(edge=1024, iters=500, seed=SEED):
    """Decompositions of the 1024^3 grid: (label, Spec)."""
    out = []
    for nb in (4, 8, 16):
        out.append((f"{nb}^3 blocks of {edge // nb}^3", Spec(n=(edge,) * 3, nblk=(nb,) * 3, iters=iters)))
    rng = np.random.default_rng(seed)
    split = tuple(tuple(uneven_split(edge, 100, 160, rng)) for _ in range(3))
    nblk = tuple(len(s) for s in split)
    out.append((f"uneven {nblk[0]}x{nblk[1]}x{nblk[2]} blocks of 100..160",
                Spec(n=(edge,) * 3, nblk=nblk, split=split, iters=iters)))
    return out


def batch(count=256, seed=SEED, lo=32, hi=256, it_lo=100, it_hi=1000):
    """Independent problems of uneven, non-cubic sizes."""
    rng = np.random.default_rng([seed, 3])
    specs = []
    for i in range(count):
        n = tuple(int(min(hi, np.floor(lo * (hi / lo) ** rng.uniform()))) for _ in range(3))
        bc = tuple(float(v) for v in rng.uniform(-1.0, 1.0, 6))
        iters = int(rng.integers(it_lo, it_hi + 1))
        specs.append(Spec(n=n, bc=bc, seed=seed, pid=i, iters=iters))
    return specs


@dataclasses.dataclass
class Request:
    arrival: float   # seconds after the start of the trace
    spec: Spec


def serve_trace(count=1100, rate=10.0, seed=SEED, lo=32, hi=384, it_lo=50, it_hi=2000):
    """Poisson arrivals at `rate` per second (exponential gaps)."""
    rng = np.random.default_rng([seed, 5])
    t = 0.0
    out = []
    for i in range(count):
        t += float(rng.exponential(1.0 / rate))
        n = tuple(int(v) for v in rng.integers(lo, hi + 1, 3))
        iters = int(rng.integers(it_lo, it_hi + 1))
        out.append(Request(arrival=t, spec=Spec(n=n, seed=seed, pid=i, iters=iters)))
    return out


def rescale_arrivals(trace, rate):
    """Same requests and gap pattern at a different mean rate."""
    if not trace:
        return trace
    mean_gap = trace[-1].arrival / len(trace)
    f = (1.0 / rate) / mean_gap
    return [Request(arrival=r.arrival * f, spec=r.spec) for r in trace]


def to_problem(spec: Spec):
    """The library's problem object for a spec (imports the HIP binding)."""
    from . import j3d
    return j3d.Problem(spec.n, spec.nblk, spec.split, spec.bc, spec.seed, spec.pid)
