"""Host-side helpers of the served form (no GPU)."""
from paper_2202_11819_amd import serve


def test_nearest_rank_percentiles():
    v = list(range(1, 101))
    assert serve.nearest_rank(v, 50) == 50
    assert serve.nearest_rank(v, 99) == 99
    assert serve.nearest_rank(v, 100) == 100
    assert serve.nearest_rank([5.0], 99) == 5.0
    assert serve.nearest_rank([3, 1, 2], 50) == 2


def test_summary_discards_warmup():
    recs = [{"i": i, "arrival": float(i), "done": float(i) + 0.5, "latency": 0.5 if i >= 2 else 9.0,
             "cells": 10, "iters": 2} for i in range(6)]
    s = serve.summarize(recs, warmup=2)
    assert s["requests"] == 4
    assert s["p99_ms"] == 500.0 and s["p50_ms"] == 500.0
    assert abs(s["solves_per_s"] - 4 / 3.5) < 1e-3
