"""The seeded input generators produce the shapes and ranges the workloads state."""
import numpy as np

from paper_2202_11819_amd import workloads as W


def test_uneven_split_bounds_and_sum():
    rng = np.random.default_rng(0)
    for n, lo, hi in [(1024, 100, 160), (500, 10, 30), (7, 1, 7), (64, 64, 64)]:
        for _ in range(20):
            ext = W.uneven_split(n, lo, hi, rng)
            assert sum(ext) == n
            assert all(lo <= e <= hi for e in ext)
            assert lo * len(ext) <= n <= hi * len(ext)


def test_block_sweep_configs():
    cfgs = W.block_sweep()
    assert [c[1].nblk for c in cfgs[:3]] == [(4,) * 3, (8,) * 3, (16,) * 3]
    label, spec = cfgs[3]
    assert spec.n == (1024,) * 3 and spec.iters == 500
    for a in range(3):
        assert sum(spec.split[a]) == 1024
        assert 7 <= len(spec.split[a]) <= 10
        assert all(100 <= e <= 160 for e in spec.split[a])
    # deterministic
    assert W.block_sweep()[3][1].split == spec.split


def test_batch_specs():
    specs = W.batch()
    assert len(specs) == 256
    ns = np.array([s.n for s in specs])
    assert ns.min() >= 32 and ns.max() <= 256
    assert len({s.n for s in specs}) > 200                 # non-cubic, varied
    assert sum(1 for s in specs if len(set(s.n)) == 1) < 10
    its = np.array([s.iters for s in specs])
    assert its.min() >= 100 and its.max() <= 1000
    bcs = np.array([s.bc for s in specs])
    assert bcs.min() >= -1 and bcs.max() <= 1
    assert len({s.pid for s in specs}) == 256
    cells = sum(int(np.prod(s.n)) for s in specs)
    assert 1e8 < cells < 6e8


def test_serve_trace():
    tr = W.serve_trace(count=500, rate=20.0)
    t = np.array([r.arrival for r in tr])
    assert np.all(np.diff(t) > 0)
    assert abs(len(tr) / t[-1] - 20.0) < 3.0
    ns = np.array([r.spec.n for r in tr])
    assert ns.min() >= 32 and ns.max() <= 384
    its = np.array([r.spec.iters for r in tr])
    assert its.min() >= 50 and its.max() <= 2000
    tr2 = W.rescale_arrivals(tr, 40.0)
    assert abs(len(tr2) / tr2[-1].arrival - 40.0) < 1e-6
    assert [r.spec for r in tr2] == [r.spec for r in tr]
