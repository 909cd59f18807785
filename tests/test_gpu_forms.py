"""GPU parity of the batched and served forms (through the C ABI).

Every problem of a batch and every request of the pool must reproduce the
oracle's bits and residual exactly, whatever the tile shape or schedule, and
a request must give the same bits alone and in a mix.
"""
import os

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

NTH = min(16, os.cpu_count() or 1)


@pytest.fixture(scope="module")
def env():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from oracle import oracle
    from paper_2202_11819_amd import api, j3d
    from paper_2202_11819_amd import workloads as W
    oracle.lib()
    return oracle, api, j3d, W


def say(*a):
    print(*a, flush=True)


def _mix(W, count=14, seed=3):
    rng = np.random.default_rng(seed)
    specs = []
    for i in range(count):
        n = tuple(int(v) for v in rng.integers(5, 90, 3))
        bc = tuple(float(v) for v in rng.uniform(-1, 1, 6))
        it = int(rng.integers(0, 30)) if i % 5 else (0 if i == 0 else 1)
        nblk = (1, 1, 1)
        split = None
        if i % 4 == 3 and min(n) >= 4:
            nblk = (2, 1, 2)
            split = ([n[0] // 2, n[0] - n[0] // 2], None, [1, n[2] - 1])
        specs.append(W.Spec(n=n, nblk=nblk, split=split, bc=bc, seed=9, pid=i, iters=it))
    return specs


def _problem(api, s):
    from paper_2202_11819_amd import j3d
    return j3d.Problem(s.n, s.nblk, s.split, s.bc, s.seed, s.pid)


@pytest.mark.parametrize("tune", [None, (0, 0, 0), (9, 16, 2), (8, 8, 3), (5, 0, 1)])
def test_batch_matches_oracle(env, tune):
    oracle, api, j3d, W = env
    specs = _mix(W)
    say(f"batch of {len(specs)} with tune {tune}")
    with api.Batch([_problem(api, s) for s in specs], [s.iters for s in specs], tune=tune) as b:
        res = b.run()
        for i, s in enumerate(specs):
            want, want_r, _ = oracle.jacobi(s.n, s.iters, bc=s.bc, seed=s.seed, pid=s.pid, nthreads=NTH)
            assert np.array_equal(b.get_interior(i), want), (i, s.n, s.iters)
            assert res[i] == want_r, i


def test_batch_two_sweep_matches_oracle(env):
    # two sweeps per launch over the batch: odd counts take one ordinary sweep
    # first; counts 0, 1, 2, 3 and ragged, non-cubic, tiny and z-chunked sizes
    oracle, api, j3d, W = env
    rng = np.random.default_rng(21)
    specs = []
    for i, it in enumerate([0, 1, 2, 3, 17, 40, 41, 8, 1, 29, 64, 5]):
        n = tuple(int(v) for v in rng.integers(3, 140, 3)) if i % 4 else (1 + i, 2, 70)
        bc = tuple(float(v) for v in rng.uniform(-1, 1, 6))
        specs.append(W.Spec(n=n, bc=bc, seed=9, pid=i, iters=it))
    with api.Batch([_problem(api, s) for s in specs], [s.iters for s in specs]) as b:
        res = b.run(two_sweep=True)
        for i, s in enumerate(specs):
            want, want_r, _ = oracle.jacobi(s.n, s.iters, bc=s.bc, seed=s.seed, pid=s.pid, nthreads=NTH)
            assert np.array_equal(b.get_interior(i), want), (i, s.n, s.iters)
            assert res[i] == want_r, i
        with pytest.raises(j3d.J3DError) as e:
            b.run(two_sweep=True)
        assert e.value.status == j3d.J3D_ESTATE


def test_batch_two_sweep_refuses_decomposed_problems(env):
    _, api, j3d, W = env
    specs = [W.Spec(n=(20, 20, 20), iters=4), W.Spec(n=(20, 20, 20), nblk=(2, 1, 1), iters=4, pid=1)]
    with api.Batch([_problem(api, s) for s in specs], [s.iters for s in specs]) as b:
        with pytest.raises(j3d.J3DError) as e:
            b.run(two_sweep=True)
        assert e.value.status == j3d.J3D_EINVAL
        b.run()  # the batch is untouched and still runs once


def test_batch_run_twice_is_refused(env):
    _, api, j3d, W = env
    specs = _mix(W, count=3)
    with api.Batch([_problem(api, s) for s in specs], [s.iters for s in specs]) as b:
        b.run()
        with pytest.raises(j3d.J3DError) as e:
            b.run()
        assert e.value.status == j3d.J3D_ESTATE


def test_batch_every_autotune_candidate_is_identical(env):
    _, api, j3d, W = env
    from paper_2202_11819_amd import autotune
    specs = _mix(W, count=6, seed=11)
    probs = [_problem(api, s) for s in specs]
    iters = [s.iters for s in specs]
    ref = None
    cands = autotune.candidates(probs)[::5] + autotune.refinements([0, len(j3d.variants()) - 1])[::3]
    assert len({c[1] for c in cands}) > 2 and len({c[2] for c in cands}) == 2
    for cand in cands:
        with api.Batch(probs, iters, tune=cand) as b:
            res = b.run()
            outs = [b.get_interior(i) for i in range(len(specs))]
        if ref is None:
            ref = (outs, res)
        else:
            assert all(np.array_equal(a, c) for a, c in zip(outs, ref[0])), cand
            assert np.array_equal(res, ref[1]), cand


def _requests(W, count=12, seed=4, spread=0.02):
    rng = np.random.default_rng(seed)
    out = []
    t = 0.0
    for i in range(count):
        t += float(rng.exponential(spread))
        n = tuple(int(v) for v in rng.integers(8, 100, 3))
        it = int(rng.integers(1, 160))
        out.append(W.Request(arrival=t, spec=W.Spec(n=n, seed=5, pid=i, iters=it)))
    return out


def _flat_variant(j3d):
    return [i for i, v in enumerate(j3d.variants()) if v[0] == 0][0]


@pytest.mark.parametrize("tune", [None, "flat", (8, 16), "two_sweep"])
def test_pool_requests_match_oracle_and_solo_runs(env, tune):
    oracle, api, j3d, W = env
    from paper_2202_11819_amd import serve
    two = tune == "two_sweep"
    if two:
        tune = None
    if tune == "flat":
        tune = (_flat_variant(j3d), 64)
    trace = _requests(W)
    recs, rounds = serve.serve_pool(trace, budget_bytes=2 << 30, max_slots=8, round_sweeps=50,
                                    check_every=50, keep_results=True, tune=tune, two_sweep=two)
    assert rounds > 1
    for r, req in zip(recs, trace):
        s = req.spec
        want, want_r, done = oracle.jacobi(s.n, s.iters, seed=s.seed, pid=s.pid, check_every=50, nthreads=NTH)
        assert r["iters"] == done == s.iters
        assert np.array_equal(r["u"], want), r["i"]
        assert r["residual"] == want_r, r["i"]
    # alone in a pool of its own: the same bits
    for req in trace[:4]:
        alone, _ = serve.serve_pool([W.Request(arrival=0.0, spec=req.spec)], budget_bytes=1 << 30,
                                    max_slots=1, keep_results=True, tune=tune, two_sweep=two)
        mixed = recs[trace.index(req)]
        assert np.array_equal(alone[0]["u"], mixed["u"]) and alone[0]["residual"] == mixed["residual"]


@pytest.mark.parametrize("two", [False, True])
def test_pool_early_exit_matches_checked_oracle(env, two):
    oracle, api, j3d, W = env
    n = (30, 26, 22)
    # tolerance reached after some check point
    _, r40, _ = oracle.jacobi(n, 40, seed=6)
    tol = r40
    want, want_r, done = oracle.jacobi(n, 500, seed=6, tol=tol, check_every=10)
    assert done < 500
    with api.Pool(1 << 30, max_slots=4) as pool:
        pool.set_two_sweep(two)
        slot = pool.try_admit(j3d.Problem(n, seed=6), 500, tol=tol, check_every=10)
        finished = []
        while not finished:
            got, busy = pool.poll()
            finished += got
            if not busy and not finished:
                pool.step(7)  # rounds that do not line up with the check points
        u, r, it = pool.result(slot)
        assert it == done and r == want_r
        assert np.array_equal(u, want)
        pool.release(slot)


def test_serial_checked_solves_match_pool_and_oracle(env):
    # The served benchmark's serial baseline with a tolerance: pieces of 50
    # sweeps with a residual read after each, stopping at the first r <= tol.
    # It must stop where the pool and the oracle's checked run stop.
    oracle, api, j3d, W = env
    from paper_2202_11819_amd import serve
    specs = [W.Spec(n=(30, 26, 22), seed=6, pid=0, iters=500), W.Spec(n=(17, 40, 9), seed=6, pid=1, iters=130),
             W.Spec(n=(24, 24, 24), seed=6, pid=2, iters=75)]
    _, tol, _ = oracle.jacobi(specs[0].n, 120, seed=6, pid=0)
    trace = [W.Request(arrival=0.0, spec=s) for s in specs]
    srecs = serve.serve_serial(trace, keep_results=True, tol=tol, check_every=50)
    precs, _ = serve.serve_pool(trace, budget_bytes=1 << 30, max_slots=4, keep_results=True, tol=tol,
                                check_every=50)
    stopped = 0
    for s, a, b in zip(specs, srecs, precs):
        want, want_r, done = oracle.jacobi(s.n, s.iters, seed=s.seed, pid=s.pid, tol=tol, check_every=50,
                                           nthreads=NTH)
        stopped += done < s.iters
        assert a["iters"] == b["iters"] == done, s
        assert a["residual"] == b["residual"] == want_r, s
        assert np.array_equal(a["u"], want) and np.array_equal(b["u"], want), s
    assert stopped >= 1


def test_pool_tune_only_while_empty(env):
    _, api, j3d, _ = env
    with api.Pool(1 << 30, max_slots=2) as pool:
        pool.set_tune(_flat_variant(j3d), 64)
        slot = pool.try_admit(j3d.Problem((20, 12, 9), seed=1), 3)
        with pytest.raises(j3d.J3DError) as e:
            pool.set_tune(3, 32)
        assert e.value.status == j3d.J3D_ESTATE
        with pytest.raises(j3d.J3DError) as e:
            pool.set_two_sweep(True)
        assert e.value.status == j3d.J3D_ESTATE
        while True:
            done, busy = pool.poll()
            if slot in done:
                break
            if not busy:
                pool.step(50)
        pool.release(slot)
        pool.set_tune(3, 32)
        for bad in [(-1, 32, 0), (1 << 20, 0, 0), (1 << 20, 4, -1)]:
            with pytest.raises(j3d.J3DError) as e:
                pool.set_policy(*bad)
            assert e.value.status == j3d.J3D_EINVAL
        pool.set_policy(1 << 22, 8, 4)
        for bad in [(len(j3d.variants()), 32), (3, 0)]:
            with pytest.raises(j3d.J3DError) as e:
                pool.set_tune(*bad)
            assert e.value.status == j3d.J3D_EINVAL


def test_pool_admission_limits_and_errors(env):
    _, api, j3d, W = env
    small = j3d.Problem((32, 32, 32))
    need = j3d.j3d_pool_request_bytes(small)
    with api.Pool(2 * need + need // 2, max_slots=3) as pool:
        a = pool.try_admit(small, 10)
        b = pool.try_admit(small, 10)
        assert a is not None and b is not None
        assert pool.try_admit(small, 10) is None          # budget exhausted
        used, nbytes = pool.usage()
        assert used == 2 and nbytes == 2 * need
        pool.release(a)
        c = pool.try_admit(small, 10)                      # freed bytes are reused
        assert c is not None
        with pytest.raises(j3d.J3DError) as e:
            j3d.j3d_pool_result(pool.h, b)                  # not finished yet
        assert e.value.status == j3d.J3D_ESTATE
        pool.release(b)
        pool.release(c)
        with pytest.raises(j3d.J3DError) as e:
            pool.release(c)                                # double release
        assert e.value.status == j3d.J3D_ESTATE
        with pytest.raises(j3d.J3DError) as e:
            j3d.j3d_pool_admit(pool.h, j3d.Problem((64, 64, 64), (2, 1, 1)), 5, 0.0, 0, 1 << 20)
        assert e.value.status == j3d.J3D_EINVAL
    with api.Pool(1 << 28, max_slots=1) as pool:
        assert pool.try_admit(small, 5) is not None
        st, _ = j3d.j3d_pool_try_admit(pool.h, small, 5, 0.0, 0, pool.results[0][0].data_ptr())
        assert st == j3d.J3D_EBUSY


def test_pool_fetch_through_the_c_abi_matches_oracle(env):
    # j3d_pool_fetch copies a finished request's interior from the device,
    # whether the request was admitted without a host buffer (result kept on
    # the device) or with one (copied asynchronously at the finish)
    import ctypes
    oracle, api, j3d, W = env
    L = j3d._lib
    specs = [((37, 21, 13), 41, 0.0, 10), ((16, 40, 9), 23, 0.0, 0), ((30, 26, 22), 500, None, 10)]
    _, tol, _ = oracle.jacobi(specs[2][0], 60, seed=4, pid=2)
    with api.Pool(1 << 29, max_slots=4) as pool:
        slots, hosts = [], []
        for i, (n, it, t, ce) in enumerate(specs):
            p = j3d.Problem(n, seed=4, pid=i, bc=(0.25, -0.5, 1.0, 0.0, -1.0, 0.5))
            host = np.zeros(n[0] * n[1] * n[2]) if i == 1 else None
            hosts.append(host)
            s = ctypes.c_int32(-1)
            st = L.j3d_pool_admit(pool.h, ctypes.byref(p.c), it, tol if t is None else t, ce,
                                  host.ctypes.data if host is not None else None, ctypes.byref(s))
            assert st == j3d.J3D_OK
            slots.append(s.value)
        # not finished yet: ESTATE, nothing written
        r, k = ctypes.c_double(-1.0), ctypes.c_int64(-1)
        assert L.j3d_pool_fetch(pool.h, slots[0], None, ctypes.byref(r), ctypes.byref(k)) == j3d.J3D_ESTATE
        assert r.value == -1.0 and k.value == -1
        assert L.j3d_pool_fetch(pool.h, 4, None, None, None) == j3d.J3D_EINVAL
        done = set()
        while len(done) < len(slots):
            got, busy = pool.poll()
            done.update(got)
            if not busy and len(done) < len(slots):
                pool.step(50)
        for i, (n, it, t, ce) in enumerate(specs):
            want, want_r, want_k = oracle.jacobi(n, it, bc=(0.25, -0.5, 1.0, 0.0, -1.0, 0.5), seed=4, pid=i,
                                                 tol=tol if t is None else t, check_every=ce, nthreads=NTH)
            out = np.full((n[2], n[1], n[0]), np.nan)
            assert L.j3d_pool_fetch(pool.h, slots[i], out.ctypes.data, ctypes.byref(r), ctypes.byref(k)) == 0
            say(f"fetched slot {slots[i]} {n}: {k.value} sweeps, residual {r.value!r}")
            assert np.array_equal(out, want), i
            assert r.value == want_r and k.value == want_k, i
            if hosts[i] is not None:
                assert np.array_equal(hosts[i].reshape(n[2], n[1], n[0]), want)
            pool.release(slots[i])
        assert specs[2][1] > want_k  # the third request stopped early at its tolerance
        assert L.j3d_pool_fetch(pool.h, slots[0], None, None, None) == j3d.J3D_ESTATE  # released


def test_pool_zero_iterations_returns_initial_grid(env):
    oracle, api, j3d, W = env
    with api.Pool(1 << 28, max_slots=2) as pool:
        slot = pool.try_admit(j3d.Problem((17, 9, 5), seed=3, pid=2), 0)
        import time
        got = []
        t0 = time.time()
        while not got and time.time() - t0 < 20:
            g, busy = pool.poll()
            got += g
        assert got == [slot]
        u, r, it = pool.result(slot)
        assert it == 0 and r == 0.0
        assert np.array_equal(u, oracle.init_interior((17, 9, 5), 3, 2))


# ---- the batched and served workloads at their own sizes -----------------------

@pytest.mark.slow
def test_batch_two_sweep_full_workload_matches_oracle(env):
    # all 256 problems of the batched benchmark, two sweeps per launch
    oracle, api, j3d, W = env
    specs = W.batch()
    with api.Batch([_problem(api, s) for s in specs], [s.iters for s in specs]) as b:
        res = b.run(two_sweep=True)
        for i, s in enumerate(specs):
            want, want_r, _ = oracle.jacobi(s.n, s.iters, bc=s.bc, seed=s.seed, pid=s.pid, nthreads=NTH)
            assert res[i] == want_r, i
            assert np.array_equal(b.get_interior(i), want), i


@pytest.mark.slow
def test_batch_full_workload_matches_oracle(env):
    # all 256 problems of the batched benchmark (sizes 32..256 per axis,
    # 100..1000 sweeps), default tile, against the oracle problem by problem
    oracle, api, j3d, W = env
    specs = W.batch()
    with api.Batch([_problem(api, s) for s in specs], [s.iters for s in specs]) as b:
        res = b.run()
        for i, s in enumerate(specs):
            want, want_r, _ = oracle.jacobi(s.n, s.iters, bc=s.bc, seed=s.seed, pid=s.pid, nthreads=NTH)
            assert res[i] == want_r, i
            assert np.array_equal(b.get_interior(i), want), i


@pytest.mark.slow
@pytest.mark.parametrize("two", [False, True])
def test_pool_served_sizes_sample_matches_oracle(env, two):
    # a seeded sample of 32 requests of the served benchmark's mix (32..384
    # per axis, 50..2000 sweeps, residual every 50) plus its smallest and its
    # largest request, all admitted together, against the oracle's checked run
    oracle, api, j3d, W = env
    from paper_2202_11819_amd import serve
    trace = W.serve_trace(count=1100, rate=1.0)
    rng = np.random.default_rng(11)
    pick = sorted(set(rng.choice(len(trace), 32, replace=False).tolist()))
    cells = [int(np.prod(r.spec.n)) for r in trace]
    pick += [int(np.argmin(cells)), int(np.argmax(cells))]
    reqs = [W.Request(arrival=0.0, spec=trace[i].spec) for i in pick]
    recs, _ = serve.serve_pool(reqs, budget_bytes=40 << 30, max_slots=64, keep_results=True, two_sweep=two)
    for rec, req in zip(recs, reqs):
        s = req.spec
        want, want_r, done = oracle.jacobi(s.n, s.iters, bc=s.bc, seed=s.seed, pid=s.pid, check_every=50,
                                           nthreads=NTH)
        assert rec["iters"] == done == s.iters
        assert rec["residual"] == want_r, s.n
        assert np.array_equal(rec["u"], want), s.n

