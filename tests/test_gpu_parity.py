"""GPU parity of the plain solver against the CPU oracle, through the C ABI.

The bar is bit-exact equality of the final interior and of the residual:
the update is the same expression in the same order on both sides, in
binary64 without contraction, so every decomposition, mode, tile shape and
schedule must reproduce the oracle's bits.  The eigenmode check at full size
uses the closed-form bound instead (no oracle run at that size).
"""
import os

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

NTH = min(16, os.cpu_count() or 1)
MODES = ("graph", "fused", "unfused_phase", "unfused_block", "block_a", "block_b", "block_c",
         "unfused_block+graph", "block_a+graph", "block_b+graph", "block_c+graph", "unfused_phase+graph",
         "host_staged", "host_overlap", "host_overlap+graph")


@pytest.fixture(scope="module")
def env():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from oracle import oracle
    from paper_2202_11819_amd import api, j3d
    oracle.lib()
    return oracle, api, j3d


def say(*a):
    print(*a, flush=True)


def check(oracle, api, n, nblk=(1, 1, 1), split=None, bc=(0.0,) * 6, seed=1, iters=10, mode="graph",
          tune=None):
    say(f"case n={n} nblk={nblk} split={'yes' if split else 'no'} iters={iters} mode={mode} tune={tune}")
    with api.Solver(n, nblk=nblk, split=split, bc=bc, seed=seed) as s:
        if tune is not None:
            s.set_tune(*tune)
        r = s.run(iters, mode=mode, residual=True)
        got = s.get_interior()
    want, want_r, _ = oracle.jacobi(n, iters, bc=bc, seed=seed, nthreads=NTH)
    assert np.array_equal(got, want), f"max |diff| {np.abs(got - want).max()}"
    assert r == want_r
    return got


def test_small_single_block_all_modes(env):
    # 64^3, one block, zero boundary, seeded U[0,1), 100 sweeps
    oracle, api, _ = env
    for mode in MODES:
        check(oracle, api, (64, 64, 64), iters=100, mode=mode)


def test_seeded_init_is_decomposition_independent(env):
    oracle, api, _ = env
    n = (37, 29, 23)
    want = oracle.init_interior(n, 5, 0)
    for nblk, split in [((1, 1, 1), None), ((3, 2, 4), ([10, 20, 7], [1, 28], [5, 5, 6, 7]))]:
        with api.Solver(n, nblk=nblk, split=split, seed=5) as s:
            assert s.run(0, residual=True) == 0.0
            assert np.array_equal(s.get_interior(), want)


def test_modes_agree_on_overdecomposed_grid(env):
    oracle, api, _ = env
    bc = (0.25, -0.5, 1.0, 0.0, -0.75, 0.5)
    for mode in MODES:
        check(oracle, api, (96, 64, 80), nblk=(3, 4, 2), bc=bc, iters=17, mode=mode, seed=3)


def test_random_decompositions(env):
    oracle, api, _ = env
    rng = np.random.default_rng(1234)
    for case in range(10):
        n = tuple(int(v) for v in rng.integers(8, 70, 3))
        nblk, split = [], []
        for a in range(3):
            nb = int(rng.integers(1, min(6, n[a]) + 1))
            cuts = np.sort(rng.choice(np.arange(1, n[a]), nb - 1, replace=False)) if nb > 1 else []
            ext = np.diff(np.concatenate([[0], cuts, [n[a]]])).astype(int).tolist()
            nblk.append(nb)
            split.append(ext)
        bc = tuple(float(v) for v in rng.uniform(-1, 1, 6))
        iters = int(rng.integers(1, 25))
        mode = MODES[case % len(MODES)]
        check(oracle, api, n, nblk=tuple(nblk), split=tuple(split), bc=bc, iters=iters, mode=mode,
              seed=int(rng.integers(1, 1000)))


def test_one_cell_thick_blocks_and_tiny_grids(env):
    oracle, api, _ = env
    check(oracle, api, (5, 4, 3), nblk=(5, 4, 3), bc=(1, 2, 3, 4, 5, 6), iters=9, mode="fused")
    check(oracle, api, (1, 1, 1), bc=(1, -1, 0.5, 0.25, 0, 2), iters=7, mode="graph")
    check(oracle, api, (1, 7, 1), nblk=(1, 7, 1), iters=5, mode="unfused_phase")
    check(oracle, api, (130, 1, 2), nblk=(2, 1, 2), split=([1, 129], None, None), iters=6, mode="fused")


def test_overlap_shell_recompute_on_thin_blocks(env):
    # the overlapped host-staged mode recomputes each block's one-cell shell;
    # blocks 1, 2 and 3 cells thick along each axis take every branch of its
    # cell enumeration
    oracle, api, _ = env
    cases = [((5, 4, 3), (5, 4, 3), None),
             ((9, 7, 8), (3, 3, 3), ([1, 2, 6], [3, 2, 2], [2, 1, 5])),
             ((12, 3, 10), (2, 1, 2), ([2, 10], None, [1, 9])),
             ((6, 11, 2), (3, 2, 1), ([2, 3, 1], [4, 7], None))]
    for n, nblk, split in cases:
        bc = (0.5, -1.0, 0.25, 2.0, -0.125, 1.0)
        for mode in ("host_overlap", "host_overlap+graph"):
            check(oracle, api, n, nblk=nblk, split=split, bc=bc, iters=9, mode=mode, seed=4)


def test_every_tile_shape_and_schedule(env):
    oracle, api, j3d = env
    n = (150, 70, 37)
    split = ([60, 90], [33, 37], [37])
    bc = (0.1, 0.2, 0.3, 0.4, 0.5, 0.6)
    want, want_r, _ = oracle.jacobi(n, 12, bc=bc, seed=9, nthreads=NTH)
    for v in range(len(j3d.variants())):
        for zchunk, bpc in [(0, 0), (5, 0), (16, 2)]:
            say(f"variant {v} zchunk {zchunk} blocks_per_cu {bpc}")
            with api.Solver(n, nblk=(2, 2, 1), split=split, bc=bc, seed=9) as s:
                s.set_tune(v, zchunk, bpc)
                r = s.run(12, mode="graph" if bpc else "fused", residual=True)
                assert np.array_equal(s.get_interior(), want), (v, zchunk, bpc)
                assert r == want_r


def test_xcd_runs_of_unequal_length(env):
    # 1216 tiles of 7 or 8 planes (32 per plane, 512-cell flattened tiles):
    # each XCD's run of tiles is cut by streamed planes, so the runs differ
    # in length (150 to 162 tiles) and the surplus workgroups of the shorter
    # ones exit; every tile must still run exactly once
    oracle, api, _ = env
    bc = (0.5, -0.25, 1.0, 0.125, -1.0, 0.75)
    for mode in ("fused", "graph", "unfused_phase"):
        check(oracle, api, (64, 256, 300), nblk=(1, 1, 2), split=(None, None, [44, 256]), bc=bc, iters=6,
              mode=mode, seed=11, tune=(33, 8, 0))


def test_unpadded_rows_and_line_shifted_tiles(env):
    # Rows are unpadded and planes start on 128-byte lines; a flattened tile of
    # whole rows whose first cell is not on a line shifts its slots.  Widths off
    # the 16-cell grid with many y-tiles per plane make every shift 0..15 occur;
    # width 1 and tiny planes cover the edge of the plane padding.
    oracle, api, j3d = env
    flat = [v for v, (tx, ty, nt) in enumerate(j3d.variants()) if tx == 0]
    bc = (0.75, -0.5, 0.25, 1.0, -1.0, 0.5)
    for n in [(17, 301, 5), (33, 97, 9), (100, 64, 7), (250, 40, 6), (1, 77, 3), (15, 15, 15), (241, 3, 4)]:
        want, want_r, _ = oracle.jacobi(n, 6, bc=bc, seed=13, nthreads=NTH)
        for v in flat:
            say(f"shape {n} variant {v}")
            with api.Solver(n, bc=bc, seed=13) as s:
                s.set_tune(v, 4, 0)
                r = s.run(6, mode="fused", residual=True)
                assert np.array_equal(s.get_interior(), want), (n, v)
                assert r == want_r, (n, v)


def test_linear_field_with_per_cell_faces_is_fixed(env):
    oracle, api, _ = env
    n = (40, 24, 18)
    nx, ny, nz = n
    a, b, c, d = 0.5, 0.25, -0.125, 2.0
    i = np.arange(nx + 2, dtype=np.float64)
    j = np.arange(ny + 2, dtype=np.float64)
    k = np.arange(nz + 2, dtype=np.float64)
    full = a + b * i[None, None, :] + c * j[None, :, None] + d * k[:, None, None]
    u0 = np.ascontiguousarray(full[1:-1, 1:-1, 1:-1])
    faces = [full[1:-1, 1:-1, 0], full[1:-1, 1:-1, -1], full[1:-1, 0, 1:-1], full[1:-1, -1, 1:-1],
             full[0, 1:-1, 1:-1], full[-1, 1:-1, 1:-1]]
    for mode in ("graph", "unfused_block"):
        with api.Solver(n, nblk=(4, 3, 2)) as s:
            s.set_interior(u0)
            for f in range(6):
                s.set_face(f, faces[f])
            r = s.run(31, mode=mode, residual=True)
            assert np.array_equal(s.get_interior(), u0)
            assert r == 0.0
    # and the oracle agrees on the same input
    out, r, _ = oracle.jacobi(n, 31, u0=u0, faces=faces)
    assert np.array_equal(out, u0) and r == 0.0


def test_per_cell_faces_match_oracle(env):
    oracle, api, _ = env
    rng = np.random.default_rng(77)
    n = (21, 17, 13)
    nx, ny, nz = n
    faces = [rng.uniform(-1, 1, (nz, ny)), rng.uniform(-1, 1, (nz, ny)), rng.uniform(-1, 1, (nz, nx)),
             rng.uniform(-1, 1, (nz, nx)), rng.uniform(-1, 1, (ny, nx)), rng.uniform(-1, 1, (ny, nx))]
    with api.Solver(n, nblk=(3, 1, 2), split=([5, 6, 10], None, [6, 7]), seed=4) as s:
        for f in range(6):
            s.set_face(f, faces[f])
        r = s.run(15, mode="graph", residual=True)
        got = s.get_interior()
    want, want_r, _ = oracle.jacobi(n, 15, seed=4, faces=faces, nthreads=NTH)
    assert np.array_equal(got, want) and r == want_r


def test_subnormals_are_kept(env):
    oracle, api, _ = env
    with api.Solver((1, 1, 1)) as s:
        s.set_interior(np.ones(1))
        s.run(380, mode="fused")
        got = s.get_interior()
    want, _, _ = oracle.jacobi((1, 1, 1), 380, u0=np.ones((1, 1, 1)))
    assert 0.0 < got[0, 0, 0] < 2.0 ** -1022
    assert np.array_equal(got, want)


def test_resume_and_mode_switch(env):
    oracle, api, _ = env
    n, nblk, bc = (48, 40, 44), (2, 2, 2), (0.5, 0, 0, 0.5, 1, 0)
    want, want_r, _ = oracle.jacobi(n, 30, bc=bc, seed=2, nthreads=NTH)
    with api.Solver(n, nblk=nblk, bc=bc, seed=2) as s:
        s.run(7, mode="unfused_block")
        s.run(5, mode="graph")
        s.run(3, mode="block_c+graph")
        s.run(3, mode="block_a")
        s.run(2, mode="host_overlap")
        s.run(3, mode="unfused_phase")
        r = s.run(7, mode="fused", residual=True)
        assert s.iters_done() == 30
        assert np.array_equal(s.get_interior(), want) and r == want_r
        # checkpoint / restart: interior + sweep count is the whole state
        snap = s.get_interior()
    with api.Solver(n, nblk=(3, 1, 4), split=([10, 20, 18], None, [11, 11, 11, 11]), bc=bc) as s2:
        s2.set_interior(snap)
        s2.run(9, mode="graph")
        more, _, _ = oracle.jacobi(n, 39, bc=bc, seed=2, nthreads=NTH)
        assert np.array_equal(s2.get_interior(), more)


def test_device_side_interior_copies(env):
    import torch
    oracle, api, _ = env
    n = (33, 35, 31)
    u = torch.rand((n[2], n[1], n[0]), dtype=torch.float64, device="cuda")
    with api.Solver(n, nblk=(3, 5, 1), split=([11, 11, 11], [7, 7, 7, 7, 7], None)) as s:
        s.set_interior(u)
        assert torch.equal(s.get_interior_device(), u)
        s.run(4, mode="graph")
        got = s.get_interior_device().cpu().numpy()
    want, _, _ = oracle.jacobi(n, 4, u0=u.cpu().numpy())
    assert np.array_equal(got, want)


def test_determinism(env):
    _, api, _ = env
    outs = []
    for _ in range(2):
        with api.Solver((128, 96, 64), nblk=(2, 3, 2), seed=11, bc=0.5) as s:
            s.set_tune(-1, 0, 3)
            r = s.run(40, mode="graph", residual=True)
            outs.append((s.get_interior(), r))
    assert np.array_equal(outs[0][0], outs[1][0]) and outs[0][1] == outs[1][1]


def test_errors_leave_state_untouched(env):
    oracle, api, j3d = env
    with api.Solver((16, 16, 16), nblk=(2, 2, 2), seed=3) as s:
        with pytest.raises(j3d.J3DError) as e:
            s.run(-1)
        assert e.value.status == j3d.J3D_EINVAL
        with pytest.raises(j3d.J3DError):
            j3d.j3d_set_tune(s.h, 999, 0, 0)
        with pytest.raises(j3d.J3DError):
            j3d.j3d_set_face(s.h, 6, 0, False)
        for bad_mode in (9, 15, 3 | 16 | 32, -1):
            with pytest.raises(j3d.J3DError) as e:
                s.run(2, mode=bad_mode)
            assert e.value.status == j3d.J3D_EINVAL
        s.run(5, mode="graph")
        want, _, _ = oracle.jacobi((16, 16, 16), 5, seed=3)
        assert np.array_equal(s.get_interior(), want)


# ---- full-size workloads (the benchmark's launch configuration) ---------------

@pytest.mark.parametrize("n, iters", [((64, 64, 64), 100), ((70, 37, 11), 9), ((130, 33, 9), 20),
                                      ((5, 3, 2), 4), ((1, 1, 1), 7), ((17, 70, 5), 1), ((200, 130, 150), 12),
                                      ((64, 48, 13), 0)])
def test_two_sweep_matches_oracle(env, n, iters):
    # two sweeps per launch on an undivided grid: ragged x tiles, y tiles of
    # unequal rows, z chunks, odd counts (a fused sweep at the end), tiny grids
    oracle, api, _ = env
    check(oracle, api, n, bc=(0.25, -0.5, 1.0, 0.0, -0.75, 0.5), seed=6, iters=iters, mode="two_sweep")


def test_two_sweep_faces_fixed_point_and_mode_mix(env):
    oracle, api, j3d = env
    # a linear field with per-cell faces stays fixed under two-sweep launches
    n = (90, 20, 18)
    i, j, k = (np.arange(v + 2, dtype=np.float64) for v in n)
    full = 0.5 + 0.25 * i[None, None, :] - 0.125 * j[None, :, None] + 2.0 * k[:, None, None]
    u0 = np.ascontiguousarray(full[1:-1, 1:-1, 1:-1])
    faces = [full[1:-1, 1:-1, 0], full[1:-1, 1:-1, -1], full[1:-1, 0, 1:-1], full[1:-1, -1, 1:-1],
             full[0, 1:-1, 1:-1], full[-1, 1:-1, 1:-1]]
    with api.Solver(n) as s:
        s.set_interior(u0)
        for f in range(6):
            s.set_face(f, faces[f])
        assert s.run(24, mode="two_sweep", residual=True) == 0.0
        assert np.array_equal(s.get_interior(), u0)
    # random per-cell faces, two-sweep runs interleaved with the other modes
    rng = np.random.default_rng(5)
    n = (77, 41, 29)
    nx, ny, nz = n
    faces = [rng.uniform(-1, 1, (nz, ny)), rng.uniform(-1, 1, (nz, ny)), rng.uniform(-1, 1, (nz, nx)),
             rng.uniform(-1, 1, (nz, nx)), rng.uniform(-1, 1, (ny, nx)), rng.uniform(-1, 1, (ny, nx))]
    want, want_r, _ = oracle.jacobi(n, 40, seed=8, faces=faces, nthreads=NTH)
    with api.Solver(n, seed=8) as s:
        for f in range(6):
            s.set_face(f, faces[f])
        s.run(5, mode="fused")
        s.run(8, mode="two_sweep")
        s.run(3, mode="graph")
        s.run(7, mode="two_sweep")
        s.run(2, mode="unfused_block")
        r = s.run(15, mode="two_sweep", residual=True)
        assert s.iters_done() == 40
        assert np.array_equal(s.get_interior(), want) and r == want_r


def test_two_sweep_refuses_decomposed_grid(env):
    oracle, api, j3d = env
    n = (32, 30, 28)
    want, _, _ = oracle.jacobi(n, 4, seed=3, nthreads=NTH)
    with api.Solver(n, nblk=(2, 1, 1), seed=3) as s:
        for mode in ("two_sweep", "two_sweep+graph"):
            with pytest.raises(j3d.J3DError) as e:
                s.run(4, mode=mode)
            assert e.value.status == j3d.J3D_EINVAL
        assert s.iters_done() == 0
        s.run(4, mode="graph")
        assert np.array_equal(s.get_interior(), want)


def test_two_sweep_graphs_replay_exactly(env):
    # graphs of 24 two-sweep launches, replayed several times with eager work
    # and host synchronisation between the replays; every stage against the oracle
    oracle, api, _ = env
    n, bc = (70, 37, 50), (0.5, -0.25, 0.0, 1.0, -1.0, 0.75)
    with api.Solver(n, bc=bc, seed=12) as s:
        done = 0
        for k, (it, mode) in enumerate([(100, "two_sweep+graph"), (3, "fused"), (97, "two_sweep+graph"),
                                        (50, "graph"), (151, "two_sweep+graph")]):
            r = s.run(it, mode=mode, residual=True)
            done += it
            want, want_r, _ = oracle.jacobi(n, done, bc=bc, seed=12, nthreads=NTH)
            assert np.array_equal(s.get_interior(), want), (k, mode, done)
            assert r == want_r, (k, mode, done)
        assert s.iters_done() == done


@pytest.mark.slow
def test_two_sweep_512_full_run_matches_oracle(env):
    # the 512^3 grid undivided, 1000 sweeps in 500 two-sweep launches
    oracle, api, _ = env
    n = (512, 512, 512)
    with api.Solver(n, seed=1) as s:
        r = s.run(1000, mode="two_sweep", residual=True)
        got = s.get_interior()
    want, want_r, _ = oracle.jacobi(n, 1000, seed=1, nthreads=NTH)
    assert r == want_r
    assert np.array_equal(got, want), f"max |diff| {np.abs(got - want).max()}"


def test_overdecomposed_512_sampled_cells(env):
    # 512^3 as 8^3 blocks of 64^3: the benchmark's grid and launch shape.  A
    # cell's value after t sweeps depends only on cells within t steps, so the
    # oracle evaluates sampled cells exactly on their domain of dependence.
    oracle, api, _ = env
    n, t = (512, 512, 512), 12
    rng = np.random.default_rng(5)
    cells = [(0, 0, 0), (511, 511, 511), (63, 64, 127), (64, 63, 128), (255, 256, 0)]
    cells += [tuple(int(v) for v in rng.integers(0, 512, 3)) for _ in range(27)]
    with api.Solver(n, nblk=(8, 8, 8), seed=1) as s:
        s.run(t, mode="graph")
        u = s.get_interior()
    for (i, j, k) in cells:
        assert u[k, j, i] == oracle.cell_after(n, 1, 0, (0.0,) * 6, t, i, j, k), (i, j, k)


def test_overdecomposed_512_full_run_equals_single_block(env):
    # 1000 sweeps: the 512-block graph run must equal the 1-block run bit for bit.
    _, api, _ = env
    n = (512, 512, 512)
    with api.Solver(n, nblk=(8, 8, 8), seed=1) as s:
        r8 = s.run(1000, mode="graph", residual=True)
        u8 = s.get_interior_device()
    with api.Solver(n, nblk=(1, 1, 1), seed=1) as s:
        r1 = s.run(1000, mode="fused", residual=True)
        u1 = s.get_interior_device()
    assert r8 == r1
    assert bool((u8 == u1).all())
    assert 0.0 < r8 < 1e-2


@pytest.mark.slow
def test_overdecomposed_512_full_run_matches_oracle(env):
    # The benchmark's whole step: 512^3 as 8^3 blocks, 1000 sweeps in graph
    # mode with the last sweep's residual, against the oracle's full run on the
    # host cores (about 15 s on 16 threads).
    oracle, api, _ = env
    n = (512, 512, 512)
    with api.Solver(n, nblk=(8, 8, 8), seed=1) as s:
        r = s.run(1000, mode="graph", residual=True)
        got = s.get_interior()
    say("oracle: 512^3 x 1000 sweeps")
    want, want_r, done = oracle.jacobi(n, 1000, seed=1, nthreads=NTH)
    assert done == 1000 and r == want_r
    assert np.array_equal(got, want), f"max |diff| {np.abs(got - want).max()}"


@pytest.mark.slow
def test_block_sweep_1024_full_runs_match_oracle(env):
    # The decomposition benchmark at its real size: 1024^3, 500 sweeps, as 4^3,
    # 8^3 and 16^3 blocks and the uneven split, each in graph mode with the
    # residual, against one oracle run of the undivided grid (about 50 s on
    # 16 host threads and 26 GB of host memory).
    oracle, api, _ = env
    from paper_2202_11819_amd import workloads as W
    cases = W.block_sweep()
    n, t = cases[0][1].n, cases[0][1].iters
    say(f"oracle: {n} x {t} sweeps")
    want, want_r, _ = oracle.jacobi(n, t, seed=cases[0][1].seed, nthreads=NTH)
    for label, spec in cases:
        assert spec.n == n and spec.iters == t
        say(label)
        with api.Solver(spec.n, nblk=spec.nblk, split=spec.split, seed=spec.seed) as s:
            r = s.run(t, mode="graph", residual=True)
            got = s.get_interior()
        assert r == want_r, label
        assert np.array_equal(got, want), label
        del got


def test_overdecomposed_512_eigenmode_bound(env):
    # Lowest sine mode with zero boundary decays by lambda per sweep.
    import math
    from fractions import Fraction

    _, api, _ = env
    n, t = (512, 512, 512), 1000
    x = np.sin(np.pi * np.arange(1, 513) / 513)
    u0 = x[:, None, None] * x[None, :, None] * x[None, None, :]
    lam = (1.0 + 6.0 * math.cos(math.pi / 513)) / 7.0
    lam_t = float(Fraction(lam) ** t)
    with api.Solver(n, nblk=(8, 8, 8)) as s:
        s.set_interior(u0)
        s.run(t, mode="graph")
        u = s.get_interior()
    err = np.abs(u - lam_t * u0).max()
    assert err <= (16 * t + 16) * 2.0 ** -53, err
    assert lam_t > 0.9


def test_uneven_1024_sampled_cells(env):
    # the uneven decomposition of the 1024^3 grid (blocks of 100..160 cells)
    oracle, api, _ = env
    from paper_2202_11819_amd import workloads as W
    label, spec = W.block_sweep()[3]
    t = 8
    rng = np.random.default_rng(6)
    cells = [(0, 0, 0), (1023, 1023, 1023)] + [tuple(int(v) for v in rng.integers(0, 1024, 3))
                                               for _ in range(20)]
    say(label)
    with api.Solver(spec.n, nblk=spec.nblk, split=spec.split, seed=spec.seed) as s:
        s.run(t, mode="graph")
        u = s.get_interior_device()
        vals = u[[c[2] for c in cells], [c[1] for c in cells], [c[0] for c in cells]].cpu().numpy()
    for v, (i, j, k) in zip(vals, cells):
        assert v == oracle.cell_after(spec.n, spec.seed, 0, (0.0,) * 6, t, i, j, k), (i, j, k)


def test_tune_roundtrip_and_default_shapes(env):
    _, api, j3d = env
    vs = j3d.variants()
    with api.Solver((512, 512, 512), nblk=(8, 8, 8), seed=1) as s:
        v, zc, bpc = s.get_tune()
        # 64-wide blocks default to flattened tiles of 512 threads through whole blocks
        assert vs[v][0] == 0 and vs[v][2] == 512 and zc == 0 and bpc == 0
        s.set_tune(3, 16, 2)
        assert s.get_tune() == (3, 16, 2)
        s.set_tune(-1, 32, 0)  # -1: the default shape with the given chunking
        assert s.get_tune()[1:] == (32, 0) and s.get_tune()[0] == v
    # the default shape for other block widths
    for n, nblk, tile in [((256, 256, 256), (2, 2, 2), (128, 16, 512)), ((320, 64, 64), (2, 1, 1), (0, 2048, 512)),
                          ((384, 64, 64), (2, 1, 1), (0, 2048, 512)), ((256, 64, 64), (1, 1, 1), (128, 32, 1024)),
                          ((300, 64, 64), (1, 1, 1), (0, 2048, 512)), ((254, 64, 64), (2, 1, 1), (0, 2048, 512))]:
        with api.Solver(n, nblk=nblk, seed=1) as s:
            assert tuple(vs[s.get_tune()[0]]) == tile, (n, nblk)
