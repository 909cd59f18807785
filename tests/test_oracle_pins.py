"""Pins of the CPU oracle against facts fixed by the paper and by mathematics.

Every test here runs on the CPU.  None of them re-types the oracle's formula
and compares it with itself: each checks a consequence that a wrong oracle
(a dropped or doubled neighbour, a wrong weight, a transposed axis, a wrong
sign, an off-by-one sweep count, flushed denormals, a wrong generator) would
violate.

Passages: Jacobi3D is the Jacobi iterative method on a 3-D grid with halo
exchange in six directions per iteration and two buffers that swap
(Sec. II-A, Fig. 1, Fig. 3, Sec. III-C).  The stencil weights, the boundary,
the initial condition and the residual are readings the paper leaves open;
they are fixed in the oracle's header.
"""
import math
import os
from fractions import Fraction

import numpy as np
import pytest

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
EPS = 2.0 ** -53


def _golden_ints(name):
    vals = []
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.strip()
            if line and not line.startswith("#"):
                vals.append(int(line))
    return vals


# ---- the generator ------------------------------------------------------------

def test_splitmix64_published_vector(oracle_mod):
    want = _golden_ints("splitmix64_seed1234567.txt")
    got = [int(v) for v in oracle_mod.splitmix64_seq(1234567, len(want))]
    assert got == want


def test_init_is_stream_and_skip_ahead_agrees(oracle_mod):
    n = (7, 5, 3)
    for seed, pid in [(1, 0), (1, 3), (2**63 + 5, 17)]:
        u = oracle_mod.init_interior(n, seed, pid)
        # the interior is the (pid+1)-th output's stream, in x-fastest order
        s0 = int(oracle_mod.splitmix64_seq(seed, pid + 1)[-1])
        stream = oracle_mod.splitmix64_seq(s0, u.size)
        want = (stream >> np.uint64(11)).astype(np.float64) * 2.0 ** -53
        assert np.array_equal(u.reshape(-1), want)
        assert u.min() >= 0.0 and u.max() < 1.0
        for (i, j, k) in [(0, 0, 0), (6, 4, 2), (3, 1, 2)]:
            assert oracle_mod.init_cell(n, seed, pid, i, j, k) == u[k, j, i]


def test_init_streams_differ_per_problem(oracle_mod):
    a = oracle_mod.init_interior((4, 4, 4), 1, 0)
    b = oracle_mod.init_interior((4, 4, 4), 1, 1)
    assert not np.array_equal(a, b)
    # mean of many U[0,1) draws
    u = oracle_mod.init_interior((64, 64, 16), 7, 0)
    assert abs(u.mean() - 0.5) < 0.01


# ---- exact fixed points ---------------------------------------------------------

def _linear(n, coef):
    nx, ny, nz = n
    a, b, c, d = coef
    i = np.arange(0, nx + 2, dtype=np.float64)
    j = np.arange(0, ny + 2, dtype=np.float64)
    k = np.arange(0, nz + 2, dtype=np.float64)
    return a + b * i[None, None, :] + c * j[None, :, None] + d * k[:, None, None]


def _faces_of(full, n):
    """Per-cell Dirichlet faces of a ghosted field, in the oracle's layouts."""
    nx, ny, nz = n
    return [full[1:nz + 1, 1:ny + 1, 0], full[1:nz + 1, 1:ny + 1, nx + 1],
            full[1:nz + 1, 0, 1:nx + 1], full[1:nz + 1, ny + 1, 1:nx + 1],
            full[0, 1:ny + 1, 1:nx + 1], full[nz + 1, 1:ny + 1, 1:nx + 1]]


@pytest.mark.parametrize("n,coef", [((9, 6, 4), (0.5, 0.25, -0.125, 1.0)),
                                    ((5, 11, 7), (-3.0, 2.0, 0.5, -0.75)),
                                    ((1, 1, 1), (1.0, 0.5, 0.25, 0.125)),
                                    ((12, 1, 3), (2.0 ** 20, -8.0, 2.0 ** -6, 3.0))])
def test_linear_field_is_exact_fixed_point(oracle_mod, n, coef):
    # A field linear in (i, j, k) is reproduced exactly by the centre-inclusive
    # 7-point mean when the 7-term sum is exact, because fl(1/7) = (1/7)(1-2^-54)
    # and 7u*fl(1/7) rounds back to u.  Every neighbour must come from the right
    # axis with the right sign, or the field changes.
    nx, ny, nz = n
    full = _linear(n, coef)
    u0 = full[1:nz + 1, 1:ny + 1, 1:nx + 1]
    out, r, done = oracle_mod.jacobi(n, 25, u0=u0, faces=_faces_of(full, n))
    assert done == 25
    assert np.array_equal(out, u0)
    assert r == 0.0


def test_dyadic_constant_with_equal_faces(oracle_mod):
    out, r, _ = oracle_mod.jacobi((6, 5, 4), 30, bc=(0.375,) * 6, u0=np.full((4, 5, 6), 0.375))
    assert np.all(out == 0.375) and r == 0.0


def test_weight_is_one_seventh_exactly_once():
    w = 1.0 / 7.0
    assert Fraction(w) == Fraction(1, 7) * (1 - Fraction(1, 2 ** 54))


# ---- closed forms ---------------------------------------------------------------

def _lambda(n, modes):
    return (1.0 + sum(2.0 * math.cos(p * math.pi / (m + 1)) for p, m in zip(modes, n))) / 7.0


@pytest.mark.parametrize("n,modes,t", [((13, 9, 7), (1, 2, 1), 20),
                                       ((6, 10, 15), (3, 1, 2), 8),
                                       ((20, 20, 20), (1, 1, 1), 100)])
def test_eigenmode_decays_by_lambda(oracle_mod, n, modes, t):
    # With zero Dirichlet faces, a product of sines is an eigenvector of the
    # centre-inclusive 7-point mean with eigenvalue
    # (1 + 2cos(p pi/(nx+1)) + 2cos(q pi/(ny+1)) + 2cos(r pi/(nz+1))) / 7.
    nx, ny, nz = n
    p, q, r = modes
    i = np.arange(1, nx + 1)
    j = np.arange(1, ny + 1)
    k = np.arange(1, nz + 1)
    u0 = (np.sin(r * np.pi * k / (nz + 1))[:, None, None]
          * np.sin(q * np.pi * j / (ny + 1))[None, :, None]
          * np.sin(p * np.pi * i / (nx + 1))[None, None, :])
    out, _, _ = oracle_mod.jacobi(n, t, u0=u0)
    lam = _lambda(n, modes)
    lam_t = float(Fraction(lam) ** t)
    m = np.abs(u0).max()
    # rounding per sweep <= 5.4 M eps (non-expansive map), initial and
    # eigenvalue evaluation errors <= (4 + 3t) M eps; bound generously
    tol = (16 * t + 16) * EPS * m
    assert np.abs(out - lam_t * u0).max() <= tol
    assert abs(lam_t) * m > 1e6 * tol  # the check is discriminating


def test_single_cell_closed_form(oracle_mod):
    # 1x1x1 grid: u_{t+1} = (u_t + sum(bc)) / 7; with bc = 1 and u0 = 0 this is
    # 1 - 7^-t.  Rounding errors contract by 1/7 per sweep.
    for t in [1, 2, 3, 5, 10, 40]:
        out, r, _ = oracle_mod.jacobi((1, 1, 1), t, bc=(1.0,) * 6, u0=np.zeros((1, 1, 1)))
        exact = 1 - Fraction(1, 7 ** t)
        assert abs(Fraction(float(out[0, 0, 0])) - exact) <= 4 * Fraction(2) ** -53
        assert r > 0.0 or t > 20


def test_single_cell_reaches_subnormals(oracle_mod):
    # bc = 0, u0 = 1: u_t = (1/7)^t up to rounding; t = 380 lies in the
    # subnormal range (below 2^-1022), so flushing denormals would give 0.
    t = 380
    out, _, _ = oracle_mod.jacobi((1, 1, 1), t, bc=(0.0,) * 6, u0=np.ones((1, 1, 1)))
    v = float(out[0, 0, 0])
    assert 0.0 < v < 2.0 ** -1022
    exact = Fraction(1, 7 ** t)
    err = abs(Fraction(v) - exact)
    assert err <= Fraction(2) ** -1074 + t * Fraction(2) ** -52 * exact


# ---- exact rational iterate and maximum principle -----------------------------

def _exact_iterate(n, bc, u0, t):
    nx, ny, nz = n
    g = [[[None] * (nx + 2) for _ in range(ny + 2)] for _ in range(nz + 2)]
    for k in range(nz + 2):
        for j in range(ny + 2):
            for i in range(nx + 2):
                if i == 0:
                    g[k][j][i] = Fraction(bc[0])
                elif i == nx + 1:
                    g[k][j][i] = Fraction(bc[1])
                elif j == 0:
                    g[k][j][i] = Fraction(bc[2])
                elif j == ny + 1:
                    g[k][j][i] = Fraction(bc[3])
                elif k == 0:
                    g[k][j][i] = Fraction(bc[4])
                elif k == nz + 1:
                    g[k][j][i] = Fraction(bc[5])
                else:
                    g[k][j][i] = Fraction(float(u0[k - 1, j - 1, i - 1]))
    for _ in range(t):
        h = [[row[:] for row in plane] for plane in g]
        for k in range(1, nz + 1):
            for j in range(1, ny + 1):
                for i in range(1, nx + 1):
                    h[k][j][i] = (g[k][j][i] + g[k][j][i - 1] + g[k][j][i + 1] + g[k][j - 1][i]
                                  + g[k][j + 1][i] + g[k - 1][j][i] + g[k + 1][j][i]) / 7
        g = h
    return np.array([[[float(g[k][j][i]) for i in range(1, nx + 1)] for j in range(1, ny + 1)]
                     for k in range(1, nz + 1)])


@pytest.mark.parametrize("n,t", [((3, 4, 2), 6), ((2, 2, 5), 9), ((4, 3, 3), 4)])
def test_within_rounding_bound_of_exact_rationals(oracle_mod, n, t):
    rng = np.random.default_rng(11)
    bc = rng.uniform(-1, 1, 6)
    u0 = rng.uniform(0, 1, (n[2], n[1], n[0]))
    out, _, _ = oracle_mod.jacobi(n, t, bc=bc, u0=u0)
    exact = _exact_iterate(n, bc, u0, t)
    m = max(np.abs(bc).max(), np.abs(u0).max())
    assert np.abs(out - exact).max() <= 8 * t * EPS * m


def test_maximum_principle(oracle_mod):
    rng = np.random.default_rng(5)
    n = (17, 9, 12)
    bc = rng.uniform(-1, 1, 6)
    out, _, _ = oracle_mod.jacobi(n, 37, bc=bc, seed=3)
    u0 = oracle_mod.init_interior(n, 3)
    lo = min(bc.min(), u0.min())
    hi = max(bc.max(), u0.max())
    slack = 8 * EPS * max(abs(lo), abs(hi))
    assert out.min() >= lo - slack and out.max() <= hi + slack


# ---- brute force in pure Python (IEEE binary64, no contraction) --------------

def _brute(n, bc, u0, t):
    nx, ny, nz = n
    w = 1.0 / 7.0

    def ghost(i, j, k, cur):
        if i == 0:
            return bc[0]
        if i == nx + 1:
            return bc[1]
        if j == 0:
            return bc[2]
        if j == ny + 1:
            return bc[3]
        if k == 0:
            return bc[4]
        if k == nz + 1:
            return bc[5]
        return cur[(k - 1, j - 1, i - 1)]

    cur = {(k, j, i): float(u0[k, j, i]) for k in range(nz) for j in range(ny) for i in range(nx)}
    res = 0.0
    for _ in range(t):
        nxt = {}
        res = 0.0
        for k in range(1, nz + 1):
            for j in range(1, ny + 1):
                for i in range(1, nx + 1):
                    c = cur[(k - 1, j - 1, i - 1)]
                    s = c
                    s += ghost(i - 1, j, k, cur)
                    s += ghost(i + 1, j, k, cur)
                    s += ghost(i, j - 1, k, cur)
                    s += ghost(i, j + 1, k, cur)
                    s += ghost(i, j, k - 1, cur)
                    s += ghost(i, j, k + 1, cur)
                    v = s * w
                    nxt[(k - 1, j - 1, i - 1)] = v
                    res = max(res, abs(v - c))
        cur = nxt
    out = np.array([[[cur[(k, j, i)] for i in range(nx)] for j in range(ny)] for k in range(nz)])
    return out, res


def test_brute_force_tiny_grids_bit_exact(oracle_mod):
    rng = np.random.default_rng(2024)
    for trial in range(40):
        n = tuple(int(v) for v in rng.integers(1, 6, 3))
        t = int(rng.integers(0, 21))
        bc = rng.uniform(-1, 1, 6)
        u0 = rng.uniform(0, 1, (n[2], n[1], n[0]))
        out, r, _ = oracle_mod.jacobi(n, t, bc=bc, u0=u0)
        want, want_r = _brute(n, bc, u0, t)
        assert np.array_equal(out, want), (trial, n, t)
        assert r == want_r, (trial, n, t)


# ---- residual, sweep count, threads, checked runs ---------------------------

def test_residual_is_last_sweep_change(oracle_mod):
    n = (10, 7, 9)
    bc = (0.1, -0.2, 0.3, 0.0, 1.0, -1.0)
    prev, r0, _ = oracle_mod.jacobi(n, 0, bc=bc, seed=9)
    assert r0 == 0.0
    assert np.array_equal(prev, oracle_mod.init_interior(n, 9))
    for t in [1, 2, 7]:
        cur, r, done = oracle_mod.jacobi(n, t, bc=bc, seed=9)
        before, _, _ = oracle_mod.jacobi(n, t - 1, bc=bc, seed=9)
        assert done == t
        assert r == np.abs(cur - before).max()


def test_threads_do_not_change_bits(oracle_mod):
    n = (23, 17, 29)
    a, ra, _ = oracle_mod.jacobi(n, 13, bc=(1, 0, 0.5, 0, 0, 0.25), seed=4, nthreads=1)
    b, rb, _ = oracle_mod.jacobi(n, 13, bc=(1, 0, 0.5, 0, 0, 0.25), seed=4, nthreads=4)
    assert np.array_equal(a, b) and ra == rb


def test_host_tuned_timing_build_gives_the_same_bits(oracle_mod):
    # The CPU baseline times a copy built with -O3 -march=native on the host
    # it runs on; the parity build is portable.  Contraction stays off and no
    # fast-math is set in either, so vector code must not change a bit:
    # ragged grids, per-cell faces, subnormals and several threads.
    rng = np.random.default_rng(11)
    for n, t, thr in [((23, 17, 29), 13, 1), ((64, 9, 5), 20, 4), ((1, 1, 1), 380, 1), ((33, 40, 7), 7, 3)]:
        bc = rng.uniform(-1, 1, 6)
        u0 = np.ones((1, 1, 1)) if n == (1, 1, 1) else None
        if n == (1, 1, 1):
            bc = np.zeros(6)
        a, ra, _ = oracle_mod.jacobi(n, t, bc=bc, u0=u0, seed=5, nthreads=thr)
        b, rb, _ = oracle_mod.jacobi(n, t, bc=bc, u0=u0, seed=5, nthreads=thr, native=True)
        assert a.tobytes() == b.tobytes() and np.float64(ra).tobytes() == np.float64(rb).tobytes()
    nx, ny, nz = 19, 11, 6
    faces = [rng.uniform(-1, 1, s) for s in [(nz, ny)] * 2 + [(nz, nx)] * 2 + [(ny, nx)] * 2]
    a, ra, _ = oracle_mod.jacobi((nx, ny, nz), 9, faces=faces, seed=3, nthreads=2)
    b, rb, _ = oracle_mod.jacobi((nx, ny, nz), 9, faces=faces, seed=3, nthreads=2, native=True)
    assert a.tobytes() == b.tobytes() and ra == rb
    out, _, _ = oracle_mod.jacobi((1, 1, 1), 380, u0=np.ones((1, 1, 1)), native=True)
    assert 0.0 < float(out[0, 0, 0]) < 2.0 ** -1022  # denormals kept in the tuned build too


def test_checked_run_stops_at_first_check_below_tol(oracle_mod):
    n = (12, 10, 8)
    res = {}
    for t in range(5, 41, 5):
        _, r, _ = oracle_mod.jacobi(n, t, seed=2)
        res[t] = r
    tol = res[25]
    first = min(t for t in res if res[t] <= tol)
    out, r, done = oracle_mod.jacobi(n, 40, seed=2, tol=tol, check_every=5)
    assert done == first and r == res[first]
    plain, _, _ = oracle_mod.jacobi(n, first, seed=2)
    assert np.array_equal(out, plain)
    # tol = 0: no early exit; the last sweep is always checked
    out, r, done = oracle_mod.jacobi(n, 23, seed=2, tol=0.0, check_every=5)
    _, r23, _ = oracle_mod.jacobi(n, 23, seed=2)
    assert done == 23 and r == r23


# ---- domain-of-dependence evaluation of single cells ---------------------------

def test_cell_after_matches_full_grid(oracle_mod):
    rng = np.random.default_rng(8)
    for n, t in [((9, 8, 7), 3), ((16, 5, 11), 6), ((4, 4, 4), 9), ((30, 3, 2), 5)]:
        bc = rng.uniform(-1, 1, 6)
        full, _, _ = oracle_mod.jacobi(n, t, bc=bc, seed=6, pid=2)
        for _ in range(12):
            i, j, k = (int(rng.integers(0, m)) for m in n)
            v = oracle_mod.cell_after(n, 6, 2, bc, t, i, j, k)
            assert v == full[k, j, i]
        for (i, j, k) in [(0, 0, 0), (n[0] - 1, n[1] - 1, n[2] - 1)]:
            assert oracle_mod.cell_after(n, 6, 2, bc, t, i, j, k) == full[k, j, i]


def test_rejects_bad_arguments(oracle_mod):
    with pytest.raises(ValueError):
        oracle_mod.jacobi((0, 3, 3), 1)
    with pytest.raises(ValueError):
        oracle_mod.jacobi((3, 3, 3), -1)
    with pytest.raises(ValueError):
        oracle_mod.cell_after((3, 3, 3), 1, 0, (0,) * 6, 1, 3, 0, 0)
