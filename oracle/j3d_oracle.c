/*
 * j3d_oracle.c -- plain CPU oracle for the FP64 Jacobi3D sweep.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path (the HIP library
 * and its Python binding) may include, link, load or call this file.  Only
 * the tests, the smoke check and the benchmark's CPU-baseline leg use it.
 * It shares no code, header, table or constant generator with the HIP path.
 *
 * What it computes (Choi, Richards, Kale, "Improving Scalability with
 * GPU-Aware Asynchronous Tasks", arXiv 2202.11819):
 *
 *  - Jacobi3D is the Jacobi iterative method on a 3-D grid (Sec. I and
 *    Sec. II-A, Fig. 1).  Each iteration updates every cell of the block
 *    from the previous iterate after all six halo directions have arrived
 *    (Fig. 1 and Fig. 3: pack, exchange in six directions, unpack, update).
 *  - Two buffers hold the previous and the current iterate and swap roles
 *    every iteration (Sec. III-C).
 *  - The iteration count is fixed; neighbours only need halos from the same
 *    iteration, with no global synchronisation (Sec. II-A, Sec. IV-A).
 *
 * Because every block always exchanges halos of the same iteration, the
 * over-decomposed computation reaches exactly the synchronous Jacobi iterate
 * of the undivided global grid.  This oracle therefore computes that plain
 * definition on the whole grid, with no blocks and no halo buffers.
 *
 * Readings of points the paper leaves open (each is listed in the design
 * notes of the repository):
 *  - Stencil: centre-inclusive 7-point mean, u' = (c + six face neighbours)
 *    times W, W = fl(1/7), summed left to right in the fixed order
 *    c, x-, x+, y-, y+, z-, z+.  The paper names the method only.
 *  - Boundary: a 1-cell Dirichlet ghost layer that never changes, one
 *    constant per face or an optional per-cell array per face.  Edge and
 *    corner ghosts are never read by a 7-point stencil; they are set to NaN
 *    here so that any read of them would poison the result.
 *  - Initial interior: uniform [0,1) from SplitMix64 (Steele, Lea and Flood,
 *    OOPSLA 2014).  Problem `pid` of seed `s` uses the stream whose state
 *    starts at the (pid+1)-th SplitMix64 output of state s; the interior is
 *    that stream's output sequence in global x-fastest cell order, mapped to
 *    [0,1) as (h >> 11) * 2^-53.
 *  - Residual: max over the interior of |u_new - u_old| for the last sweep;
 *    0 when no sweep ran.  Checked runs evaluate it every `check_every`
 *    sweeps and at the last one, stopping early once it is <= tol (tol > 0).
 *
 * Arithmetic is IEEE binary64 with round-to-nearest-even; the file must be
 * built with -ffp-contract=off and without -ffast-math (denormals stay on).
 * Threads (OpenMP) only split the z-planes of one sweep; every cell is
 * computed by the same expression in the same order, so results do not
 * depend on the thread count.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* ---- SplitMix64, from its published definition -------------------------- */

#define ORACLE_SM64_GAMMA 0x9E3779B97F4A7C15ULL

/* Advance the Weyl state by the golden gamma and return the mixed output. */
uint64_t oracle_splitmix64_next(uint64_t *state)
{
    uint64_t z = (*state += ORACLE_SM64_GAMMA);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

/* First n outputs of the generator started in `seed`. */
void oracle_splitmix64_seq(uint64_t seed, int64_t n, uint64_t *out)
{
    uint64_t s = seed;
    for (int64_t i = 0; i < n; ++i) out[i] = oracle_splitmix64_next(&s);
}

/* Uniform [0,1) double from 64 random bits: the top 53 bits times 2^-53. */
static double oracle_unit(uint64_t h)
{
    return (double)(h >> 11) * (1.0 / 9007199254740992.0);
}

/* Start state of problem `pid`'s stream: the (pid+1)-th output from `seed`. */
static uint64_t oracle_stream_state(uint64_t seed, uint64_t pid)
{
    uint64_t s = seed;
    uint64_t h = 0;
    for (uint64_t i = 0; i <= pid; ++i) h = oracle_splitmix64_next(&s);
    return h;
}

/* Dense interior u0 (x fastest): the stream's outputs taken in order. */
void oracle_init_interior(int64_t nx, int64_t ny, int64_t nz, uint64_t seed,
                          uint64_t pid, double *u0)
{
    uint64_t s = oracle_stream_state(seed, pid);
    int64_t n = nx * ny * nz;
    for (int64_t g = 0; g < n; ++g) u0[g] = oracle_unit(oracle_splitmix64_next(&s));
}

/* u0 of one cell by skipping ahead: the Weyl state after g steps is
 * start + g*gamma (mod 2^64), so the g-th value needs one more step. */
double oracle_init_cell(int64_t nx, int64_t ny, uint64_t seed, uint64_t pid,
                        int64_t i, int64_t j, int64_t k)
{
    uint64_t s = oracle_stream_state(seed, pid);
    uint64_t g = (uint64_t)(i + nx * (j + ny * k));
    s += g * ORACLE_SM64_GAMMA;
    return oracle_unit(oracle_splitmix64_next(&s));
}

/* ---- the Jacobi iterate on the global grid ------------------------------- */

/* Index into a grid with a 1-cell ghost layer: i in 0..nx+1, x fastest. */
#define G(i, j, k) ((size_t)(i) + (size_t)(nx + 2) * ((size_t)(j) + (size_t)(ny + 2) * (size_t)(k)))

static const double W = 1.0 / 7.0; /* fl(1/7), rounded once at compile time */

/* Fill the ghost layer of `a`: faces from bc or the per-cell face arrays,
 * edges and corners NaN.  Face array layouts: x-faces ny*nz (j fastest),
 * y-faces nx*nz (i fastest), z-faces nx*ny (i fastest). */
static void oracle_fill_ghosts(int64_t nx, int64_t ny, int64_t nz, double *a,
                               const double bc[6], const double *const faces[6])
{
    for (int64_t k = 0; k <= nz + 1; ++k)
        for (int64_t j = 0; j <= ny + 1; ++j)
            for (int64_t i = 0; i <= nx + 1; ++i) {
                int ox = (i == 0 || i == nx + 1);
                int oy = (j == 0 || j == ny + 1);
                int oz = (k == 0 || k == nz + 1);
                int nout = ox + oy + oz;
                if (nout == 0) continue;
                if (nout > 1) { a[G(i, j, k)] = NAN; continue; }
                double v;
                if (ox) {
                    int f = (i == 0) ? 0 : 1;
                    v = faces && faces[f] ? faces[f][(j - 1) + ny * (k - 1)] : bc[f];
                } else if (oy) {
                    int f = (j == 0) ? 2 : 3;
                    v = faces && faces[f] ? faces[f][(i - 1) + nx * (k - 1)] : bc[f];
                } else {
                    int f = (k == 0) ? 4 : 5;
                    v = faces && faces[f] ? faces[f][(i - 1) + nx * (j - 1)] : bc[f];
                }
                a[G(i, j, k)] = v;
            }
}

/* One sweep b <- J(a) over the interior; returns max |b - a| if want_res. */
static double oracle_sweep(int64_t nx, int64_t ny, int64_t nz, const double *a,
                           double *b, int want_res, int nthreads)
{
    double res = 0.0;
    (void)nthreads;
#pragma omp parallel for num_threads(nthreads) schedule(static) reduction(max : res)
    for (int64_t k = 1; k <= nz; ++k)
        for (int64_t j = 1; j <= ny; ++j)
            for (int64_t i = 1; i <= nx; ++i) {
                double s = a[G(i, j, k)];
                s += a[G(i - 1, j, k)];
                s += a[G(i + 1, j, k)];
                s += a[G(i, j - 1, k)];
                s += a[G(i, j + 1, k)];
                s += a[G(i, j, k - 1)];
                s += a[G(i, j, k + 1)];
                double v = s * W;
                b[G(i, j, k)] = v;
                if (want_res) {
                    double d = fabs(v - a[G(i, j, k)]);
                    if (d > res) res = d;
                }
            }
    return res;
}

/*
 * Run the Jacobi iteration from interior u0 (dense, x fastest; NULL means the
 * seeded SplitMix64 interior of (seed, pid)) for at most t_max sweeps.
 *
 * check_every > 0: the residual is evaluated after every check_every-th sweep
 * and after sweep t_max; the run stops at the first evaluation with
 * residual <= tol when tol > 0.  check_every == 0: only the last sweep's
 * residual is evaluated.  *iters_done gets the sweeps performed.
 * Returns 0, or -1 on bad arguments / allocation failure.
 */
int oracle_jacobi(int64_t nx, int64_t ny, int64_t nz, const double *u0,
                  uint64_t seed, uint64_t pid, const double bc[6],
                  const double *const faces[6], int64_t t_max, double tol,
                  int64_t check_every, double *u_out, double *residual,
                  int64_t *iters_done, int nthreads)
{
    if (nx < 1 || ny < 1 || nz < 1 || t_max < 0 || check_every < 0 || !u_out || !bc)
        return -1;
    if (nthreads < 1) nthreads = 1;
    size_t cells = (size_t)(nx + 2) * (size_t)(ny + 2) * (size_t)(nz + 2);
    double *a = (double *)malloc(cells * sizeof(double));
    double *b = (double *)malloc(cells * sizeof(double));
    if (!a || !b) { free(a); free(b); return -1; }

    oracle_fill_ghosts(nx, ny, nz, a, bc, faces);
    oracle_fill_ghosts(nx, ny, nz, b, bc, faces);
    if (u0) {
        for (int64_t k = 1; k <= nz; ++k)
            for (int64_t j = 1; j <= ny; ++j)
                for (int64_t i = 1; i <= nx; ++i)
                    a[G(i, j, k)] = u0[(i - 1) + nx * ((j - 1) + ny * (k - 1))];
    } else {
        uint64_t s = oracle_stream_state(seed, pid);
        for (int64_t k = 1; k <= nz; ++k)
            for (int64_t j = 1; j <= ny; ++j)
                for (int64_t i = 1; i <= nx; ++i)
                    a[G(i, j, k)] = oracle_unit(oracle_splitmix64_next(&s));
    }

    double r = 0.0;
    int64_t t = 0;
    while (t < t_max) {
        int64_t next = t + 1;
        int check = (next == t_max) || (check_every > 0 && next % check_every == 0);
        double rr = oracle_sweep(nx, ny, nz, a, b, check, nthreads);
        double *tmp = a; a = b; b = tmp;   /* the new iterate becomes the input */
        t = next;
        if (check) {
            r = rr;
            if (tol > 0.0 && r <= tol) break;
        }
    }

    for (int64_t k = 1; k <= nz; ++k)
        for (int64_t j = 1; j <= ny; ++j)
            for (int64_t i = 1; i <= nx; ++i)
                u_out[(i - 1) + nx * ((j - 1) + ny * (k - 1))] = a[G(i, j, k)];
    if (residual) *residual = r;
    if (iters_done) *iters_done = t;
    free(a);
    free(b);
    return 0;
}

/*
 * Value of interior cell (ci, cj, ck) (0-based) after t sweeps of the seeded
 * problem with constant faces bc, computed on the cell's domain of dependence
 * only.  A cell's value after t sweeps depends only on cells at most t steps
 * away along each axis, so the iterate is run on the sub-box within distance
 * t of the cell (clipped to the grid).  Outside the sub-box one layer is held
 * at its initial value (or the true boundary where the sub-box reaches it):
 * a wrong value there moves inward one cell per sweep and never reaches the
 * centre within t sweeps.
 */
int oracle_cell_after(int64_t nx, int64_t ny, int64_t nz, uint64_t seed,
                      uint64_t pid, const double bc[6], int64_t t, int64_t ci,
                      int64_t cj, int64_t ck, double *value)
{
    if (nx < 1 || ny < 1 || nz < 1 || t < 0 || !value || ci < 0 || ci >= nx ||
        cj < 0 || cj >= ny || ck < 0 || ck >= nz)
        return -1;
    /* sub-box in global 1-based ghosted coordinates, including its frame */
    int64_t lo[3], hi[3];
    int64_t c[3] = {ci + 1, cj + 1, ck + 1};
    int64_t n[3] = {nx, ny, nz};
    for (int a = 0; a < 3; ++a) {
        lo[a] = c[a] - t - 1; if (lo[a] < 0) lo[a] = 0;
        hi[a] = c[a] + t + 1; if (hi[a] > n[a] + 1) hi[a] = n[a] + 1;
    }
    int64_t mx = hi[0] - lo[0] + 1, my = hi[1] - lo[1] + 1, mz = hi[2] - lo[2] + 1;
    size_t cells = (size_t)mx * (size_t)my * (size_t)mz;
    double *a = (double *)malloc(cells * sizeof(double));
    double *b = (double *)malloc(cells * sizeof(double));
    if (!a || !b) { free(a); free(b); return -1; }
#define L(i, j, k) ((size_t)((i) - lo[0]) + (size_t)mx * ((size_t)((j) - lo[1]) + (size_t)my * (size_t)((k) - lo[2])))
    uint64_t s0 = oracle_stream_state(seed, pid);
    for (int64_t k = lo[2]; k <= hi[2]; ++k)
        for (int64_t j = lo[1]; j <= hi[1]; ++j)
            for (int64_t i = lo[0]; i <= hi[0]; ++i) {
                int ox = (i == 0 || i == nx + 1), oy = (j == 0 || j == ny + 1), oz = (k == 0 || k == nz + 1);
                double v;
                if (ox + oy + oz > 1) v = NAN;
                else if (ox) v = bc[i == 0 ? 0 : 1];
                else if (oy) v = bc[j == 0 ? 2 : 3];
                else if (oz) v = bc[k == 0 ? 4 : 5];
                else {
                    uint64_t s = s0 + (uint64_t)((i - 1) + nx * ((j - 1) + ny * (k - 1))) * ORACLE_SM64_GAMMA;
                    v = oracle_unit(oracle_splitmix64_next(&s));
                }
                a[L(i, j, k)] = v;
                b[L(i, j, k)] = v;
            }
    for (int64_t step = 0; step < t; ++step) {
        for (int64_t k = lo[2] + 1; k < hi[2]; ++k)
            for (int64_t j = lo[1] + 1; j < hi[1]; ++j)
                for (int64_t i = lo[0] + 1; i < hi[0]; ++i) {
                    double s = a[L(i, j, k)];
                    s += a[L(i - 1, j, k)];
                    s += a[L(i + 1, j, k)];
                    s += a[L(i, j - 1, k)];
                    s += a[L(i, j + 1, k)];
                    s += a[L(i, j, k - 1)];
                    s += a[L(i, j, k + 1)];
                    b[L(i, j, k)] = s * W;
                }
        double *tmp = a; a = b; b = tmp;
    }
    *value = a[L(c[0], c[1], c[2])];
#undef L
    free(a);
    free(b);
    return 0;
}

/* Number of OpenMP threads a parallel region would use (1 without OpenMP). */
int oracle_max_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
