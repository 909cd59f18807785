/*
 * j3d.h -- C ABI of libj3d, an MI355X (gfx950) implementation of the FP64
 * Jacobi3D hot path of Choi, Richards and Kale, "Improving Scalability with
 * GPU-Aware Asynchronous Tasks" (arXiv 2202.11819).
 *
 * The method (Sec. II-A, Fig. 1, Fig. 3): a 3-D grid is over-decomposed into
 * blocks; every iteration each block packs its six halo faces, hands them to
 * its neighbours, unpacks the faces it receives, and applies the Jacobi
 * update to its whole block, reading the previous iterate from one buffer and
 * writing the next into the other (Sec. III-C).  Here every block sits on one
 * GPU: halos move block to block in device memory.  Fused execution follows
 * kernel-fusion strategy C (unpack, update and pack as one kernel,
 * Sec. III-D-1) and graph execution follows Sec. III-D-2.
 *
 * Numerics (readings of what the paper leaves open):
 *   u'(c) = (((((( u(c) + u(x-) ) + u(x+) ) + u(y-) ) + u(y+) ) + u(z-) ) + u(z+)) * fl(1/7)
 * in IEEE binary64, round to nearest even, no contraction, denormals kept.
 * Boundary: a fixed 1-cell Dirichlet layer (one constant per face, or a
 * per-cell array per face).  Seeded interior: uniform [0,1) from SplitMix64,
 * independent of the decomposition.  Residual: max over the interior of
 * |u_new - u_old| for the last sweep, 0 when no sweep ran.  Every mode and
 * every decomposition yields the same bits.
 *
 * Conventions for every call:
 *   - Returns j3d_status; 0 is success, negative is an error.  No exception or
 *     abort crosses the ABI.  j3d_last_error() gives this thread's message for
 *     the last non-OK status.
 *   - All validation happens before any device work: a call that fails with
 *     J3D_EINVAL / J3D_ENOMEM / J3D_EBUDGET / J3D_EBUSY / J3D_ESTATE leaves
 *     every object unchanged.  J3D_EDEVICE reports a HIP runtime error; the
 *     object should then be destroyed.
 *   - The caller owns the device arena (memory the library lays its data out
 *     in; it never allocates device memory of its own except the pool's
 *     copy-stream events), the HIP stream (void* holding a hipStream_t; NULL is
 *     the default stream) and all host buffers.  Handles are opaque and not
 *     thread-safe: use one host thread per handle.
 *   - Device arrays and arenas must be 256-byte aligned.
 *   - Work is enqueued asynchronously on the handle's stream unless a call
 *     says it synchronises.
 *   - Dense grid arrays are interior cells only, x fastest, then y, then z
 *     (nx*ny*nz doubles), independent of the decomposition.
 */
#ifndef J3D_H
#define J3D_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    J3D_OK = 0,
    J3D_EINVAL = -1,  /* bad argument */
    J3D_ENOMEM = -2,  /* arena too small */
    J3D_EBUDGET = -3, /* pool: not enough free budget for this request */
    J3D_EBUSY = -4,   /* pool: no free slot */
    J3D_EDEVICE = -5, /* HIP runtime error, or no usable gfx950 device */
    J3D_ESTATE = -6   /* call not valid in the object's current state */
} j3d_status;

/* How j3d_run drives the iterations (Sec. III-D).
 *  UNFUSED_BLOCK: per block and iteration, six pack kernels, six device copies,
 *                 six unpack kernels and one update kernel (no fusion: the
 *                 paper's baseline with one launch stream of GPU operations
 *                 per over-decomposed block).
 *  UNFUSED_PHASE: per iteration one fused pack kernel (strategy A shape: one
 *                 thread per cell of the largest face, each thread visiting
 *                 the six faces), one exchange copy kernel, one fused unpack
 *                 kernel (strategy B) and one update kernel, all blocks at once.
 *  FUSED:         per iteration one kernel for all blocks (strategy C,
 *                 generalised to all blocks): it reads its y and z halos
 *                 straight from the neighbours' current iterate, updates, and
 *                 hands its new x faces to the neighbours' x-halo storage of
 *                 the next iterate; pack, exchange and unpack need no copy.
 *  GRAPH:         FUSED iterations captured once into a HIP graph holding an
 *                 even number of sweeps (both buffer parities), replayed.
 *  BLOCK_A/B/C:   the paper's fusion strategies at block granularity (one
 *                 launch stream of operations per block, like UNFUSED_BLOCK):
 *                 A fuses each block's six pack kernels into one; B also its
 *                 six unpack kernels into one (pack, six copies, unpack,
 *                 update); C runs one kernel per block that reads its halos
 *                 where the neighbours keep them, updates, and hands its x
 *                 faces over (no copies).
 *  HOST_STAGED:   the exchange staged through host memory, as without
 *                 GPU-aware communication: one pack kernel for all blocks,
 *                 every face copied to page-locked host memory (into the
 *                 receiver's slot), each block's received faces copied back,
 *                 then unpack and update.
 *  HOST_OVERLAP:  HOST_STAGED with Fig. 1's split of the update: while the
 *                 faces are in transit, a second stream updates each block's
 *                 interior (the cells whose six neighbours lie inside the
 *                 block); once they are delivered and unpacked, the exterior
 *                 (the one-cell shell that reads halos) is updated.  Every
 *                 cell is written once per iteration.
 *  TWO_SWEEP:     two iterations per launch (temporal blocking) on a grid of
 *                 one block: each workgroup computes the intermediate iterate
 *                 on its tile plus a one-cell ring in LDS and writes only
 *                 every second iterate, halving the HBM traffic per
 *                 iteration.  An odd count ends with one FUSED sweep.  EINVAL
 *                 for a decomposed grid.  Not in the paper; it applies where
 *                 no block boundary needs an exchange.
 *  CAPTURED:      a flag OR-ed with any mode: its iterations are captured once
 *                 into HIP graphs (50 sweeps per graph for FUSED, 48 for
 *                 TWO_SWEEP, 2 for the others, whose graphs hold thousands of
 *                 nodes) and replayed;
 *                 GRAPH is FUSED | CAPTURED.  Results never depend on the mode. */
typedef enum {
    J3D_UNFUSED_BLOCK = 0,
    J3D_UNFUSED_PHASE = 1,
    J3D_FUSED = 2,
    J3D_GRAPH = 3,
    J3D_BLOCK_A = 4,
    J3D_BLOCK_B = 5,
    J3D_BLOCK_C = 6,
    J3D_HOST_STAGED = 7,
    J3D_HOST_OVERLAP = 8,
    J3D_TWO_SWEEP = 9,
    J3D_CAPTURED = 16
} j3d_mode;

/* One Jacobi3D problem.
 *  n[a]       interior cells along x, y, z; each >= 1.
 *  nblk[a]    blocks along each axis.  All three 0: the surface-minimising
 *             split of auto_parts blocks (Sec. IV-A; see j3d_auto_split),
 *             auto_parts 0 meaning one block.
 *  split[a]   optional explicit block extents along axis a (nblk[a] entries,
 *             each >= 1, summing to n[a]); NULL: even split, which requires
 *             n[a] % nblk[a] == 0.  Only read during the call it is passed to.
 *  bc[f]      Dirichlet value of global face f: 0 x-, 1 x+, 2 y-, 3 y+, 4 z-, 5 z+.
 *  seed, pid  the seeded interior: problem pid's SplitMix64 stream of seed
 *             (the stream's start state is the generator's (pid+1)-th output
 *             from state seed; cell g = i + nx*(j + ny*k) takes output g+1 of
 *             that stream, mapped to [0,1) as (h >> 11) * 2^-53).            */
typedef struct {
    int64_t n[3];
    int32_t nblk[3];
    int32_t auto_parts;
    const int64_t *split[3];
    double bc[6];
    uint64_t seed;
    uint64_t pid;
} j3d_problem;

/* Kernel shape for the sweep.  variant: index into the compiled tile shapes
 * (j3d_variant_info); -1 picks by block size.  zchunk: z-planes per tile
 * (>= 1; 0 = whole block depth).  blocks_per_cu: 0 launches one workgroup
 * per tile; > 0 launches a persistent grid of blocks_per_cu workgroups per
 * compute unit that take tiles from per-XCD queues.  Tile shape and
 * scheduling never change the result bits.                                   */
typedef struct {
    int32_t variant;
    int32_t zchunk;
    int32_t blocks_per_cu;
} j3d_tune;

typedef struct j3d_solver j3d_solver;
typedef struct j3d_batch j3d_batch;
typedef struct j3d_pool j3d_pool;

/* ---- host-only queries (no device needed) ------------------------------ */

/* Thread-local text of the last non-OK status on this thread ("" if none).
 * Not in the paper: error reporting of this library.                         */
const char *j3d_last_error(void);

/* Library version string (names the device architecture it was built for).
 * Not in the paper.                                                          */
const char *j3d_version(void);

/* Surface-minimising split of an n[0] x n[1] x n[2] grid into exactly `parts`
 * blocks (Sec. IV-A: the grid is decomposed so that the total surface area,
 * which sets the communication volume, is smallest).  Only factorisations
 * with nblk[a] <= n[a] are considered; ties go to the one with the most
 * blocks along z, then along y.  The chosen counts need not divide n[a]:
 * uneven extents follow the j3d_block_extents rule.  EINVAL if parts < 1,
 * parts > 2^22 (the block limit of a problem) or no factorisation fits.      */
j3d_status j3d_auto_split(const int64_t n[3], int32_t parts, int32_t nblk_out[3]);

/* Resolved decomposition of a problem (Sec. II-A, Fig. 1: the global grid is
 * cut into blocks, one per process or chare; Sec. IV-A: over-decomposition
 * into more blocks than GPUs): nblk_out[3] blocks per axis and, if
 * extents_out is non-NULL, the extents along x, then y, then z
 * (nblk[0]+nblk[1]+nblk[2] values, at most cap; EINVAL if more).  Auto
 * splits whose counts do not divide n[a] give the first n[a] % nblk[a]
 * blocks one extra cell.  Host only.                                         */
j3d_status j3d_block_extents(const j3d_problem *p, int32_t nblk_out[3],
                             int64_t *extents_out, int64_t cap);

/* Device bytes j3d_create needs for this problem: the two iterates of every
 * block (Sec. III-C: previous and current iterate in two buffers), their halo
 * storage, the send/receive halo buffers of the unfused modes (Fig. 1),
 * descriptor tables and staging.  Host only; EINVAL for a bad problem.       */
j3d_status j3d_arena_bytes(const j3d_problem *p, uint64_t *bytes);

/* Bytes of the two field copies only (interior plus halo storage): the
 * per-GPU memory the paper quotes for its weak-scaling grids (Sec. IV-B).
 * Host only.                                                                 */
j3d_status j3d_field_bytes(const j3d_problem *p, uint64_t *bytes);

/* Compiled sweep tile shapes: variant i covers tile_x x tile_y cells of an
 * x-y plane with `threads` threads.  tile_x == 0 marks a flattened variant:
 * its tiles are whole row segments sized per block (any width, up to tile_y
 * cells, every thread owning tile_y / threads cells).  Returns EINVAL past
 * the last variant.  Not in the paper: kernel shapes of this implementation. */
j3d_status j3d_variant_info(int32_t variant, int32_t *tile_x, int32_t *tile_y,
                            int32_t *threads);

/* ---- plain solver -------------------------------------------------------- */

/* Lay out problem p in dev_arena (arena_bytes >= j3d_arena_bytes(p)) and
 * enqueue the seeded initialisation on hip_stream.  The problem is the
 * paper's (Sec. II-A, Fig. 1): a global 3-D grid cut into blocks, each with
 * six halo faces, updated for a fixed number of iterations; the seeded
 * interior and the Dirichlet values are readings (the paper states neither).
 * EINVAL for a bad problem or NULL/unaligned arena, ENOMEM if the arena is
 * too small, EDEVICE if no gfx950 device is current; all before device work.
 * The solver keeps pointers into the arena, which must outlive it.           */
j3d_status j3d_create(const j3d_problem *p, void *dev_arena, uint64_t arena_bytes,
                      void *hip_stream, j3d_solver **out);

/* Replace the current interior with src (dense nx*ny*nz) and reset the
 * iteration count to 0.  src_on_device: 1 if src is device memory, 0 for host
 * memory (then the call synchronises).  Not in the paper (which initialises
 * in place): loads any initial iterate, and with j3d_get_interior lets a
 * solve be checkpointed and resumed.                                        */
j3d_status j3d_set_interior(j3d_solver *s, const double *src, int src_on_device);

/* Per-cell Dirichlet values for global face f (0..5), overriding bc[f].
 * Layouts: x-faces ny*nz (y fastest), y-faces nx*nz (x fastest), z-faces nx*ny
 * (x fastest).  src_on_device as above.  EINVAL for f outside 0..5 or a NULL
 * src.  Not in the paper (it states no boundary condition): a per-cell
 * boundary lets linear fields be checked as exact fixed points.             */
j3d_status j3d_set_face(j3d_solver *s, int32_t face, const double *src, int src_on_device);

/* Choose the sweep kernel shape (see j3d_tune); NULL restores the default.
 * EINVAL for a variant out of range or a negative field.  Not in the paper. */
j3d_status j3d_set_tune(j3d_solver *s, const j3d_tune *t);

/* The shape in use (the default chosen by block size until j3d_set_tune).
 * Not in the paper.                                                          */
j3d_status j3d_get_tune(const j3d_solver *s, j3d_tune *out);

/* Enqueue `iters` (>= 0) Jacobi iterations in the given mode: the paper's
 * iteration loop (Fig. 1; Fig. 3 for its GPU form: pack, exchange in six
 * directions, unpack, update, with the buffers swapped every iteration,
 * Sec. III-C), executed as the chosen j3d_mode (fusion Sec. III-D-1, graphs
 * Sec. III-D-2, host staging Sec. II-B, overlap Fig. 1).  If residual_out is
 * non-NULL the last sweep's residual is written there and the call
 * synchronises (the residual is a reading: the paper runs a fixed count);
 * otherwise it returns once the work is enqueued.  EINVAL for iters < 0 or
 * an unknown mode, before any device work.                                   */
j3d_status j3d_run(j3d_solver *s, int64_t iters, j3d_mode mode, double *residual_out);

/* Iterations performed since creation or the last j3d_set_interior.  Not in
 * the paper (resume bookkeeping).                                            */
j3d_status j3d_iters_done(const j3d_solver *s, int64_t *iters);

/* Copy the current interior to dst (dense nx*ny*nz, independent of the
 * decomposition).  Synchronises for host destinations; device destinations
 * are written asynchronously.  Not in the paper (readback of the result).   */
j3d_status j3d_get_interior(j3d_solver *s, double *dst, int dst_on_device);

/* Release the solver's host objects (graphs, tables); the arena stays the
 * caller's.  Synchronises the stream first.  Not in the paper.              */
j3d_status j3d_destroy(j3d_solver *s);

/* ---- batched form: many independent problems, one launch per step -------
 * Not in the paper.  Each problem is the paper's Jacobi3D problem (Sec. II-A);
 * the form extends fusion strategy C (one kernel per iteration, Sec. III-D-1)
 * across independent problems.                                              */

/* Device bytes for a batch of `count` problems (host only). */
j3d_status j3d_batch_arena_bytes(int32_t count, const j3d_problem *probs, uint64_t *bytes);

/* Lay out `count` problems (each with its own decomposition, boundary and
 * seed) and their iteration counts iters[i] >= 0, and enqueue their seeded
 * initialisation.  tune: the kernel shape for every launch of the batch, as
 * resolved by the caller's autotuner from its tune cache (the cache itself,
 * a file of measured shapes per device and problem mix, is kept by the
 * caller, not parsed here); NULL picks the default shape.  EINVAL for count
 * < 1, NULL arrays, a bad problem or a bad shape; ENOMEM if the arena is too
 * small; all before device work.                                            */
j3d_status j3d_batch_create(int32_t count, const j3d_problem *probs, const int64_t *iters,
                            void *dev_arena, uint64_t arena_bytes, void *hip_stream,
                            const j3d_tune *tune, j3d_batch **out);

/* Run every problem to its iteration count: step s is one launch covering
 * every tile of every problem with iters > s.  residuals_out (count doubles
 * or NULL) receives each problem's last-sweep residual; with it the call
 * synchronises.  A batch runs once; ESTATE afterwards.                       */
j3d_status j3d_batch_run(j3d_batch *b, double *residuals_out);

/* The same run with two sweeps per launch (the TWO_SWEEP scheme of j3d_run)
 * for batches whose problems are all undivided (one block each; EINVAL
 * otherwise, before any device work): problems with an odd count first take
 * one ordinary sweep in one launch over the batch, then launch k covers the
 * problems with more than k sweep pairs left, each advancing two sweeps.
 * Results and residuals are bit-identical to j3d_batch_run.  The batch's
 * tile shape from j3d_tune is used for the odd sweep only; the two-sweep
 * launches use 64 x 16 tiles and z-chunks of 32.  Not in the paper.  A batch
 * runs once, by either call; ESTATE afterwards.                              */
j3d_status j3d_batch_run_two_sweep(j3d_batch *b, double *residuals_out);

/* Copy problem i's interior to dst (dense).  Synchronises for host dst. */
j3d_status j3d_batch_get_interior(j3d_batch *b, int32_t i, double *dst, int dst_on_device);

j3d_status j3d_batch_destroy(j3d_batch *b);

/* ---- served form: continuous batching under an HBM budget ----------------
 * Not in the paper.  Each request is the paper's Jacobi3D problem
 * (Sec. II-A) as one block; rounds use the fused update (Sec. III-D-1), and
 * finished work is found by polling events, as the paper detects the
 * completion of asynchronous GPU work (Sec. III-A).                         */

/* Device bytes one request of problem p occupies in a pool (host only;
 * EINVAL unless p is a single-block problem).                               */
j3d_status j3d_pool_request_bytes(const j3d_problem *p, uint64_t *bytes);

/* A pool over dev_arena: budget_bytes of it hold request grids, the rest (see
 * j3d_pool_overhead_bytes) its tables; arena_bytes (>= overhead + budget) is
 * the arena's size, checked so that a short arena is refused (ENOMEM) rather
 * than overrun.  At most max_slots (1..65536) requests are resident.  The
 * pool creates one extra stream for result copies.  EINVAL for NULL or
 * unaligned arena, budget 0 or max_slots out of range; before device work.  */
j3d_status j3d_pool_overhead_bytes(int32_t max_slots, uint64_t *bytes);
j3d_status j3d_pool_create(void *dev_arena, uint64_t arena_bytes, uint64_t budget_bytes,
                           int32_t max_slots, void *hip_stream, j3d_pool **out);

/* Admit a request: solve p for at most max_iters sweeps, evaluating the
 * residual every check_every sweeps (0: only at the end) and at max_iters,
 * stopping once it is <= tol (tol <= 0: never early).  host_result (nx*ny*nz
 * doubles, best page-locked, or NULL) receives the final interior by an
 * asynchronous copy as soon as the request finishes, while later rounds run;
 * with NULL the result stays in device memory until j3d_pool_fetch.  The
 * caller keeps host_result valid until the slot is reported done or is
 * released.  EBUSY without a free slot, EBUDGET without enough free budget,
 * EINVAL for a bad problem, max_iters < 0 or check_every < 0; nothing
 * changes then.  The request joins the next round.                         */
j3d_status j3d_pool_admit(j3d_pool *pl, const j3d_problem *p, int64_t max_iters, double tol,
                          int32_t check_every, double *host_result, int32_t *slot);

/* Enqueue one round of up to `sweeps` sweeps for the running requests the
 * round policy picks (each request stops at its own limit and never passes a
 * residual check point within a round).  Asynchronous.  ESTATE if a round is
 * still in flight (poll first).                                             */
j3d_status j3d_pool_step(j3d_pool *pl, int32_t sweeps);

/* Round policy.  fill_cells > 0: requests join a round in order of least
 * remaining work (cells x sweeps left) until the round holds at least
 * max(fill_cells, running cells / backlog_share) cells (backlog_share 0: just
 * fill_cells), so rounds grow with the backlog; a request left out of
 * max_wait_rounds consecutive rounds joins first.  fill_cells == 0: every
 * running request joins every round.  Default: fill_cells = 2^25,
 * max_wait_rounds = 32, backlog_share = 2.  Results do not depend on the
 * policy, only latencies and throughput do.                                 */
j3d_status j3d_pool_set_policy(j3d_pool *pl, int64_t fill_cells, int32_t max_wait_rounds,
                               int32_t backlog_share);

/* Sweep kernel shape of the pool's rounds: variant (-1 keeps the default
 * flattened 512-thread tile) and zchunk (>= 1 planes per tile, default 32);
 * blocks_per_cu must be 0.
 * NULL restores the default.  ESTATE unless every slot is free (a request's
 * tile count is checked against the pool's tile table at admission).       */
j3d_status j3d_pool_set_tune(j3d_pool *pl, const j3d_tune *t);

/* enable 1: rounds advance requests two sweeps per launch (the TWO_SWEEP
 * scheme of j3d_run; every request is an undivided grid): a request whose
 * share of the round is odd takes one ordinary sweep first.  Results,
 * residuals and check points are unchanged (bit-identical).  enable 0: one
 * sweep per launch (the default).  Only while the pool is empty (ESTATE
 * otherwise); EINVAL for other values.  Not in the paper.                  */
j3d_status j3d_pool_set_two_sweep(j3d_pool *pl, int32_t enable);

/* Non-blocking progress: retires a completed round (updating every request's
 * sweep count and residual, deciding which finished), starts the result
 * copies of finished requests, and reports in done[] (at most cap) the slots
 * whose results have fully arrived in host memory since the last poll.
 * *round_busy is set to 1 while a round is still in flight.                 */
j3d_status j3d_pool_poll(j3d_pool *pl, int32_t *done, int32_t cap, int32_t *n_done,
                         int32_t *round_busy);

/* Residual and sweep count of a finished request (either may be NULL).
 * ESTATE until the request is reported done by j3d_pool_poll.                */
j3d_status j3d_pool_result(j3d_pool *pl, int32_t slot, double *residual, int64_t *iters_done);

/* Fetch a finished request: its final interior (dense nx*ny*nz, x fastest)
 * is copied to host_dst (NULL: not copied) and its residual and sweep count
 * are written (each may be NULL).  Synchronises with the copy.  Works
 * whether or not a host_result was given at admission (the result stays in
 * device memory until release).  EINVAL for a NULL pool or a slot out of
 * range, ESTATE for a slot that is free or not finished; before any copy.   */
j3d_status j3d_pool_fetch(j3d_pool *pl, int32_t slot, double *host_dst, double *residual, int64_t *iters_done);

/* Free a finished (or still queued/running: cancel) request's slot and bytes.
 * Waits for a result copy still in flight.  ESTATE for a free slot.          */
j3d_status j3d_pool_release(j3d_pool *pl, int32_t slot);

/* Occupancy: resident requests and bytes in use (host only). */
j3d_status j3d_pool_usage(const j3d_pool *pl, int32_t *slots_used, uint64_t *bytes_used);

j3d_status j3d_pool_destroy(j3d_pool *pl);

/* ---- allocation-free solve ---------------------------------------------- */

/* For callers that cannot allocate device memory (code under stream capture,
 * tight serving loops, harnesses that forbid allocation): a one-shot solve of
 * problem p in FUSED mode (the j3d_run path) that calls no hipMalloc, hipFree,
 * hipHostMalloc, stream, event or graph creation.
 *  fields        caller device memory, 256-byte aligned, of at least
 *                j3d_field_bytes(p) bytes (ENOMEM otherwise): the two iterates
 *                of every block and their halo storage.  Contents on entry are
 *                ignored; they hold the final state on return.
 *  interior_in   device array, dense nx*ny*nz (x fastest): the initial
 *                interior; NULL: the seeded interior of p (seed, pid).
 *  interior_out  device array, dense nx*ny*nz: the interior after `iters`
 *                sweeps.  Neither array may overlap `fields` (EINVAL).
 *  iters         sweeps (>= 0).
 *  residual_out  host pointer or NULL: the last sweep's residual (0 for
 *                iters == 0); with it the call synchronises at the end.
 * The descriptor, tile and map tables live in a static device array of
 * 4 MiB per GPU (held until the process ends): EINVAL for a problem whose
 * tables need more (256 bytes per block and 48 per tile: about 13 000 blocks
 * of one tile each, fewer with more tiles).  The call uploads those tables
 * from host memory and synchronises the stream once before its first launch.
 * Every call on a GPU shares that GPU's array, so calls that overlap on one
 * GPU (other threads or streams) race; run them one at a time per GPU.
 * Results are bit-identical to j3d_create + j3d_set_interior (or the seeded
 * init) + j3d_run + j3d_get_interior.  EINVAL for NULL p / fields /
 * interior_out, misaligned fields or iters < 0; all before device work.     */
j3d_status j3d_solve_noalloc(const j3d_problem *p, void *fields, uint64_t fields_bytes,
                             const double *interior_in, double *interior_out, int64_t iters,
                             double *residual_out, void *hip_stream);

/* ---- measurement helpers ------------------------------------------------- */

/* Enqueue a plain device copy of `bytes` (multiple of 16) from src to dst: the
 * streaming-bandwidth reference kernel used to calibrate HBM counters.  Not
 * in the paper (measurement).                                               */
j3d_status j3d_device_copy(void *dst, const void *src, uint64_t bytes, void *hip_stream);

/* Number of compute units of the current device (EDEVICE without a device).
 * Not in the paper.                                                          */
j3d_status j3d_device_cus(int32_t *cus);

#ifdef __cplusplus
}
#endif

#endif /* J3D_H */
