// j3d_internal.hpp -- descriptors shared by the host engine and the HIP kernels.
//
// Memory layout of one block b (interior extents ex, ey, ez) for each of the
// two iterates (parity 0 and 1; Sec. III-C keeps two copies of the block and
// swaps their roles every iteration):
//
//   field  F[p][b]: (ez+2) planes of (ey+2) rows x pitch doubles, x fastest,
//          pitch = ex (rows unpadded: the rows of a plane are one contiguous
//          run); the plane stride plane_stride(ex, ey) rounds (ey+2)*ex up to
//          16 cells so that every plane starts on a 128-byte line.  Plane 0
//          and plane ez+1 hold the z- / z+ halos, row 0 and row ey+1 of every
//          plane hold the y- / y+ halos; interior cell (x, y, z) sits at
//          (z+1)*plane_stride + (y+1)*pitch + x.  Rows carry no x ghosts, so a
//          row of the interior and a y- or z-halo row are the same contiguous
//          ex doubles; edge rows of the halo planes are never read.
//   x-halo X[p][b]: two arrays of ey*ez doubles (x- then x+), y fastest.  The
//          x-halos live apart from the rows so that a neighbour writes them as
//          contiguous runs instead of one double per row.
//
// A global-boundary face holds its Dirichlet values in the same halo storage,
// written once for both parities.  For interior faces the unfused modes
// unpack received faces into this storage; the fused sweep reads y and z
// halos from the neighbour's field directly and receives only x halos.
// The unfused modes also use per-block contiguous send and receive buffers
// S[b], R[b], each the six faces in the order x-, x+, y-, y+, z-, z+ with
// sizes ey*ez, ey*ez, ex*ez, ex*ez, ex*ey, ex*ey (Fig. 1's send_halo/recv_halo).
#pragma once

#include <cstddef>
#include <cstdint>
#include <vector>

#include "../../include/j3d.h"

namespace j3d {

// Face numbering: 0 x-, 1 x+, 2 y-, 3 y+, 4 z-, 5 z+.  opp(f) = f ^ 1.

// Plane stride of a block's field in doubles: (ey+2) rows of ex cells,
// rounded up to a multiple of 16 cells (128 bytes).
constexpr int64_t plane_stride(int64_t ex, int64_t ey) { return ((ey + 2) * ex + 15) / 16 * 16; }

struct BlockDesc {          // 256 bytes, read by kernels through scalar loads
    int64_t off[2];         // F[p][b] offset, in doubles from the arena base
    int64_t xoff[2];        // X[p][b] offset (x- array, then x+ array)
    int64_t sr_off;         // S[b] offset; R[b] follows at sr_off + face_total
    int64_t face_total;     // 2*ey*ez + 2*ex*ez + 2*ex*ey
    int32_t ext[3];         // ex, ey, ez
    int32_t prob;           // index of the owning problem in the problem table
    int32_t nbr[6];         // neighbour block per face (table index) or -1
    int32_t org[3];         // global coordinates of the block's first cell
    int32_t pitch;          // row stride of the field in doubles (= ex: rows unpadded)
    int32_t pad[6];
    // Fused sweep: where this block's halos come from and where its x faces
    // go, worked out from the neighbours when the plan is made (doubles from
    // the arena base, per iterate parity; -1: no neighbour on that face, the
    // own ghost layer serves), so a workgroup finds them in its own block's
    // descriptor instead of through a chain of loads of the neighbours' ones.
    int64_t fx_m[2];        // x- neighbour's X[q] x+ half: takes this block's x- face of iterate q
    int64_t fx_p[2];        // x+ neighbour's X[q] x- half
    int64_t fy_m[2];        // y- neighbour's F[p]: its last interior row, at plane index 0
    int64_t fy_p[2];        // y+ neighbour's F[p]: its first interior row, at plane index 0
    int64_t fz_m[2];        // z- neighbour's F[p]: its last interior plane
    int64_t fz_p[2];        // z+ neighbour's F[p]: its first interior plane
    int64_t fy_step[2];     // plane strides of the y- and y+ neighbours' fields, doubles
    int64_t pad2[2];
};
static_assert(sizeof(BlockDesc) == 256, "BlockDesc layout");

// Problem state seen by the multi-problem sweep (batched and served forms).
struct ProbDesc {           // 64 bytes
    int64_t base;           // sweeps already done when step 0 of this launch sequence runs
    int64_t limit;          // sweep count at which the problem stops
    int32_t check_every;    // residual every k-th sweep (0: only at `limit`)
    int32_t res_slot;       // index of the problem's residual word
    int32_t flags;          // PF_RES_LAST: evaluate the residual at `limit`
    int32_t pad0;
    int64_t pad[4];
};
static_assert(sizeof(ProbDesc) == 64, "ProbDesc layout");

enum : int32_t { PF_RES_LAST = 1 };

// One sweep tile: block index, tile coordinates along x, y, z, and the cells
// it covers (x0.., y0.., z0.., extents nxv, nyv, nzv), worked out on the host
// when the table is built, so a workgroup reads its rectangle instead of
// recomputing it (every wave would run the divisions on the compute unit's
// one scalar unit).
struct Tile {
    int32_t block, tx, ty, tz;
    int32_t x0, y0, z0;
    int32_t nxv, nyv, nzv;
    int32_t pad[2];
};
static_assert(sizeof(Tile) == 48, "Tile layout");

enum : int32_t {
    SW_FUSED = 1,   // halos from the neighbours (y, z read directly; x faces handed over)
    SW_RES = 2,     // plain mode: residual of this sweep into res[0] (via the block's problem)
    SW_MULTI = 4,   // per-problem activity, parity and residual policy from ProbDesc
    SW_PERSIST = 8, // persistent grid with per-XCD tile queues
    SW_INNER = 16   // only the cells whose six neighbours lie inside the block (Fig. 1's
                    // interior update): every tile clipped to [1, e-1) on each axis
};

constexpr int kXcdCount = 8;  // XCDs (each with its own L2) per MI355X

struct SweepArgs {
    // A workgroup first reads the fields of the first 64 bytes (one scalar
    // cache line): where its tile is.
    const Tile *tiles;
    int32_t tile_begin;
    // One workgroup per tile: XCD x runs tiles [xcut[x], xcut[x+1]) of the
    // launch (relative to tile_begin); launch_sweep fills equal counts when
    // the caller leaves them all zero.
    int32_t xcut[kXcdCount + 1];
    int32_t tile_count;
    int32_t zchunk;
    int32_t parity;               // plain mode: parity of the input iterate
    int32_t flags;
    double *base;                 // arena base
    const BlockDesc *blocks;
    const ProbDesc *probs;
    unsigned long long *res;      // residual words (bit patterns of non-negative doubles)
    unsigned int *queue;          // persistent mode: 2 x 8 tile counters
    int64_t step;                 // multi mode: sweep index of this launch
    int32_t queue_slot;           // persistent mode: which half of `queue` this launch uses
};
static_assert(offsetof(SweepArgs, flags) + sizeof(int32_t) <= 64, "tile lookup fields in one 64-byte line");

// ---- kernel variants ----------------------------------------------------------

// tile_x == 0 marks a flattened variant: its tiles cover whole row segments
// of any width and tile_y is its cell capacity per plane (threads * rows per
// thread).
struct VariantInfo {
    int tile_x, tile_y, threads;
    int prefetch;  // planes of loads in flight beyond the next one
};
int variant_count();
VariantInfo variant_info(int v);

// ---- flattened tiles ------------------------------------------------------------
// A flattened tile covers nxv x nyv cells of an x-y plane.  Its cells are
// numbered x fastest and dealt to the threads in order (slot f is cell
// (f % nxv, f / nxv)), so no lane idles except in the tile's last partial
// wave.  Rows are stored unpadded (pitch = width), so a tile of whole rows is
// one contiguous run of memory per plane: consecutive lanes read and write
// consecutive doubles.  Planes start on 128-byte lines; a tile of whole rows
// whose first cell is not on a line shifts its slots by up to 15 (slots before
// the first cell idle), so that every wave covers whole lines.  Per block the
// tile covers whole rows, hy of them with ex * hy <= cap (cap - 15 for widths
// off the 16-cell grid, room for the shift), as long as the halo ring still
// has one loader thread per cell with that many rows (2 * (ex + hy) <= nt).
// Wider blocks are cut into tnx pieces of at most flat_max_x(nt) columns (each
// after the first starting on a 16-column boundary) and y into tny near-equal
// pieces of at most hy rows, with wx * hy <= cap and 2 * (wx + hy) <= nt, wx
// being the widest x piece.  Host and kernels evaluate the same functions.
struct FlatShape {
    int tnx, tny, wx, hy;
};
constexpr int flat_max_x(int nt) { return nt >= 512 ? 192 : nt / 2 - 32; }
constexpr FlatShape flat_shape(int ex, int ey, int nt, int cap)
{
    const int capw = ex % 16 ? cap - 15 : cap;  // whole rows: room for the alignment shift
    int tnx = 1, wx = ex, budget = capw;
    const int rows = capw / ex < ey ? capw / ex : ey;
    if (rows < 1 || nt / 2 - ex < rows) {  // the ring would limit whole rows: cut x
        const int mx = flat_max_x(nt);
        tnx = (ex + mx - 1) / mx;
        wx = tnx == 1 ? ex : (ex + tnx - 1) / tnx + 15;
        budget = tnx == 1 ? capw : cap;
    }
    int hy = budget / wx;
    if (nt / 2 - wx < hy) hy = nt / 2 - wx;
    if (ey < hy) hy = ey;
    if (hy < 1) hy = 1;
    return FlatShape{tnx, (ey + hy - 1) / hy, wx, hy};
}
constexpr int flat_x0(int ex, int tnx, int tx)
{
    return tx == 0 ? 0 : tx >= tnx ? ex : (int)(((int64_t)tx * ex / tnx) & ~(int64_t)15);
}

// Two sweeps per launch on grids of one block (j3d_twostep.hip).  A launch
// reads iterate t from one buffer and writes iterate t+2 to the other; x-y
// tiles of 64 x 16 cells (512 threads), z cut into near-equal pieces.
// Single grid: blocks == nullptr, the fields below `blocks` are unused.
// Multi-problem (batched) launch: tile_count tiles from tiles[tile_begin..];
// a tile's problem takes part while step < limit, reading buffer
// (base + step) & 1, and adds its residual when step + 1 == limit (ProbDesc
// counts launches here, not sweeps).
struct TwoStepArgs {
    const double *cur;        // field of iterate t (plane index 0: the z- ghost plane)
    double *nxt;              // field that receives iterate t+2
    const double *xh;         // x-halo arrays (x- then x+, ey*ez each, y fastest)
    unsigned long long *res;  // residual word(s) of the second sweep (bit pattern)
    int32_t ex, ey, ez, pitch;
    int32_t ntx, nty, ntz;
    int32_t want_res;
    const BlockDesc *blocks;  // multi-problem launch only
    const ProbDesc *probs;
    const Tile *tiles;
    double *base;
    int64_t step;
    int32_t tile_begin, tile_count, zchunk;
};
// Tile counts for a block and z-chunk (0 or >= ez: whole planes); returns the total.
int twostep_tiles(int ex, int ey, int ez, int zchunk, int *ntx, int *nty, int *ntz);
// Tiles of blocks b0..b1-1 for a multi-problem launch with z-chunks of zchunk planes.
void twostep_make_tiles(const BlockDesc *blocks, int32_t b0, int32_t b1, int zchunk, std::vector<Tile> *tiles);
int launch_twostep(const TwoStepArgs &a, void *stream);

// ---- launchers (defined in j3d_kernels.hip); all enqueue on `stream` ----------
// Every launcher returns 0 or a hipError_t value.

int launch_sweep(int variant, const SweepArgs &a, int grid, void *stream);
// Init: interior of parity `parity` from SplitMix64 state s0 (global dims n),
// halo storage of both parities: Dirichlet value on global faces, NaN elsewhere.
int launch_init(double *base, const BlockDesc *blocks, int32_t block_begin, int32_t nblocks,
                int32_t max_cells, int32_t max_xface, int parity, const int64_t n[3], uint64_t s0,
                const double bc[6], int write_interior, void *stream);
// Pack (faces in `face_mask`) of parity `parity` into send buffers.
int launch_pack(double *base, const BlockDesc *blocks, int32_t block_begin, int32_t nblocks,
                int32_t max_face, int parity, int face_mask, void *stream);
// Recompute the outer one-cell shell of each block (parity -> parity^1) from the
// current halo storage; max_shell bounds the shell cells of any block.
int launch_shell(double *base, const BlockDesc *blocks, int32_t block_begin, int32_t nblocks, int64_t max_shell,
                 int parity, void *stream);
// Exchange S[b][f] -> R[nbr][opp f] for all blocks in the range.
int launch_exchange(double *base, const BlockDesc *blocks, int32_t block_begin, int32_t nblocks,
                    int32_t max_face, void *stream);
// Unpack R[b][f] into the halo storage of parity `parity`.
int launch_unpack(double *base, const BlockDesc *blocks, int32_t block_begin, int32_t nblocks,
                  int32_t max_face, int parity, int face_mask, void *stream);
// Dense global array chunk (planes z0..z1-1) <-> block interiors of parity p.
// maps: for axis a, n[a] pairs (block coordinate, local coordinate).
int launch_scatter(double *base, const BlockDesc *blocks, int32_t block_base, const int32_t nb[3],
                   const int32_t *maps, const int64_t n[3], int64_t z0, int64_t z1,
                   const double *src, int parity, void *stream);
int launch_gather(const double *base, const BlockDesc *blocks, int32_t block_base,
                  const int32_t nb[3], const int32_t *maps, const int64_t n[3], int64_t z0,
                  int64_t z1, double *dst, int parity, void *stream);
// Per-cell Dirichlet face f from a dense device array into both parities.
int launch_set_face(double *base, const BlockDesc *blocks, int32_t block_base, const int32_t nb[3],
                    const int32_t *maps, const int64_t n[3], int face, const double *src,
                    void *stream);
int launch_fill_u64(unsigned long long *p, int64_t count, unsigned long long value, void *stream);
int launch_fill_u32(unsigned int *p, int64_t count, unsigned int value, void *stream);
int launch_copy(void *dst, const void *src, uint64_t bytes, void *stream);
// Dense interior of one single-block problem gathered into `dst` (device).
int launch_gather_block(const double *base, const BlockDesc *blocks, int32_t block, int parity,
                        double *dst, void *stream);

}  // namespace j3d
