// j3d_host.hpp -- host-side planning shared by the solver, batch and pool.
//
// Planning is pure host code (no HIP calls): it resolves each problem's
// decomposition (Sec. IV-A), builds the block table with its neighbour links
// (the 3-D chare array of Fig. 3 and its idx[dir] proxies, as plain indices),
// assigns every array its place in the caller's arena, and cuts blocks into
// sweep tiles.
#pragma once

#include <algorithm>
#include <cstdint>
#include <string>
#include <vector>

#include "j3d_internal.hpp"

namespace j3d {

// ---- errors --------------------------------------------------------------------

j3d_status set_error(j3d_status st, const char *fmt, ...);
void clear_error();

// ---- host SplitMix64 (start state of a problem's stream) -----------------------

// The (pid+1)-th output of SplitMix64 started in state `seed`.
uint64_t stream_start(uint64_t seed, uint64_t pid);

// ---- decomposition -------------------------------------------------------------

struct Decomp {
    int64_t n[3];
    int32_t nb[3];
    std::vector<int64_t> ext[3];  // block extents per axis
    std::vector<int64_t> org[3];  // block origins per axis
};

j3d_status resolve_decomp(const j3d_problem *p, Decomp *d);
j3d_status auto_split(const int64_t n[3], int32_t parts, int32_t nb[3]);

// ---- arena plan ----------------------------------------------------------------

struct ProbPlan {
    Decomp d;
    double bc[6];
    uint64_t s0;
    int32_t block_begin = 0, nblocks = 0;
    uint64_t maps_off = 0;        // bytes: int32 pairs, x then y then z
    uint64_t field_cells = 0;     // doubles of one parity's fields (all blocks)
    uint64_t f_off[2] = {0, 0};   // bytes: start of the problem's fields per parity
    int64_t iters = 0;            // batch: sweeps to run
};

struct Plan {
    std::vector<BlockDesc> blocks;
    std::vector<ProbPlan> probs;
    bool with_sr = true;          // send/receive buffers of the unfused modes
    uint64_t off_blocks = 0, off_probs = 0, off_tiles = 0, off_res = 0, off_queue = 0;
    uint64_t off_bounce = 0, bounce_doubles = 0;
    uint64_t tiles_cap = 0;
    uint64_t total = 0;           // arena bytes
    int32_t max_face = 0;         // largest face (cells) over all blocks
    int32_t max_cells = 0;        // largest ghosted field (cells) over all blocks
};

// Plan `count` problems; the bounce area holds at least min_bounce doubles
// (and at least the largest plane and face of every problem).
j3d_status make_plan(int32_t count, const j3d_problem *probs, bool with_sr, Plan *plan);

// Fills each block's fused-sweep halo sources and x-face targets (fx_*, fy_*,
// fz_*) from its neighbour links and the neighbours' offsets; -1 where a face
// has no neighbour.  Every block table the sweep reads must pass through it
// once its offsets are final (the planner's and the pool's).
inline void link_halo_sources(BlockDesc *blocks, size_t count)
{
    for (size_t b = 0; b < count; ++b) {
        BlockDesc &B = blocks[b];
        const int64_t ey = B.ext[1], ez = B.ext[2], pitch = B.pitch;
        const int64_t ps = plane_stride(pitch, ey);
        B.fy_step[0] = B.fy_step[1] = 0;
        for (int q = 0; q < 2; ++q) {
            B.fx_m[q] = B.fx_p[q] = B.fy_m[q] = B.fy_p[q] = B.fz_m[q] = B.fz_p[q] = -1;
            if (B.nbr[0] >= 0) B.fx_m[q] = blocks[B.nbr[0]].xoff[q] + ey * ez;
            if (B.nbr[1] >= 0) B.fx_p[q] = blocks[B.nbr[1]].xoff[q];
            if (B.nbr[2] >= 0) {
                const BlockDesc &N = blocks[B.nbr[2]];
                const int64_t psn = plane_stride(pitch, N.ext[1]);
                B.fy_m[q] = N.off[q] + psn + (int64_t)N.ext[1] * pitch;
                B.fy_step[0] = psn;
            }
            if (B.nbr[3] >= 0) {
                const BlockDesc &N = blocks[B.nbr[3]];
                const int64_t psn = plane_stride(pitch, N.ext[1]);
                B.fy_p[q] = N.off[q] + psn + pitch;
                B.fy_step[1] = psn;
            }
            if (B.nbr[4] >= 0) {
                const BlockDesc &N = blocks[B.nbr[4]];
                B.fz_m[q] = N.off[q] + (int64_t)N.ext[2] * ps;
            }
            if (B.nbr[5] >= 0) B.fz_p[q] = blocks[B.nbr[5]].off[q] + ps;
        }
    }
}

// Tiles of blocks [b0, b1) for a variant and z-chunk (0 = whole block), block
// by block, z then y then x slowest to fastest, each with the cells it covers.
void make_tiles(const Plan &plan, int32_t b0, int32_t b1, int variant, int zchunk,
                std::vector<Tile> *tiles, std::vector<int32_t> *block_first);

// Prefix sums of the estimated time of each tile (the planes it reads, plus
// one for its first memory latency): prefix[i] covers tiles [0, i).
void tile_work(const std::vector<Tile> &tiles, std::vector<uint64_t> *prefix);

// Cuts tiles [t0, t0+cnt) into one contiguous range per XCD of about equal
// work (SweepArgs::xcut) and returns the grid that covers the longest range
// (kXcdCount workgroups per range index).  Launches too small to matter keep
// equal counts: xcut stays zero and the grid is cnt.
inline int xcd_split(const std::vector<uint64_t> &prefix, int32_t t0, int32_t cnt, int32_t *xcut)
{
    for (int x = 0; x <= kXcdCount; ++x) xcut[x] = 0;
    // below a few tiles per compute unit the launch is short and equal counts do
    if (cnt < 4 * 256 || prefix.size() < (size_t)t0 + cnt + 1) return cnt;
    const uint64_t w0 = prefix[t0], total = prefix[t0 + cnt] - w0;
    int longest = 0;
    for (int x = 1; x <= kXcdCount; ++x) {
        int32_t c = cnt;
        if (x < kXcdCount) {
            // first tile boundary at or past the target, or the one before if nearer
            const uint64_t target = w0 + (uint64_t)((__uint128_t)total * x / kXcdCount);
            const auto it = std::lower_bound(prefix.begin() + t0, prefix.begin() + t0 + cnt + 1, target);
            c = (int32_t)(it - (prefix.begin() + t0));
            if (c > 0 && target - prefix[t0 + c - 1] < prefix[t0 + c] - target) --c;
            c = std::max(c, xcut[x - 1]);
        }
        xcut[x] = c;
        longest = std::max(longest, xcut[x] - xcut[x - 1]);
    }
    return kXcdCount * std::max(longest, 1);
}

// Default sweep shape for the blocks of a plan.
void default_tune(const Plan &plan, int cus, j3d_tune *t);

// Number of tiles that variant/zchunk give over the blocks of a plan.
uint64_t count_tiles(const Plan &plan, int variant, int zchunk);
// Index of the fixed-tile variant of this shape, or of the flattened variant
// with this thread count, cell capacity and prefetch depth; -1 if none.
int find_variant(int tile_x, int tile_y, int threads);
int find_flat_variant(int threads, int cells, int prefetch);
// Tiles of a block's x-y plane under variant vi: ntx along x, nty along y.
inline void tiles_xy(const VariantInfo &vi, int64_t ex, int64_t ey, int64_t *ntx, int64_t *nty)
{
    if (vi.tile_x == 0) {
        const FlatShape s = flat_shape((int)ex, (int)ey, vi.threads, vi.tile_y);
        *ntx = s.tnx;
        *nty = s.tny;
    } else {
        *ntx = (ex + vi.tile_x - 1) / vi.tile_x;
        *nty = (ey + vi.tile_y - 1) / vi.tile_y;
    }
}

// Validates a tune against a plan; fills the effective z-chunk.
j3d_status check_tune(const Plan &plan, const j3d_tune *t, int *zchunk_eff);

// Row stride of a block's field in doubles: rows are stored unpadded, so the
// rows of a plane form one contiguous run and a tile of whole rows reads and
// writes one run per plane (no padding bytes move, no line is half used
// except where two tiles meet).
inline int64_t row_pitch(int64_t ex) { return ex; }

// Cells of one block's field (one parity), halos included.
inline int64_t block_field_cells(int64_t ex, int64_t ey, int64_t ez)
{
    return plane_stride(row_pitch(ex), ey) * (ez + 2);
}

inline uint64_t align_up(uint64_t v, uint64_t a) { return (v + a - 1) / a * a; }

constexpr int kMinZchunk = 4;

}  // namespace j3d
