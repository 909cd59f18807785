// j3d_pool.cpp -- served form: continuous batching of Jacobi3D solves on one GPU.
//
// Requests are admitted while others run, as long as a slot and enough of the
// HBM budget are free; their grids stay resident in the arena.  A round is a
// few fused sweeps (one launch per sweep) over the tiles of every running
// request; each request advances at its own pace and parity.  A residual is
// evaluated at every check point (every check_every sweeps and at the last);
// a round never carries a request past its next check point, so the early
// exit (residual <= tol) is decided at exactly that sweep.  Finished requests
// are gathered into their free buffer and copied to host memory on a second
// stream while later rounds run.  This form is not in the paper; it reuses the
// paper's fused update (Sec. III-D-1) as its compute step and its asynchronous
// completion detection by polling events (Sec. III-A) for retirement.
#include <algorithm>
#include <cstring>
#include <map>
#include <new>

#include "j3d_device.hpp"

using namespace j3d;

namespace {

// 64x32 tiles of 256 threads and 32-plane z-chunks: enough workgroups per
// request that a round of a few mid-sized requests fills the GPU
constexpr int kPoolZchunk = 32;
constexpr int kPoolTwoZchunk = 64;  // z-chunk of the two-sweep rounds
constexpr int64_t kPoolTilesPerReq = 4096;

enum ReqState { R_FREE = 0, R_RUNNING, R_COPYING, R_DONE, R_REPORTED };

struct Req {
    int state = R_FREE;
    uint32_t gen = 0;
    uint64_t region = 0, bytes = 0;
    BlockDesc blk;
    int64_t n[3] = {0, 0, 0};
    int64_t iters_done = 0, max_iters = 0;
    double tol = 0.0, residual = 0.0;
    int32_t check_every = 0;
    int32_t waited = 0;  // consecutive rounds this request was left out of
    int buf = 0;         // field buffer holding the current iterate
    double *host_result = nullptr;
    hipEvent_t gather_ev = nullptr, copy_ev = nullptr;
};

struct RoundEntry {
    int32_t slot;
    uint32_t gen;
    int64_t base, limit;
    int newbuf;  // buffer of the iterate after the round
};

struct Layout {
    uint64_t off_blocks, off_probs, off_tiles, off_res, off_queue, total;
};

Layout pool_layout(int32_t max_slots)
{
    Layout l;
    uint64_t o = 0;
    l.off_blocks = o;
    o = align_up(o + (uint64_t)max_slots * sizeof(BlockDesc), 256);
    l.off_probs = o;
    o = align_up(o + (uint64_t)max_slots * sizeof(ProbDesc), 256);
    l.off_tiles = o;
    o = align_up(o + (uint64_t)max_slots * kPoolTilesPerReq * sizeof(Tile), 256);
    l.off_res = o;
    o = align_up(o + (uint64_t)max_slots * sizeof(uint64_t), 256);
    l.off_queue = o;
    o = align_up(o + 16 * sizeof(uint32_t), 4096);
    l.total = o;
    return l;
}

// Requests come in every width, so rounds use flattened tiles (512 threads,
// 4 cells each: rows of any width, whole cache lines written at row ends).
int pool_variant()
{
    const int v = find_flat_variant(512, 2048, 1);
    return v >= 0 ? v : 0;
}

// Single-block request geometry and bytes.
j3d_status request_geometry(const j3d_problem *p, Decomp *d, uint64_t *bytes)
{
    j3d_status st = resolve_decomp(p, d);
    if (st != J3D_OK) return st;
    if (d->nb[0] * d->nb[1] * d->nb[2] != 1)
        return set_error(J3D_EINVAL, "pool requests are single-block problems (got %dx%dx%d blocks)", d->nb[0],
                         d->nb[1], d->nb[2]);
    const uint64_t cells = (uint64_t)block_field_cells(d->n[0], d->n[1], d->n[2]);
    const uint64_t xc = 2ull * d->n[1] * d->n[2];
    *bytes = 2 * align_up(cells * sizeof(double), 4096) + 2 * align_up(xc * sizeof(double), 4096);
    return J3D_OK;
}

}  // namespace

struct j3d_pool {
    char *arena = nullptr;
    uint64_t arena_bytes = 0, budget_off = 0, budget = 0, used = 0;
    int32_t max_slots = 0;
    hipStream_t stream = nullptr, copy_stream = nullptr;
    Layout lay{};
    int variant = 0, zchunk = kPoolZchunk, cus = 256;
    std::vector<Req> reqs;
    std::map<uint64_t, uint64_t> free_ranges;  // offset -> size, within the budget
    bool round_busy = false;
    int32_t round_sweeps = 0;
    hipEvent_t round_ev = nullptr;
    std::vector<RoundEntry> round;
    unsigned long long *host_res = nullptr;  // page-locked
    ProbDesc *host_probs = nullptr;
    Tile *host_tiles = nullptr;
    BlockDesc *host_blocks = nullptr;
    std::vector<int32_t> ready;
    // round policy: shortest remaining work first until the round holds at
    // least fill_cells cells (0: every running request joins every round);
    // a request left out of max_wait consecutive rounds joins first
    int64_t fill_cells = int64_t(1) << 25;
    int32_t max_wait = 32;
    int32_t backlog_share = 2;  // > 0: the target is at least 1/backlog_share of the running cells
    // two sweeps per launch: tables of the pair launches (page-locked, apart
    // from the single-sweep ones, which are still in flight when these are filled)
    bool two_sweep = false;
    ProbDesc *host_probs2 = nullptr;
    Tile *host_tiles2 = nullptr;
};

namespace {

bool alloc_range(j3d_pool *pl, uint64_t bytes, uint64_t *off)
{
    for (auto it = pl->free_ranges.begin(); it != pl->free_ranges.end(); ++it) {
        if (it->second >= bytes) {
            *off = it->first;
            const uint64_t rest = it->second - bytes;
            const uint64_t at = it->first + bytes;
            pl->free_ranges.erase(it);
            if (rest) pl->free_ranges[at] = rest;
            return true;
        }
    }
    return false;
}

void free_range(j3d_pool *pl, uint64_t off, uint64_t bytes)
{
    auto it = pl->free_ranges.emplace(off, bytes).first;
    auto next = std::next(it);
    if (next != pl->free_ranges.end() && it->first + it->second == next->first) {
        it->second += next->second;
        pl->free_ranges.erase(next);
    }
    if (it != pl->free_ranges.begin()) {
        auto prev = std::prev(it);
        if (prev->first + prev->second == it->first) {
            prev->second += it->second;
            pl->free_ranges.erase(it);
        }
    }
}

SweepArgs pool_args(j3d_pool *pl)
{
    SweepArgs a;
    std::memset(&a, 0, sizeof a);
    a.base = reinterpret_cast<double *>(pl->arena);
    a.blocks = reinterpret_cast<const BlockDesc *>(pl->arena + pl->lay.off_blocks);
    a.probs = reinterpret_cast<const ProbDesc *>(pl->arena + pl->lay.off_probs);
    a.tiles = reinterpret_cast<const Tile *>(pl->arena + pl->lay.off_tiles);
    a.res = reinterpret_cast<unsigned long long *>(pl->arena + pl->lay.off_res);
    a.queue = reinterpret_cast<unsigned int *>(pl->arena + pl->lay.off_queue);
    a.zchunk = pl->zchunk;
    a.flags = SW_FUSED | SW_MULTI;
    return a;
}

// Gather the finished request's interior into its free buffer and copy it to
// the host on the copy stream.
j3d_status start_copy(j3d_pool *pl, int32_t slot)
{
    Req &r = pl->reqs[slot];
    const int p = r.buf;
    double *dst = reinterpret_cast<double *>(pl->arena) + r.blk.off[p ^ 1];
    j3d_status st = hip_status(
        launch_gather_block(reinterpret_cast<double *>(pl->arena),
                            reinterpret_cast<const BlockDesc *>(pl->arena + pl->lay.off_blocks), slot, p, dst,
                            pl->stream),
        "result gather");
    if (st != J3D_OK) return st;
    st = hip_status(hipEventRecord(r.gather_ev, pl->stream), "gather event");
    if (st != J3D_OK) return st;
    st = hip_status(hipStreamWaitEvent(pl->copy_stream, r.gather_ev, 0), "copy wait");
    if (st != J3D_OK) return st;
    // without a host buffer the gathered interior waits in the free buffer
    // until j3d_pool_fetch or release
    if (r.host_result) {
        const size_t bytes = (size_t)(r.n[0] * r.n[1] * r.n[2]) * sizeof(double);
        st = hip_status(hipMemcpyAsync(r.host_result, dst, bytes, hipMemcpyDeviceToHost, pl->copy_stream),
                        "result copy");
        if (st != J3D_OK) return st;
    }
    st = hip_status(hipEventRecord(r.copy_ev, pl->copy_stream), "copy event");
    if (st != J3D_OK) return st;
    r.state = R_COPYING;
    return J3D_OK;
}

}  // namespace

extern "C" {

j3d_status j3d_pool_request_bytes(const j3d_problem *p, uint64_t *bytes)
{
    if (!bytes) return set_error(J3D_EINVAL, "bytes is NULL");
    Decomp d;
    return request_geometry(p, &d, bytes);
}

j3d_status j3d_pool_overhead_bytes(int32_t max_slots, uint64_t *bytes)
{
    if (!bytes) return set_error(J3D_EINVAL, "bytes is NULL");
    if (max_slots < 1 || max_slots > 65536) return set_error(J3D_EINVAL, "max_slots %d out of range", max_slots);
    *bytes = pool_layout(max_slots).total;
    return J3D_OK;
}

j3d_status j3d_pool_create(void *dev_arena, uint64_t arena_bytes, uint64_t budget_bytes, int32_t max_slots,
                           void *hip_stream, j3d_pool **out)
{
    if (!out || !dev_arena) return set_error(J3D_EINVAL, "NULL argument");
    if (reinterpret_cast<uintptr_t>(dev_arena) % 256) return set_error(J3D_EINVAL, "arena not 256-byte aligned");
    if (max_slots < 1 || max_slots > 65536) return set_error(J3D_EINVAL, "max_slots %d out of range", max_slots);
    const Layout lay = pool_layout(max_slots);
    if (budget_bytes == 0) return set_error(J3D_EINVAL, "budget is 0");
    if (arena_bytes < lay.total + budget_bytes)
        return set_error(J3D_ENOMEM, "arena holds %llu bytes, %llu needed", (unsigned long long)arena_bytes,
                         (unsigned long long)(lay.total + budget_bytes));
    int dev = 0, cus = 0;
    j3d_status st = require_device(&dev, &cus);
    if (st != J3D_OK) return st;
    j3d_pool *pl = new (std::nothrow) j3d_pool();
    if (!pl) return set_error(J3D_EINVAL, "out of host memory");
    pl->arena = static_cast<char *>(dev_arena);
    pl->arena_bytes = arena_bytes;
    pl->lay = lay;
    pl->budget_off = lay.total;
    pl->budget = budget_bytes;
    pl->max_slots = max_slots;
    pl->stream = static_cast<hipStream_t>(hip_stream);
    pl->variant = pool_variant();
    pl->cus = cus;
    pl->reqs.resize(max_slots);
    pl->free_ranges[pl->budget_off] = budget_bytes;
    st = hip_status(hipStreamCreateWithFlags(&pl->copy_stream, hipStreamNonBlocking), "copy stream");
    if (st == J3D_OK) st = hip_status(hipEventCreateWithFlags(&pl->round_ev, hipEventDisableTiming), "event");
    for (int32_t i = 0; i < max_slots && st == J3D_OK; ++i) {
        st = hip_status(hipEventCreateWithFlags(&pl->reqs[i].gather_ev, hipEventDisableTiming), "event");
        if (st == J3D_OK)
            st = hip_status(hipEventCreateWithFlags(&pl->reqs[i].copy_ev, hipEventDisableTiming), "event");
    }
    if (st == J3D_OK)
        st = hip_status(hipHostMalloc((void **)&pl->host_res, max_slots * sizeof(unsigned long long), 0),
                        "pinned residuals");
    if (st == J3D_OK)
        st = hip_status(hipHostMalloc((void **)&pl->host_probs, max_slots * sizeof(ProbDesc), 0), "pinned table");
    if (st == J3D_OK)
        st = hip_status(hipHostMalloc((void **)&pl->host_blocks, max_slots * sizeof(BlockDesc), 0),
                        "pinned table");
    if (st == J3D_OK)
        st = hip_status(
            hipHostMalloc((void **)&pl->host_tiles, (size_t)max_slots * kPoolTilesPerReq * sizeof(Tile), 0),
            "pinned table");
    if (st == J3D_OK)
        st = hip_status(launch_fill_u32(reinterpret_cast<unsigned int *>(pl->arena + lay.off_queue), 16, 0,
                                        pl->stream),
                        "queue init");
    if (st != J3D_OK) {
        j3d_pool_destroy(pl);
        return st;
    }
    *out = pl;
    return J3D_OK;
}

j3d_status j3d_pool_admit(j3d_pool *pl, const j3d_problem *p, int64_t max_iters, double tol,
                          int32_t check_every, double *host_result, int32_t *slot)
{
    if (!pl || !p || !slot) return set_error(J3D_EINVAL, "NULL argument");
    if (max_iters < 0) return set_error(J3D_EINVAL, "max_iters %lld < 0", (long long)max_iters);
    if (check_every < 0) return set_error(J3D_EINVAL, "check_every %d < 0", check_every);
    Decomp d;
    uint64_t bytes = 0;
    j3d_status st = request_geometry(p, &d, &bytes);
    if (st != J3D_OK) return st;
    const VariantInfo vi = variant_info(pl->variant);
    int64_t ntx, nty;
    tiles_xy(vi, d.n[0], d.n[1], &ntx, &nty);
    const int64_t tiles = ntx * nty * ((d.n[2] + pl->zchunk - 1) / pl->zchunk);
    int tx2 = 0, ty2 = 0, tz2 = 0;
    const int64_t tiles2 = pl->two_sweep ? twostep_tiles((int)d.n[0], (int)d.n[1], (int)d.n[2], kPoolTwoZchunk,
                                                         &tx2, &ty2, &tz2)
                                         : 0;
    if (tiles > kPoolTilesPerReq || tiles2 > kPoolTilesPerReq)
        return set_error(J3D_EINVAL, "request of %lldx%lldx%lld needs %lld tiles, more than %lld",
                         (long long)d.n[0], (long long)d.n[1], (long long)d.n[2],
                         (long long)std::max(tiles, tiles2), (long long)kPoolTilesPerReq);
    int32_t s = -1;
    for (int32_t i = 0; i < pl->max_slots; ++i)
        if (pl->reqs[i].state == R_FREE) {
            s = i;
            break;
        }
    if (s < 0) return set_error(J3D_EBUSY, "all %d slots are in use", pl->max_slots);
    uint64_t region = 0;
    if (!alloc_range(pl, bytes, &region))
        return set_error(J3D_EBUDGET, "%llu bytes requested, %llu of %llu in use (fragmented or full)",
                         (unsigned long long)bytes, (unsigned long long)pl->used, (unsigned long long)pl->budget);
    Req &r = pl->reqs[s];
    r.gen++;
    r.region = region;
    r.bytes = bytes;
    std::memset(&r.blk, 0, sizeof r.blk);
    const int64_t cells = block_field_cells(d.n[0], d.n[1], d.n[2]);
    const uint64_t fbytes = align_up((uint64_t)cells * sizeof(double), 4096);
    const uint64_t xbytes = align_up(2ull * d.n[1] * d.n[2] * sizeof(double), 4096);
    r.blk.off[0] = (int64_t)(region / sizeof(double));
    r.blk.off[1] = (int64_t)((region + fbytes) / sizeof(double));
    r.blk.xoff[0] = (int64_t)((region + 2 * fbytes) / sizeof(double));
    r.blk.xoff[1] = (int64_t)((region + 2 * fbytes + xbytes) / sizeof(double));
    for (int a = 0; a < 3; ++a) {
        r.blk.ext[a] = (int32_t)d.n[a];
        r.n[a] = d.n[a];
    }
    for (int f = 0; f < 6; ++f) r.blk.nbr[f] = -1;
    r.blk.pitch = (int32_t)row_pitch(d.n[0]);
    r.blk.prob = s;
    r.blk.face_total = 2 * (d.n[1] * d.n[2] + d.n[0] * d.n[2] + d.n[0] * d.n[1]);
    link_halo_sources(&r.blk, 1);  // one block, no neighbours: every face reads the own ghost layer
    r.iters_done = 0;
    r.buf = 0;
    r.max_iters = max_iters;
    r.tol = tol;
    r.check_every = check_every;
    r.residual = 0.0;
    r.waited = 0;
    r.host_result = host_result;
    pl->host_blocks[s] = r.blk;
    BlockDesc *dblk = reinterpret_cast<BlockDesc *>(pl->arena + pl->lay.off_blocks);
    st = hip_status(hipMemcpyAsync(dblk + s, &pl->host_blocks[s], sizeof(BlockDesc), hipMemcpyHostToDevice,
                                   pl->stream),
                    "admit upload");
    if (st == J3D_OK)
        st = hip_status(launch_init(reinterpret_cast<double *>(pl->arena), dblk, s, 1, (int32_t)cells,
                                    (int32_t)(d.n[1] * d.n[2]), 0, d.n, stream_start(p->seed, p->pid), p->bc, 1,
                                    pl->stream),
                        "admit init");
    if (st != J3D_OK) {
        free_range(pl, region, bytes);
        return st;
    }
    pl->used += bytes;
    r.state = R_RUNNING;
    if (max_iters == 0) {
        st = start_copy(pl, s);
        if (st != J3D_OK) return st;
    }
    *slot = s;
    return J3D_OK;
}

j3d_status j3d_pool_step(j3d_pool *pl, int32_t sweeps)
{
    if (!pl) return set_error(J3D_EINVAL, "pool is NULL");
    if (sweeps < 1) return set_error(J3D_EINVAL, "sweeps %d < 1", sweeps);
    if (pl->round_busy) return set_error(J3D_ESTATE, "a round is still in flight");
    pl->round.clear();
    std::vector<Tile> tiles;
    // choose this round's requests
    struct Cand {
        bool starving;
        double remaining;  // cell-sweeps left
        int32_t slot;
    };
    std::vector<Cand> cands;
    for (int32_t s = 0; s < pl->max_slots; ++s) {
        const Req &r = pl->reqs[s];
        if (r.state != R_RUNNING) continue;
        cands.push_back(Cand{r.waited >= pl->max_wait,
                             (double)(r.max_iters - r.iters_done) * (double)(r.n[0] * r.n[1] * r.n[2]), s});
    }
    std::sort(cands.begin(), cands.end(), [](const Cand &a, const Cand &b) {
        if (a.starving != b.starving) return a.starving;
        if (a.remaining != b.remaining) return a.remaining < b.remaining;
        return a.slot < b.slot;
    });
    std::vector<char> chosen(pl->max_slots, 0);
    int64_t target = pl->fill_cells;
    if (target > 0 && pl->backlog_share > 0) {
        // under a backlog, larger rounds: fewer, longer launches serve more cells per second
        int64_t running = 0;
        for (const Cand &c : cands) {
            const Req &r = pl->reqs[c.slot];
            running += r.n[0] * r.n[1] * r.n[2];
        }
        target = std::max(target, running / pl->backlog_share);
    }
    int64_t cells = 0;
    for (const Cand &c : cands) {
        if (target > 0 && cells >= target) break;
        chosen[c.slot] = 1;
        const Req &r = pl->reqs[c.slot];
        cells += r.n[0] * r.n[1] * r.n[2];
    }
    for (const Cand &c : cands) {
        Req &r = pl->reqs[c.slot];
        r.waited = chosen[c.slot] ? 0 : r.waited + 1;
    }
    // Per chosen request: k sweeps this round (up to its next residual check).
    // One sweep per launch: step j advances every request with j < k.  Two
    // sweeps per launch: a request with odd k first takes one ordinary sweep
    // (one launch for the round), then k / 2 two-sweep launches; descriptors
    // then carry buffer parities instead of sweep counts.
    std::vector<Tile> tiles2;
    bool any_odd = false;
    int64_t max_pairs = 0;
    for (int32_t s = 0; s < pl->max_slots; ++s) {
        Req &r = pl->reqs[s];
        if (r.state != R_RUNNING || !chosen[s]) continue;
        const int64_t base = r.iters_done;
        int64_t limit = r.max_iters;
        if (r.check_every > 0) limit = std::min(limit, (base / r.check_every + 1) * r.check_every);
        const int64_t k = std::max<int64_t>(0, std::min<int64_t>(sweeps, limit - base));
        ProbDesc &pd = pl->host_probs[s];
        std::memset(&pd, 0, sizeof pd);
        pd.res_slot = s;
        int newbuf;
        if (!pl->two_sweep) {
            pd.base = base;
            pd.limit = limit;
            pd.flags = PF_RES_LAST;
            newbuf = (int)((base + k) & 1);
        } else {
            pd.base = r.buf;
            pd.limit = r.buf + (k & 1);
            pd.flags = k == 1 ? PF_RES_LAST : 0;
            ProbDesc &q = pl->host_probs2[s];
            std::memset(&q, 0, sizeof q);
            q.base = r.buf ^ (int)(k & 1);
            q.limit = k / 2;
            q.res_slot = s;
            newbuf = r.buf ^ (int)(k & 1) ^ (int)((k / 2) & 1);
            any_odd = any_odd || (k & 1) != 0;
            max_pairs = std::max<int64_t>(max_pairs, k / 2);
            const size_t at = tiles2.size();
            twostep_make_tiles(&r.blk, 0, 1, kPoolTwoZchunk, &tiles2);
            for (size_t i = at; i < tiles2.size(); ++i) tiles2[i].block = s;
        }
        pl->round.push_back(RoundEntry{s, r.gen, base, limit, newbuf});
        Plan one;
        one.blocks.assign(1, r.blk);
        std::vector<Tile> t;
        make_tiles(one, 0, 1, pl->variant, pl->zchunk, &t, nullptr);
        for (Tile &x : t) x.block = s;
        tiles.insert(tiles.end(), t.begin(), t.end());
    }
    if (pl->round.empty()) return J3D_OK;
    std::memcpy(pl->host_tiles, tiles.data(), tiles.size() * sizeof(Tile));
    j3d_status st = hip_status(hipMemcpyAsync(pl->arena + pl->lay.off_probs, pl->host_probs,
                                              pl->max_slots * sizeof(ProbDesc), hipMemcpyHostToDevice, pl->stream),
                               "round upload");
    if (st == J3D_OK)
        st = hip_status(hipMemcpyAsync(pl->arena + pl->lay.off_tiles, pl->host_tiles, tiles.size() * sizeof(Tile),
                                       hipMemcpyHostToDevice, pl->stream),
                        "round upload");
    unsigned long long *res = reinterpret_cast<unsigned long long *>(pl->arena + pl->lay.off_res);
    if (st == J3D_OK) st = hip_status(launch_fill_u64(res, pl->max_slots, 0ull, pl->stream), "residual reset");
    SweepArgs a = pool_args(pl);
    a.tile_begin = 0;
    a.tile_count = (int32_t)tiles.size();
    std::vector<uint64_t> work;
    tile_work(tiles, &work);
    const int grid = xcd_split(work, 0, a.tile_count, a.xcut);
    const int32_t one_sweep_launches = pl->two_sweep ? (any_odd ? 1 : 0) : sweeps;
    for (int32_t j = 0; j < one_sweep_launches && st == J3D_OK; ++j) {
        a.step = j;
        st = hip_status(launch_sweep(pl->variant, a, grid, pl->stream), "round sweep");
    }
    if (st == J3D_OK && max_pairs > 0) {
        // the pair launches' tables replace the single sweep's, in stream order
        std::memcpy(pl->host_tiles2, tiles2.data(), tiles2.size() * sizeof(Tile));
        st = hip_status(hipMemcpyAsync(pl->arena + pl->lay.off_probs, pl->host_probs2,
                                       pl->max_slots * sizeof(ProbDesc), hipMemcpyHostToDevice, pl->stream),
                        "round upload");
        if (st == J3D_OK)
            st = hip_status(hipMemcpyAsync(pl->arena + pl->lay.off_tiles, pl->host_tiles2,
                                           tiles2.size() * sizeof(Tile), hipMemcpyHostToDevice, pl->stream),
                            "round upload");
        TwoStepArgs a2;
        std::memset(&a2, 0, sizeof a2);
        a2.base = reinterpret_cast<double *>(pl->arena);
        a2.blocks = reinterpret_cast<const BlockDesc *>(pl->arena + pl->lay.off_blocks);
        a2.probs = reinterpret_cast<const ProbDesc *>(pl->arena + pl->lay.off_probs);
        a2.tiles = reinterpret_cast<const Tile *>(pl->arena + pl->lay.off_tiles);
        a2.res = res;
        a2.zchunk = kPoolTwoZchunk;
        a2.tile_begin = 0;
        a2.tile_count = (int32_t)tiles2.size();
        for (int64_t s2 = 0; s2 < max_pairs && st == J3D_OK; ++s2) {
            a2.step = s2;
            st = hip_status(launch_twostep(a2, pl->stream), "round two-sweep launch");
        }
    }
    if (st == J3D_OK)
        st = hip_status(hipMemcpyAsync(pl->host_res, res, pl->max_slots * sizeof(unsigned long long),
                                       hipMemcpyDeviceToHost, pl->stream),
                        "residual readback");
    if (st == J3D_OK) st = hip_status(hipEventRecord(pl->round_ev, pl->stream), "round event");
    if (st != J3D_OK) return st;
    pl->round_busy = true;
    pl->round_sweeps = sweeps;
    return J3D_OK;
}

j3d_status j3d_pool_poll(j3d_pool *pl, int32_t *done, int32_t cap, int32_t *n_done, int32_t *round_busy)
{
    if (!pl || !n_done || (cap > 0 && !done)) return set_error(J3D_EINVAL, "NULL argument");
    if (pl->round_busy) {
        const hipError_t q = hipEventQuery(pl->round_ev);
        if (q == hipSuccess) {
            for (const RoundEntry &e : pl->round) {
                Req &r = pl->reqs[e.slot];
                if (r.state != R_RUNNING || r.gen != e.gen) continue;  // released meanwhile
                const int64_t adv = std::min<int64_t>(pl->round_sweeps, e.limit - e.base);
                r.iters_done = e.base + adv;
                r.buf = e.newbuf;
                if (r.iters_done == e.limit) {
                    double v;
                    std::memcpy(&v, &pl->host_res[e.slot], sizeof v);
                    r.residual = v;
                    const bool fin = r.iters_done == r.max_iters || (r.tol > 0.0 && r.residual <= r.tol);
                    if (fin) {
                        j3d_status st = start_copy(pl, e.slot);
                        if (st != J3D_OK) return st;
                    }
                }
            }
            pl->round_busy = false;
        } else if (q != hipErrorNotReady) {
            return hip_status(q, "round event");
        }
    }
    for (int32_t s = 0; s < pl->max_slots; ++s) {
        Req &r = pl->reqs[s];
        if (r.state != R_COPYING) continue;
        const hipError_t q = hipEventQuery(r.copy_ev);
        if (q == hipSuccess) {
            r.state = R_DONE;
            pl->ready.push_back(s);
        } else if (q != hipErrorNotReady) {
            return hip_status(q, "copy event");
        }
    }
    int32_t n = 0;
    while (n < cap && !pl->ready.empty()) {
        const int32_t s = pl->ready.front();
        pl->ready.erase(pl->ready.begin());
        if (pl->reqs[s].state != R_DONE) continue;
        pl->reqs[s].state = R_REPORTED;
        done[n++] = s;
    }
    *n_done = n;
    if (round_busy) *round_busy = pl->round_busy ? 1 : 0;
    return J3D_OK;
}

j3d_status j3d_pool_result(j3d_pool *pl, int32_t slot, double *residual, int64_t *iters_done)
{
    if (!pl) return set_error(J3D_EINVAL, "pool is NULL");
    if (slot < 0 || slot >= pl->max_slots) return set_error(J3D_EINVAL, "slot %d out of range", slot);
    const Req &r = pl->reqs[slot];
    if (r.state != R_DONE && r.state != R_REPORTED) return set_error(J3D_ESTATE, "slot %d has no result", slot);
    if (residual) *residual = r.residual;
    if (iters_done) *iters_done = r.iters_done;
    return J3D_OK;
}

j3d_status j3d_pool_fetch(j3d_pool *pl, int32_t slot, double *host_dst, double *residual, int64_t *iters_done)
{
    if (!pl) return set_error(J3D_EINVAL, "pool is NULL");
    if (slot < 0 || slot >= pl->max_slots) return set_error(J3D_EINVAL, "slot %d out of range", slot);
    const Req &r = pl->reqs[slot];
    if (r.state != R_DONE && r.state != R_REPORTED) return set_error(J3D_ESTATE, "slot %d has no result", slot);
    if (host_dst) {
        // the finished iterate was gathered (dense, x fastest) into the
        // request's other field buffer, which no round touches until release
        const double *src = reinterpret_cast<const double *>(pl->arena) + r.blk.off[r.buf ^ 1];
        const size_t bytes = (size_t)(r.n[0] * r.n[1] * r.n[2]) * sizeof(double);
        j3d_status st = hip_status(hipMemcpyAsync(host_dst, src, bytes, hipMemcpyDeviceToHost, pl->copy_stream),
                                   "fetch copy");
        if (st == J3D_OK) st = hip_status(hipStreamSynchronize(pl->copy_stream), "fetch wait");
        if (st != J3D_OK) return st;
    }
    if (residual) *residual = r.residual;
    if (iters_done) *iters_done = r.iters_done;
    return J3D_OK;
}

j3d_status j3d_pool_set_policy(j3d_pool *pl, int64_t fill_cells, int32_t max_wait_rounds, int32_t backlog_share)
{
    if (!pl) return set_error(J3D_EINVAL, "pool is NULL");
    if (fill_cells < 0 || max_wait_rounds < 1 || backlog_share < 0)
        return set_error(J3D_EINVAL, "fill_cells %lld < 0, max_wait_rounds %d < 1 or backlog_share %d < 0",
                         (long long)fill_cells, max_wait_rounds, backlog_share);
    pl->fill_cells = fill_cells;
    pl->max_wait = max_wait_rounds;
    pl->backlog_share = backlog_share;
    return J3D_OK;
}

j3d_status j3d_pool_set_tune(j3d_pool *pl, const j3d_tune *t)
{
    if (!pl) return set_error(J3D_EINVAL, "pool is NULL");
    for (const Req &r : pl->reqs)
        if (r.state != R_FREE) return set_error(J3D_ESTATE, "pool tile shape can change only while the pool is empty");
    int v = pool_variant(), zc = kPoolZchunk;
    if (t) {
        if (t->variant < -1 || t->variant >= variant_count())
            return set_error(J3D_EINVAL, "tune variant %d out of range [-1, %d)", t->variant, variant_count());
        if (t->zchunk < 1) return set_error(J3D_EINVAL, "pool zchunk %d < 1", t->zchunk);
        if (t->blocks_per_cu != 0)
            return set_error(J3D_EINVAL, "the pool launches one workgroup per tile (blocks_per_cu must be 0)");
        if (t->variant >= 0) v = t->variant;
        zc = t->zchunk;
    }
    pl->variant = v;
    pl->zchunk = zc;
    return J3D_OK;
}

j3d_status j3d_pool_set_two_sweep(j3d_pool *pl, int32_t enable)
{
    if (!pl) return set_error(J3D_EINVAL, "pool is NULL");
    if (enable != 0 && enable != 1) return set_error(J3D_EINVAL, "enable %d is not 0 or 1", enable);
    for (const Req &r : pl->reqs)
        if (r.state != R_FREE)
            return set_error(J3D_ESTATE, "sweeps per launch can change only while the pool is empty");
    if (enable && !pl->host_probs2) {
        j3d_status st = hip_status(hipHostMalloc((void **)&pl->host_probs2, pl->max_slots * sizeof(ProbDesc), 0),
                                   "pinned table");
        if (st != J3D_OK) return st;
        st = hip_status(hipHostMalloc((void **)&pl->host_tiles2,
                                      (size_t)pl->max_slots * kPoolTilesPerReq * sizeof(Tile), 0),
                        "pinned table");
        if (st != J3D_OK) {
            (void)hipHostFree(pl->host_probs2);
            pl->host_probs2 = nullptr;
            return st;
        }
    }
    pl->two_sweep = enable != 0;
    return J3D_OK;
}

j3d_status j3d_pool_release(j3d_pool *pl, int32_t slot)
{
    if (!pl) return set_error(J3D_EINVAL, "pool is NULL");
    if (slot < 0 || slot >= pl->max_slots) return set_error(J3D_EINVAL, "slot %d out of range", slot);
    Req &r = pl->reqs[slot];
    if (r.state == R_FREE) return set_error(J3D_ESTATE, "slot %d is not in use", slot);
    if (r.state == R_COPYING) {
        j3d_status st = hip_status(hipEventSynchronize(r.copy_ev), "release wait");
        if (st != J3D_OK) return st;
    }
    free_range(pl, r.region, r.bytes);
    pl->used -= r.bytes;
    r.state = R_FREE;
    return J3D_OK;
}

j3d_status j3d_pool_usage(const j3d_pool *pl, int32_t *slots_used, uint64_t *bytes_used)
{
    if (!pl) return set_error(J3D_EINVAL, "pool is NULL");
    int32_t n = 0;
    for (const Req &r : pl->reqs) n += r.state != R_FREE;
    if (slots_used) *slots_used = n;
    if (bytes_used) *bytes_used = pl->used;
    return J3D_OK;
}

j3d_status j3d_pool_destroy(j3d_pool *pl)
{
    if (!pl) return set_error(J3D_EINVAL, "pool is NULL");
    j3d_status st = J3D_OK;
    if (pl->stream || pl->copy_stream) {
        st = hip_status(hipStreamSynchronize(pl->stream), "pool destroy");
        if (pl->copy_stream) (void)hipStreamSynchronize(pl->copy_stream);
    }
    for (Req &r : pl->reqs) {
        if (r.gather_ev) (void)hipEventDestroy(r.gather_ev);
        if (r.copy_ev) (void)hipEventDestroy(r.copy_ev);
    }
    if (pl->round_ev) (void)hipEventDestroy(pl->round_ev);
    if (pl->copy_stream) (void)hipStreamDestroy(pl->copy_stream);
    if (pl->host_res) (void)hipHostFree(pl->host_res);
    if (pl->host_probs) (void)hipHostFree(pl->host_probs);
    if (pl->host_blocks) (void)hipHostFree(pl->host_blocks);
    if (pl->host_tiles) (void)hipHostFree(pl->host_tiles);
    if (pl->host_probs2) (void)hipHostFree(pl->host_probs2);
    if (pl->host_tiles2) (void)hipHostFree(pl->host_tiles2);
    delete pl;
    return st;
}

}  // extern "C"
