// j3d_solver.cpp -- the plain solver and the batched form behind the C ABI.
//
// Iteration order (Fig. 1, Fig. 3): pack the six halo faces, exchange them,
// unpack, update the whole block.  The modes differ in how these steps become
// GPU work: per block and face (no fusion, strategies A and B of
// Sec. III-D-1), per phase for all blocks, through host memory (with or
// without the update overlapping the transfers), or as one fused kernel per
// block or for all blocks, which reads y and z halos across the block
// boundary and hands its x faces over at the end of the previous sweep (so the
// first fused sweep is preceded by one pack / exchange / unpack).  Any mode can
// be captured into HIP graphs.  Host and device never synchronise inside the
// iteration loop (Sec. III-C removes such synchronisations); only a requested
// residual or a host copy waits.
#include <algorithm>
#include <climits>
#include <cstdint>
#include <cstring>
#include <new>

#include "j3d_device.hpp"

namespace j3d {

j3d_status hip_status(hipError_t e, const char *what)
{
    if (e == hipSuccess) return J3D_OK;
    return set_error(J3D_EDEVICE, "%s: %s", what, hipGetErrorString(e));
}

j3d_status require_device(int *device, int *cus)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_status(e, "hipGetDevice");
    hipDeviceProp_t prop;
    e = hipGetDeviceProperties(&prop, dev);
    if (e != hipSuccess) return hip_status(e, "hipGetDeviceProperties");
    if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0)
        return set_error(J3D_EDEVICE, "device %d is %s, not gfx950", dev, prop.gcnArchName);
    if (device) *device = dev;
    if (cus) *cus = prop.multiProcessorCount;
    return J3D_OK;
}

namespace {

double *dbase(char *arena) { return reinterpret_cast<double *>(arena); }
const BlockDesc *dblocks(const Plan &plan, char *arena)
{
    return reinterpret_cast<const BlockDesc *>(arena + plan.off_blocks);
}

}  // namespace

j3d_status upload_tables(const Plan &plan, char *arena, hipStream_t stream)
{
    hipError_t e = hipMemcpyAsync(arena + plan.off_blocks, plan.blocks.data(),
                                  plan.blocks.size() * sizeof(BlockDesc), hipMemcpyHostToDevice, stream);
    if (e != hipSuccess) return hip_status(e, "upload blocks");
    std::vector<ProbDesc> probs(plan.probs.size());
    for (size_t i = 0; i < probs.size(); ++i) {
        std::memset(&probs[i], 0, sizeof(ProbDesc));
        probs[i].res_slot = (int32_t)i;
        probs[i].limit = plan.probs[i].iters;
        probs[i].flags = PF_RES_LAST;
    }
    e = hipMemcpyAsync(arena + plan.off_probs, probs.data(), probs.size() * sizeof(ProbDesc),
                       hipMemcpyHostToDevice, stream);
    if (e != hipSuccess) return hip_status(e, "upload problems");
    std::vector<int32_t> maps;
    for (const ProbPlan &pp : plan.probs) {
        maps.clear();
        for (int a = 0; a < 3; ++a)
            for (int32_t b = 0; b < pp.d.nb[a]; ++b)
                for (int64_t l = 0; l < pp.d.ext[a][b]; ++l) {
                    maps.push_back(b);
                    maps.push_back((int32_t)l);
                }
        e = hipMemcpyAsync(arena + pp.maps_off, maps.data(), maps.size() * sizeof(int32_t),
                           hipMemcpyHostToDevice, stream);
        if (e != hipSuccess) return hip_status(e, "upload maps");
        e = hipStreamSynchronize(stream);  // `maps` is reused
        if (e != hipSuccess) return hip_status(e, "upload maps");
    }
    return hip_status(hipStreamSynchronize(stream), "upload tables");
}

j3d_status upload_tiles(const Plan &plan, const std::vector<Tile> &tiles, char *arena,
                        hipStream_t stream)
{
    if (tiles.size() > plan.tiles_cap) return set_error(J3D_EINVAL, "tile table overflow");
    hipError_t e = hipMemcpyAsync(arena + plan.off_tiles, tiles.data(), tiles.size() * sizeof(Tile),
                                  hipMemcpyHostToDevice, stream);
    if (e != hipSuccess) return hip_status(e, "upload tiles");
    return hip_status(hipStreamSynchronize(stream), "upload tiles");
}

j3d_status init_fields(const Plan &plan, char *arena, hipStream_t stream)
{
    for (const ProbPlan &pp : plan.probs) {
        int64_t maxc = 0, maxx = 0;
        for (int32_t b = pp.block_begin; b < pp.block_begin + pp.nblocks; ++b) {
            const BlockDesc &B = plan.blocks[b];
            maxc = std::max<int64_t>(maxc, block_field_cells(B.ext[0], B.ext[1], B.ext[2]));
            maxx = std::max<int64_t>(maxx, (int64_t)B.ext[1] * B.ext[2]);
        }
        j3d_status st = hip_status(
            launch_init(dbase(arena), dblocks(plan, arena), pp.block_begin, pp.nblocks, (int32_t)maxc,
                        (int32_t)maxx, 0, pp.d.n, pp.s0, pp.bc, 1, stream),
            "init launch");
        if (st != J3D_OK) return st;
    }
    return J3D_OK;
}

j3d_status refresh_halos(const Plan &plan, char *arena, int32_t b0, int32_t b1, int parity,
                         hipStream_t stream)
{
    bool any = false;
    for (int32_t b = b0; b < b1 && !any; ++b)
        for (int f = 0; f < 6; ++f) any = any || plan.blocks[b].nbr[f] >= 0;
    if (!any) return J3D_OK;
    if (!plan.with_sr) return set_error(J3D_ESTATE, "halo refresh needs send/receive buffers");
    j3d_status st = hip_status(launch_pack(dbase(arena), dblocks(plan, arena), b0, b1 - b0,
                                           plan.max_face, parity, 63, stream),
                               "pack launch");
    if (st != J3D_OK) return st;
    st = hip_status(launch_exchange(dbase(arena), dblocks(plan, arena), b0, b1 - b0, plan.max_face, stream),
                    "exchange launch");
    if (st != J3D_OK) return st;
    return hip_status(launch_unpack(dbase(arena), dblocks(plan, arena), b0, b1 - b0, plan.max_face,
                                    parity, 63, stream),
                      "unpack launch");
}

j3d_status copy_dense(const Plan &plan, char *arena, int32_t i, int parity, double *dense,
                      int dense_on_device, bool to_dense, hipStream_t stream)
{
    const ProbPlan &pp = plan.probs[i];
    const int32_t *maps = reinterpret_cast<const int32_t *>(arena + pp.maps_off);
    const int64_t *n = pp.d.n;
    const int64_t plane = n[0] * n[1];
    if (dense_on_device) {
        const int e = to_dense ? launch_gather(dbase(arena), dblocks(plan, arena), pp.block_begin, pp.d.nb,
                                               maps, n, 0, n[2], dense, parity, stream)
                               : launch_scatter(dbase(arena), dblocks(plan, arena), pp.block_begin,
                                                pp.d.nb, maps, n, 0, n[2], dense, parity, stream);
        return hip_status(e, to_dense ? "gather launch" : "scatter launch");
    }
    double *bounce = reinterpret_cast<double *>(arena + plan.off_bounce);
    const int64_t per = std::max<int64_t>(1, (int64_t)plan.bounce_doubles / plane);
    for (int64_t z0 = 0; z0 < n[2]; z0 += per) {
        const int64_t z1 = std::min(n[2], z0 + per);
        const size_t bytes = (size_t)((z1 - z0) * plane) * sizeof(double);
        hipError_t e;
        if (to_dense) {
            j3d_status st = hip_status(launch_gather(dbase(arena), dblocks(plan, arena), pp.block_begin,
                                                     pp.d.nb, maps, n, z0, z1, bounce, parity, stream),
                                       "gather launch");
            if (st != J3D_OK) return st;
            e = hipMemcpyAsync(dense + z0 * plane, bounce, bytes, hipMemcpyDeviceToHost, stream);
        } else {
            e = hipMemcpyAsync(bounce, dense + z0 * plane, bytes, hipMemcpyHostToDevice, stream);
            if (e == hipSuccess)
                e = (hipError_t)launch_scatter(dbase(arena), dblocks(plan, arena), pp.block_begin, pp.d.nb,
                                               maps, n, z0, z1, bounce, parity, stream);
        }
        if (e != hipSuccess) return hip_status(e, "dense copy");
    }
    return hip_status(hipStreamSynchronize(stream), "dense copy");
}

}  // namespace j3d

using namespace j3d;

// ---- plain solver ---------------------------------------------------------------

struct j3d_solver {
    Plan plan;
    char *arena = nullptr;
    hipStream_t stream = nullptr;
    int device = 0, cus = 256;
    int parity = 0;
    bool ghosts_fresh = false;
    int64_t iters_done = 0;
    j3d_tune tune{0, 0, 0};
    int zchunk = 1;
    int32_t ntiles = 0;
    std::vector<Tile> tiles;
    std::vector<uint64_t> work;  // prefix sums of the tiles' estimated work
    std::vector<int32_t> block_first;
    uint32_t persist_launches = 0;
    hipStream_t cap_stream = nullptr;
    // Per-block modes: blocks' operations go round-robin to these streams, as
    // each chare had its own stream, so independent blocks overlap on the GPU;
    // phases are joined by events (fork/join on the caller's stream).
    static constexpr int kSideStreams = 4;
    hipStream_t side[kSideStreams] = {};
    hipEvent_t fork_ev = nullptr, join_ev[kSideStreams] = {};
    // Host-staged modes: page-locked mirror of the send/receive region.
    double *host_sr = nullptr;
    int64_t sr_lo = 0, sr_hi = 0;  // doubles from the arena base
    int64_t max_shell = 0;
    struct GraphEntry {
        int mode, parity, slot;
        hipGraph_t graph;
        hipGraphExec_t exec;
    };
    std::vector<GraphEntry> graphs;
};

namespace {

void drop_graphs(j3d_solver *s)
{
    for (auto &g : s->graphs) {
        (void)hipGraphExecDestroy(g.exec);
        (void)hipGraphDestroy(g.graph);
    }
    s->graphs.clear();
}

j3d_status apply_tune(j3d_solver *s, const j3d_tune &t)
{
    int zc = 0;
    j3d_status st = check_tune(s->plan, &t, &zc);
    if (st != J3D_OK) return st;
    std::vector<Tile> tiles;
    std::vector<int32_t> first;
    make_tiles(s->plan, 0, (int32_t)s->plan.blocks.size(), t.variant, t.zchunk, &tiles, &first);
    st = upload_tiles(s->plan, tiles, s->arena, s->stream);
    if (st != J3D_OK) return st;
    s->tune = t;
    s->zchunk = zc;
    tile_work(tiles, &s->work);
    s->tiles.swap(tiles);
    s->block_first.swap(first);
    s->ntiles = (int32_t)s->tiles.size();
    drop_graphs(s);
    return J3D_OK;
}

SweepArgs base_args(j3d_solver *s)
{
    SweepArgs a;
    std::memset(&a, 0, sizeof a);
    a.base = reinterpret_cast<double *>(s->arena);
    a.blocks = reinterpret_cast<const BlockDesc *>(s->arena + s->plan.off_blocks);
    a.probs = reinterpret_cast<const ProbDesc *>(s->arena + s->plan.off_probs);
    a.tiles = reinterpret_cast<const Tile *>(s->arena + s->plan.off_tiles);
    a.res = reinterpret_cast<unsigned long long *>(s->arena + s->plan.off_res);
    a.queue = reinterpret_cast<unsigned int *>(s->arena + s->plan.off_queue);
    a.zchunk = s->zchunk;
    return a;
}

// One sweep over tiles [t0, t0+cnt) reading parity `parity`.  `slot` is the
// persistent-queue half (ignored for one-workgroup-per-tile launches).
j3d_status sweep(j3d_solver *s, int parity, bool fused, bool res, int32_t t0, int32_t cnt, int slot,
                 hipStream_t st)
{
    SweepArgs a = base_args(s);
    a.tile_begin = t0;
    a.tile_count = cnt;
    a.parity = parity;
    a.flags = (fused ? SW_FUSED : 0) | (res ? SW_RES : 0);
    int grid;
    if (s->tune.blocks_per_cu > 0) {
        a.flags |= SW_PERSIST;
        a.queue_slot = slot;
        grid = std::min(cnt, s->cus * s->tune.blocks_per_cu);
    } else {
        grid = xcd_split(s->work, t0, cnt, a.xcut);
    }
    return hip_status(launch_sweep(s->tune.variant, a, grid, st), "sweep launch");
}

// One workgroup per tile, whatever the tune's schedule (per-block launches).
// extra_flags: SW_INNER restricts the sweep to the cells that read no halo.
j3d_status sweep_tiles(j3d_solver *s, int parity, bool fused, bool res, int32_t t0, int32_t cnt, hipStream_t st,
                       int32_t extra_flags = 0)
{
    SweepArgs a = base_args(s);
    a.tile_begin = t0;
    a.tile_count = cnt;
    a.parity = parity;
    a.flags = (fused ? SW_FUSED : 0) | (res ? SW_RES : 0) | extra_flags;
    return hip_status(launch_sweep(s->tune.variant, a, cnt, st), "sweep launch");
}

// Launches per HIP graph (one_sweep calls; a TWO_SWEEP launch performs two
// sweeps): an even number, so a replay returns to the same buffer parity.  A
// fused sweep is one node; the per-block modes put thousands of nodes into
// one sweep, so their graphs hold two.
int graph_sweeps(int mode) { return mode == J3D_FUSED ? 50 : mode == J3D_TWO_SWEEP ? 24 : 2; }

// Modes whose sweep is one launch that may use the persistent schedule.
bool persistent_mode(const j3d_solver *s, int mode)
{
    return s->tune.blocks_per_cu > 0 && (mode == J3D_FUSED || mode == J3D_UNFUSED_PHASE);
}

j3d_status one_sweep(j3d_solver *s, int mode, int p, bool res, int slot, hipStream_t st);

j3d_status get_graph(j3d_solver *s, int mode, int parity, int slot, hipGraphExec_t *out)
{
    for (auto &g : s->graphs)
        if (g.mode == mode && g.parity == parity && g.slot == slot) {
            *out = g.exec;
            return J3D_OK;
        }
    if (!s->cap_stream) {
        j3d_status st = hip_status(hipStreamCreateWithFlags(&s->cap_stream, hipStreamNonBlocking),
                                   "capture stream");
        if (st != J3D_OK) return st;
    }
    j3d_status st = hip_status(hipStreamBeginCapture(s->cap_stream, hipStreamCaptureModeThreadLocal),
                               "begin capture");
    if (st != J3D_OK) return st;
    j3d_status launch_st = J3D_OK;
    for (int i = 0; i < graph_sweeps(mode) && launch_st == J3D_OK; ++i) {
        const int sl = persistent_mode(s, mode) ? ((slot + i) & 1) : 0;
        launch_st = one_sweep(s, mode, parity ^ (i & 1), false, sl, s->cap_stream);
    }
    hipGraph_t graph = nullptr;
    st = hip_status(hipStreamEndCapture(s->cap_stream, &graph), "end capture");
    if (launch_st != J3D_OK) {
        if (graph) (void)hipGraphDestroy(graph);
        return launch_st;
    }
    if (st != J3D_OK) return st;
    hipGraphExec_t exec = nullptr;
    st = hip_status(hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0), "graph instantiate");
    if (st != J3D_OK) {
        (void)hipGraphDestroy(graph);
        return st;
    }
    s->graphs.push_back({mode, parity, slot, graph, exec});
    *out = exec;
    return J3D_OK;
}

j3d_status ensure_side_streams(j3d_solver *s)
{
    if (s->fork_ev) return J3D_OK;
    for (int k = 0; k < j3d_solver::kSideStreams; ++k) {
        j3d_status st = hip_status(hipStreamCreateWithFlags(&s->side[k], hipStreamNonBlocking), "side stream");
        if (st == J3D_OK)
            st = hip_status(hipEventCreateWithFlags(&s->join_ev[k], hipEventDisableTiming), "join event");
        if (st != J3D_OK) return st;
    }
    return hip_status(hipEventCreateWithFlags(&s->fork_ev, hipEventDisableTiming), "fork event");
}

// The side streams start after everything enqueued on `main` so far.
j3d_status fork_side(j3d_solver *s, hipStream_t main)
{
    j3d_status st = hip_status(hipEventRecord(s->fork_ev, main), "fork");
    for (int k = 0; k < j3d_solver::kSideStreams && st == J3D_OK; ++k)
        st = hip_status(hipStreamWaitEvent(s->side[k], s->fork_ev, 0), "fork");
    return st;
}

// `main` continues after everything enqueued on the side streams so far.
j3d_status join_side(j3d_solver *s, hipStream_t main)
{
    j3d_status st = J3D_OK;
    for (int k = 0; k < j3d_solver::kSideStreams && st == J3D_OK; ++k) {
        st = hip_status(hipEventRecord(s->join_ev[k], s->side[k]), "join");
        if (st == J3D_OK) st = hip_status(hipStreamWaitEvent(main, s->join_ev[k], 0), "join");
    }
    return st;
}

// Per-block launch streams (the paper's per-chare GPU operations) under
// fusion strategy `strat`: 0 none (six pack kernels, six copies, six unpack
// kernels, one update per block), 1 = A (one pack kernel for the six faces),
// 2 = B (A, and one unpack kernel), 3 = C (one kernel per block: halo reads,
// update and x-face hand-off, no copies).
j3d_status run_per_block(j3d_solver *s, int p, bool res_last, int strat, hipStream_t main)
{
    const Plan &plan = s->plan;
    const int32_t nb = (int32_t)plan.blocks.size();
    j3d_status fst = ensure_side_streams(s);
    if (fst == J3D_OK) fst = fork_side(s, main);
    if (fst != J3D_OK) return fst;
    auto lane = [&](int32_t b) { return s->side[b % j3d_solver::kSideStreams]; };
    if (strat == 3) {
        for (int32_t b = 0; b < nb; ++b) {
            j3d_status st = sweep_tiles(s, p, true, res_last, s->block_first[b],
                                        s->block_first[b + 1] - s->block_first[b], lane(b));
            if (st != J3D_OK) return st;
        }
        return join_side(s, main);
    }
    double *base = reinterpret_cast<double *>(s->arena);
    const BlockDesc *blocks = reinterpret_cast<const BlockDesc *>(s->arena + plan.off_blocks);
    auto faces = [](const BlockDesc &B, int64_t fsz[6]) {
        const int64_t ex = B.ext[0], ey = B.ext[1], ez = B.ext[2];
        fsz[0] = fsz[1] = ey * ez;
        fsz[2] = fsz[3] = ex * ez;
        fsz[4] = fsz[5] = ex * ey;
    };
    // every block packs and sends its faces ...
    for (int32_t b = 0; b < nb; ++b) {
        const BlockDesc &B = plan.blocks[b];
        hipStream_t stream = lane(b);
        int64_t fsz[6], fo[6];
        faces(B, fsz);
        fo[0] = 0;
        for (int f = 1; f < 6; ++f) fo[f] = fo[f - 1] + fsz[f - 1];
        int mask = 0;
        int64_t maxf = 0;
        for (int f = 0; f < 6; ++f)
            if (B.nbr[f] >= 0) {
                mask |= 1 << f;
                maxf = std::max(maxf, fsz[f]);
            }
        if (strat == 0) {
            for (int f = 0; f < 6; ++f) {
                if (B.nbr[f] < 0) continue;
                j3d_status st = hip_status(launch_pack(base, blocks, b, 1, (int32_t)fsz[f], p, 1 << f, stream),
                                           "pack launch");
                if (st != J3D_OK) return st;
            }
        } else if (mask) {
            j3d_status st = hip_status(launch_pack(base, blocks, b, 1, (int32_t)maxf, p, mask, stream),
                                       "pack launch");
            if (st != J3D_OK) return st;
        }
        for (int f = 0; f < 6; ++f) {
            if (B.nbr[f] < 0) continue;
            const BlockDesc &N = plan.blocks[B.nbr[f]];
            int64_t nsz[6];
            faces(N, nsz);
            int64_t no = 0;
            for (int g = 0; g < (f ^ 1); ++g) no += nsz[g];
            double *dst = base + N.sr_off + N.face_total + no;
            const double *src = base + B.sr_off + fo[f];
            j3d_status st = hip_status(hipMemcpyAsync(dst, src, (size_t)fsz[f] * sizeof(double),
                                                      hipMemcpyDeviceToDevice, stream),
                                       "halo copy");
            if (st != J3D_OK) return st;
        }
    }
    // ... then, once every face has arrived, every block unpacks what it
    // received and updates.
    j3d_status jst = join_side(s, main);
    if (jst == J3D_OK) jst = fork_side(s, main);
    if (jst != J3D_OK) return jst;
    for (int32_t b = 0; b < nb; ++b) {
        const BlockDesc &B = plan.blocks[b];
        hipStream_t stream = lane(b);
        int64_t fsz[6];
        faces(B, fsz);
        int mask = 0;
        int64_t maxf = 0;
        for (int f = 0; f < 6; ++f)
            if (B.nbr[f] >= 0) {
                mask |= 1 << f;
                maxf = std::max(maxf, fsz[f]);
            }
        if (strat == 2) {
            if (mask) {
                j3d_status st = hip_status(launch_unpack(base, blocks, b, 1, (int32_t)maxf, p, mask, stream),
                                           "unpack launch");
                if (st != J3D_OK) return st;
            }
        } else {
            for (int f = 0; f < 6; ++f) {
                if (B.nbr[f] < 0) continue;
                j3d_status st = hip_status(launch_unpack(base, blocks, b, 1, (int32_t)fsz[f], p, 1 << f, stream),
                                           "unpack launch");
                if (st != J3D_OK) return st;
            }
        }
        j3d_status st = sweep_tiles(s, p, false, res_last, s->block_first[b],
                                    s->block_first[b + 1] - s->block_first[b], stream);
        if (st != J3D_OK) return st;
    }
    return join_side(s, main);
}

j3d_status ensure_host_mirror(j3d_solver *s)
{
    if (s->host_sr) return J3D_OK;
    int64_t lo = INT64_MAX, hi = 0, shell = 0;
    for (const BlockDesc &B : s->plan.blocks) {
        lo = std::min<int64_t>(lo, B.sr_off);
        hi = std::max<int64_t>(hi, B.sr_off + 2 * B.face_total);
        const int64_t ex = B.ext[0], ey = B.ext[1], ez = B.ext[2];
        const int64_t plane = ex * ey, ring = (ex <= 2 || ey <= 2) ? plane : 2 * ex + 2 * (ey - 2);
        shell = std::max(shell, (ez >= 2 ? 2 : 1) * plane + std::max<int64_t>(ez - 2, 0) * ring);
    }
    j3d_status st = hip_status(hipHostMalloc((void **)&s->host_sr, (size_t)(hi - lo) * sizeof(double), 0),
                               "page-locked staging buffer");
    if (st != J3D_OK) {
        s->host_sr = nullptr;
        return st;
    }
    s->sr_lo = lo;
    s->sr_hi = hi;
    s->max_shell = shell;
    return J3D_OK;
}

// One iteration with the exchange staged through host memory.  overlap
// (Fig. 1): the interior update (the cells that read no halo) runs on a side
// stream while the faces travel, and the exterior update (the one-cell shell
// of each block) runs once the halos are unpacked; every cell is written once.
j3d_status run_host_staged(j3d_solver *s, int p, bool res, bool overlap, hipStream_t main)
{
    const Plan &plan = s->plan;
    const int32_t nb = (int32_t)plan.blocks.size();
    double *base = reinterpret_cast<double *>(s->arena);
    const BlockDesc *blocks = reinterpret_cast<const BlockDesc *>(s->arena + plan.off_blocks);
    double *H = s->host_sr - s->sr_lo;  // indexed like the arena, over the send/receive region only
    j3d_status st = J3D_OK;
    if (overlap) {
        st = ensure_side_streams(s);
        if (st == J3D_OK) st = fork_side(s, main);
        // the interior update (cells that read no halo) while the faces travel
        if (st == J3D_OK) st = sweep_tiles(s, p, false, false, 0, s->ntiles, s->side[0], SW_INNER);
        if (st != J3D_OK) return st;
    }
    st = hip_status(launch_pack(base, blocks, 0, nb, plan.max_face, p, 0x3f, main), "pack launch");
    if (st != J3D_OK) return st;
    // every face to host memory, into the receiver's slot ...
    for (int32_t b = 0; b < nb; ++b) {
        const BlockDesc &B = plan.blocks[b];
        const int64_t fsz[6] = {(int64_t)B.ext[1] * B.ext[2], (int64_t)B.ext[1] * B.ext[2],
                                (int64_t)B.ext[0] * B.ext[2], (int64_t)B.ext[0] * B.ext[2],
                                (int64_t)B.ext[0] * B.ext[1], (int64_t)B.ext[0] * B.ext[1]};
        int64_t fo = 0;
        for (int f = 0; f < 6; fo += fsz[f], ++f) {
            if (B.nbr[f] < 0) continue;
            const BlockDesc &N = plan.blocks[B.nbr[f]];
            const int64_t nsz[6] = {(int64_t)N.ext[1] * N.ext[2], (int64_t)N.ext[1] * N.ext[2],
                                    (int64_t)N.ext[0] * N.ext[2], (int64_t)N.ext[0] * N.ext[2],
                                    (int64_t)N.ext[0] * N.ext[1], (int64_t)N.ext[0] * N.ext[1]};
            int64_t no = 0;
            for (int g = 0; g < (f ^ 1); ++g) no += nsz[g];
            st = hip_status(hipMemcpyAsync(H + N.sr_off + N.face_total + no, base + B.sr_off + fo,
                                           (size_t)fsz[f] * sizeof(double), hipMemcpyDeviceToHost, main),
                            "face to host");
            if (st != J3D_OK) return st;
        }
    }
    // ... and each block's received faces back to the device
    for (int32_t b = 0; b < nb; ++b) {
        const BlockDesc &B = plan.blocks[b];
        st = hip_status(hipMemcpyAsync(base + B.sr_off + B.face_total, H + B.sr_off + B.face_total,
                                       (size_t)B.face_total * sizeof(double), hipMemcpyHostToDevice, main),
                        "faces to device");
        if (st != J3D_OK) return st;
    }
    if (overlap) {
        st = join_side(s, main);
        if (st != J3D_OK) return st;
    }
    st = hip_status(launch_unpack(base, blocks, 0, nb, plan.max_face, p, 0x3f, main), "unpack launch");
    if (st != J3D_OK) return st;
    if (overlap) return hip_status(launch_shell(base, blocks, 0, nb, s->max_shell, p, main), "shell launch");
    return sweep_tiles(s, p, false, res, 0, s->ntiles, main);
}

// One launch of the two-sweep kernel: iterate in buffer p -> two sweeps later
// in buffer p^1.  Whole planes when the x-y tiles alone give every compute
// unit two workgroups, else z-chunks (at least 4 planes) for about that many.
j3d_status two_sweep_launch(j3d_solver *s, int p, bool res, hipStream_t st)
{
    const BlockDesc &B = s->plan.blocks[0];
    double *base = reinterpret_cast<double *>(s->arena);
    TwoStepArgs a;
    std::memset(&a, 0, sizeof a);
    a.ex = B.ext[0];
    a.ey = B.ext[1];
    a.ez = B.ext[2];
    a.pitch = B.pitch;
    a.res = reinterpret_cast<unsigned long long *>(s->arena + s->plan.off_res);
    int ntx = 0, nty = 0, ntz = 0;
    twostep_tiles(a.ex, a.ey, a.ez, 0, &ntx, &nty, &ntz);
    int zc = 0;
    if (ntx * nty < 2 * s->cus) {
        const int want = (2 * s->cus + ntx * nty - 1) / (ntx * nty);
        zc = std::max(4, (a.ez + want - 1) / want);
    }
    twostep_tiles(a.ex, a.ey, a.ez, zc, &a.ntx, &a.nty, &a.ntz);
    a.cur = base + B.off[p];
    a.nxt = base + B.off[p ^ 1];
    a.xh = base + B.xoff[p];
    a.want_res = res ? 1 : 0;
    return hip_status(launch_twostep(a, st), "two-sweep launch");
}

// One sweep of `mode` reading parity p, enqueued on st.
j3d_status one_sweep(j3d_solver *s, int mode, int p, bool res, int slot, hipStream_t st)
{
    switch (mode) {
    case J3D_FUSED:
        return sweep(s, p, true, res, 0, s->ntiles, slot, st);
    case J3D_UNFUSED_PHASE: {
        j3d_status r = refresh_halos(s->plan, s->arena, 0, (int32_t)s->plan.blocks.size(), p, st);
        return r != J3D_OK ? r : sweep(s, p, false, res, 0, s->ntiles, slot, st);
    }
    case J3D_UNFUSED_BLOCK:
        return run_per_block(s, p, res, 0, st);
    case J3D_BLOCK_A:
        return run_per_block(s, p, res, 1, st);
    case J3D_BLOCK_B:
        return run_per_block(s, p, res, 2, st);
    case J3D_BLOCK_C:
        return run_per_block(s, p, res, 3, st);
    case J3D_HOST_STAGED:
        return run_host_staged(s, p, res, false, st);
    case J3D_HOST_OVERLAP:
        // the overlapped update's shell pass carries no residual
        return run_host_staged(s, p, res, !res, st);
    case J3D_TWO_SWEEP:  // one launch, two sweeps
        return two_sweep_launch(s, p, res, st);
    }
    return set_error(J3D_EINVAL, "unknown mode %d", mode);
}

// Read back a requested residual (synchronises) after a run.
j3d_status finish_run(j3d_solver *s, double *residual_out, const unsigned long long *res)
{
    if (!residual_out) return J3D_OK;
    unsigned long long bits = 0;
    j3d_status st = hip_status(hipMemcpyAsync(&bits, res, sizeof bits, hipMemcpyDeviceToHost, s->stream),
                               "residual readback");
    if (st == J3D_OK) st = hip_status(hipStreamSynchronize(s->stream), "residual readback");
    if (st != J3D_OK) return st;
    double r;
    std::memcpy(&r, &bits, sizeof r);
    *residual_out = r;
    return J3D_OK;
}

// TWO_SWEEP: iters / 2 two-sweep launches (each reads the current buffer and
// writes the other), replayed from HIP graphs of 24 launches when captured,
// then one fused sweep if iters is odd.  The residual comes from the launch
// that performs the last sweep, which is never inside a graph.
j3d_status run_two_sweep(j3d_solver *s, int64_t iters, bool want_res, bool captured)
{
    int p = s->parity;
    const int64_t pairs = iters / 2;
    const bool res_in_pair = want_res && (iters & 1) == 0;
    int64_t k = 0;
    if (captured) {
        const int g = graph_sweeps(J3D_TWO_SWEEP);
        const int64_t plain = pairs - (res_in_pair ? 1 : 0);
        for (; k + g <= plain; k += g) {
            hipGraphExec_t exec = nullptr;
            j3d_status st = get_graph(s, J3D_TWO_SWEEP, p, 0, &exec);
            if (st != J3D_OK) return st;
            st = hip_status(hipGraphLaunch(exec, s->stream), "graph launch");
            if (st != J3D_OK) return st;
        }
    }
    for (; k < pairs; ++k) {
        j3d_status st = two_sweep_launch(s, p, res_in_pair && k + 1 == pairs, s->stream);
        if (st != J3D_OK) return st;
        p ^= 1;
    }
    if (iters & 1) {
        const int slot = persistent_mode(s, J3D_FUSED) ? (int)(s->persist_launches++ & 1) : 0;
        j3d_status st = one_sweep(s, J3D_FUSED, p, want_res, slot, s->stream);
        if (st != J3D_OK) return st;
        p ^= 1;
    }
    s->parity = p;
    s->iters_done += iters;
    return J3D_OK;
}

}  // namespace

extern "C" {

j3d_status j3d_create(const j3d_problem *p, void *dev_arena, uint64_t arena_bytes, void *hip_stream,
                      j3d_solver **out)
{
    if (!out) return set_error(J3D_EINVAL, "out is NULL");
    if (!dev_arena) return set_error(J3D_EINVAL, "arena is NULL");
    if (reinterpret_cast<uintptr_t>(dev_arena) % 256) return set_error(J3D_EINVAL, "arena not 256-byte aligned");
    Plan plan;
    j3d_status st = make_plan(1, p, true, &plan);
    if (st != J3D_OK) return st;
    if (arena_bytes < plan.total)
        return set_error(J3D_ENOMEM, "arena holds %llu bytes, %llu needed", (unsigned long long)arena_bytes,
                         (unsigned long long)plan.total);
    int dev = 0, cus = 0;
    st = require_device(&dev, &cus);
    if (st != J3D_OK) return st;
    j3d_solver *s = new (std::nothrow) j3d_solver();
    if (!s) return set_error(J3D_EINVAL, "out of host memory");
    s->plan = std::move(plan);
    s->arena = static_cast<char *>(dev_arena);
    s->stream = static_cast<hipStream_t>(hip_stream);
    s->device = dev;
    s->cus = cus;
    st = upload_tables(s->plan, s->arena, s->stream);
    if (st == J3D_OK) {
        j3d_tune t;
        default_tune(s->plan, s->cus, &t);
        st = apply_tune(s, t);
    }
    if (st == J3D_OK)
        st = hip_status(launch_fill_u32(reinterpret_cast<unsigned int *>(s->arena + s->plan.off_queue), 16, 0,
                                        s->stream),
                        "queue init");
    if (st == J3D_OK) st = init_fields(s->plan, s->arena, s->stream);
    if (st != J3D_OK) {
        delete s;
        return st;
    }
    *out = s;
    return J3D_OK;
}

j3d_status j3d_set_interior(j3d_solver *s, const double *src, int src_on_device)
{
    if (!s || !src) return set_error(J3D_EINVAL, "NULL argument");
    j3d_status st = copy_dense(s->plan, s->arena, 0, s->parity, const_cast<double *>(src), src_on_device,
                               false, s->stream);
    if (st != J3D_OK) return st;
    s->ghosts_fresh = false;
    s->iters_done = 0;
    return J3D_OK;
}

j3d_status j3d_set_face(j3d_solver *s, int32_t face, const double *src, int src_on_device)
{
    if (!s || !src) return set_error(J3D_EINVAL, "NULL argument");
    if (face < 0 || face > 5) return set_error(J3D_EINVAL, "face %d out of range [0, 5]", face);
    const ProbPlan &pp = s->plan.probs[0];
    const int64_t *n = pp.d.n;
    const int axis = face / 2;
    const int64_t count = axis == 0 ? n[1] * n[2] : (axis == 1 ? n[0] * n[2] : n[0] * n[1]);
    const double *dsrc = src;
    if (!src_on_device) {
        double *bounce = reinterpret_cast<double *>(s->arena + s->plan.off_bounce);
        j3d_status st = hip_status(hipMemcpyAsync(bounce, src, (size_t)count * sizeof(double),
                                                  hipMemcpyHostToDevice, s->stream),
                                   "face upload");
        if (st != J3D_OK) return st;
        dsrc = bounce;
    }
    j3d_status st = hip_status(
        launch_set_face(reinterpret_cast<double *>(s->arena),
                        reinterpret_cast<const BlockDesc *>(s->arena + s->plan.off_blocks), pp.block_begin,
                        pp.d.nb, reinterpret_cast<const int32_t *>(s->arena + pp.maps_off), n, face, dsrc,
                        s->stream),
        "set_face launch");
    if (st != J3D_OK) return st;
    if (!src_on_device) return hip_status(hipStreamSynchronize(s->stream), "set_face");
    return J3D_OK;
}

j3d_status j3d_set_tune(j3d_solver *s, const j3d_tune *t)
{
    if (!s) return set_error(J3D_EINVAL, "solver is NULL");
    j3d_tune d;
    if (t) {
        d = *t;
        if (d.variant == -1) {
            j3d_tune def;
            default_tune(s->plan, s->cus, &def);
            d.variant = def.variant;
        }
    } else {
        default_tune(s->plan, s->cus, &d);
    }
    return apply_tune(s, d);
}

j3d_status j3d_get_tune(const j3d_solver *s, j3d_tune *out)
{
    if (!s || !out) return set_error(J3D_EINVAL, "NULL argument");
    *out = s->tune;
    return J3D_OK;
}

j3d_status j3d_run(j3d_solver *s, int64_t iters, j3d_mode mode_in, double *residual_out)
{
    if (!s) return set_error(J3D_EINVAL, "solver is NULL");
    if (iters < 0) return set_error(J3D_EINVAL, "iters %lld < 0", (long long)iters);
    int mode = (int)mode_in;
    bool captured = (mode & J3D_CAPTURED) != 0;
    mode &= ~(int)J3D_CAPTURED;
    if (mode == J3D_GRAPH) {
        mode = J3D_FUSED;
        captured = true;
    }
    if (mode < J3D_UNFUSED_BLOCK || mode > J3D_TWO_SWEEP)
        return set_error(J3D_EINVAL, "unknown mode %d", (int)mode_in);
    if (mode == J3D_TWO_SWEEP) {
        if (s->plan.blocks.size() != 1)
            return set_error(J3D_EINVAL, "the two-sweep mode needs a grid of one block (%zu blocks)",
                             s->plan.blocks.size());
    }
    if (iters == 0) {
        if (residual_out) *residual_out = 0.0;
        return J3D_OK;
    }
    const bool want_res = residual_out != nullptr;
    unsigned long long *res = reinterpret_cast<unsigned long long *>(s->arena + s->plan.off_res);
    j3d_status st = J3D_OK;
    if (mode == J3D_TWO_SWEEP) {
        if (want_res) {
            st = hip_status(launch_fill_u64(res, 1, 0ull, s->stream), "residual reset");
            if (st != J3D_OK) return st;
        }
        st = run_two_sweep(s, iters, want_res, captured);
        if (st != J3D_OK) return st;
        return finish_run(s, residual_out, res);
    }
    // modes that read x halos where the previous fused sweep handed them over
    const bool fused = mode == J3D_FUSED || mode == J3D_BLOCK_C;
    if (fused && !s->ghosts_fresh) {
        st = refresh_halos(s->plan, s->arena, 0, (int32_t)s->plan.blocks.size(), s->parity, s->stream);
        if (st != J3D_OK) return st;
        s->ghosts_fresh = true;
    }
    if (mode == J3D_HOST_STAGED || mode == J3D_HOST_OVERLAP) {
        st = ensure_host_mirror(s);
        if (st != J3D_OK) return st;
    }
    if (want_res) {
        st = hip_status(launch_fill_u64(res, 1, 0ull, s->stream), "residual reset");
        if (st != J3D_OK) return st;
    }
    const bool persist = persistent_mode(s, mode);
    int p = s->parity;
    int64_t done = 0;
    if (captured) {
        const int gs = graph_sweeps(mode);
        const int64_t plain = iters - (want_res ? 1 : 0);
        for (int64_t r = 0; r < plain / gs; ++r) {
            const int slot = persist ? (int)(s->persist_launches & 1) : 0;
            hipGraphExec_t exec = nullptr;
            st = get_graph(s, mode, p, slot, &exec);
            if (st != J3D_OK) return st;
            st = hip_status(hipGraphLaunch(exec, s->stream), "graph launch");
            if (st != J3D_OK) return st;
            if (persist) s->persist_launches += (uint32_t)gs;
            done += gs;
        }
    }
    for (; done < iters; ++done) {
        const bool res_here = want_res && done + 1 == iters;
        const int slot = persist ? (int)(s->persist_launches++ & 1) : 0;
        st = one_sweep(s, mode, p, res_here, slot, s->stream);
        if (st != J3D_OK) return st;
        p ^= 1;
    }
    p = (int)((s->parity + iters) & 1);
    s->parity = p;
    s->iters_done += iters;
    s->ghosts_fresh = fused;
    return finish_run(s, residual_out, res);
}

j3d_status j3d_iters_done(const j3d_solver *s, int64_t *iters)
{
    if (!s || !iters) return set_error(J3D_EINVAL, "NULL argument");
    *iters = s->iters_done;
    return J3D_OK;
}

j3d_status j3d_get_interior(j3d_solver *s, double *dst, int dst_on_device)
{
    if (!s || !dst) return set_error(J3D_EINVAL, "NULL argument");
    return copy_dense(s->plan, s->arena, 0, s->parity, dst, dst_on_device, true, s->stream);
}

j3d_status j3d_destroy(j3d_solver *s)
{
    if (!s) return set_error(J3D_EINVAL, "solver is NULL");
    j3d_status st = hip_status(hipStreamSynchronize(s->stream), "destroy");
    for (hipStream_t x : s->side)
        if (x) (void)hipStreamSynchronize(x);
    drop_graphs(s);
    if (s->cap_stream) (void)hipStreamDestroy(s->cap_stream);
    for (int k = 0; k < j3d_solver::kSideStreams; ++k) {
        if (s->side[k]) (void)hipStreamDestroy(s->side[k]);
        if (s->join_ev[k]) (void)hipEventDestroy(s->join_ev[k]);
    }
    if (s->fork_ev) (void)hipEventDestroy(s->fork_ev);
    if (s->host_sr) (void)hipHostFree(s->host_sr);
    delete s;
    return st;
}

}  // extern "C"

// ---- batched form -------------------------------------------------------------

struct j3d_batch {
    Plan plan;
    char *arena = nullptr;
    hipStream_t stream = nullptr;
    int device = 0, cus = 256;
    j3d_tune tune{0, 0, 0};
    int zchunk = 1;
    std::vector<int32_t> order;         // problems by iteration count, descending
    std::vector<int32_t> prefix_tiles;  // tiles of the first k problems of `order`
    std::vector<uint64_t> work;         // prefix sums of the tiles' estimated work
    int64_t max_iters = 0;
    bool ran = false;
    uint32_t persist_launches = 0;
    std::vector<int> final_parity;      // buffer holding each problem's result after the run
};

extern "C" {

j3d_status j3d_batch_create(int32_t count, const j3d_problem *probs, const int64_t *iters,
                            void *dev_arena, uint64_t arena_bytes, void *hip_stream,
                            const j3d_tune *tune, j3d_batch **out)
{
    if (!out || !iters || !probs) return set_error(J3D_EINVAL, "NULL argument");
    if (!dev_arena) return set_error(J3D_EINVAL, "arena is NULL");
    if (reinterpret_cast<uintptr_t>(dev_arena) % 256) return set_error(J3D_EINVAL, "arena not 256-byte aligned");
    for (int32_t i = 0; i < count; ++i)
        if (iters[i] < 0) return set_error(J3D_EINVAL, "iters[%d] < 0", i);
    Plan plan;
    j3d_status st = make_plan(count, probs, true, &plan);
    if (st != J3D_OK) return st;
    for (int32_t i = 0; i < count; ++i) plan.probs[i].iters = iters[i];
    if (arena_bytes < plan.total)
        return set_error(J3D_ENOMEM, "arena holds %llu bytes, %llu needed", (unsigned long long)arena_bytes,
                         (unsigned long long)plan.total);
    int dev = 0, cus = 0;
    st = require_device(&dev, &cus);
    if (st != J3D_OK) return st;
    j3d_tune t;
    if (tune) {
        t = *tune;
        if (t.variant == -1) {
            j3d_tune def;
            default_tune(plan, cus, &def);
            t.variant = def.variant;
        }
    } else {
        default_tune(plan, cus, &t);
    }
    int zc = 0;
    st = check_tune(plan, &t, &zc);
    if (st != J3D_OK) return st;

    j3d_batch *b = new (std::nothrow) j3d_batch();
    if (!b) return set_error(J3D_EINVAL, "out of host memory");
    b->plan = std::move(plan);
    b->arena = static_cast<char *>(dev_arena);
    b->stream = static_cast<hipStream_t>(hip_stream);
    b->device = dev;
    b->cus = cus;
    b->tune = t;
    b->zchunk = zc;
    b->order.resize(count);
    for (int32_t i = 0; i < count; ++i) b->order[i] = i;
    std::stable_sort(b->order.begin(), b->order.end(),
                     [&](int32_t x, int32_t y) { return iters[x] > iters[y]; });
    std::vector<Tile> tiles;
    b->prefix_tiles.assign(1, 0);
    for (int32_t k = 0; k < count; ++k) {
        const ProbPlan &pp = b->plan.probs[b->order[k]];
        make_tiles(b->plan, pp.block_begin, pp.block_begin + pp.nblocks, t.variant, t.zchunk, &tiles, nullptr);
        b->prefix_tiles.push_back((int32_t)tiles.size());
    }
    b->max_iters = count > 0 ? iters[b->order[0]] : 0;
    tile_work(tiles, &b->work);
    st = upload_tables(b->plan, b->arena, b->stream);
    if (st == J3D_OK) st = upload_tiles(b->plan, tiles, b->arena, b->stream);
    if (st == J3D_OK)
        st = hip_status(launch_fill_u32(reinterpret_cast<unsigned int *>(b->arena + b->plan.off_queue), 16, 0,
                                        b->stream),
                        "queue init");
    if (st == J3D_OK) st = init_fields(b->plan, b->arena, b->stream);
    if (st != J3D_OK) {
        delete b;
        return st;
    }
    *out = b;
    return J3D_OK;
}

j3d_status j3d_batch_run(j3d_batch *b, double *residuals_out)
{
    if (!b) return set_error(J3D_EINVAL, "batch is NULL");
    if (b->ran) return set_error(J3D_ESTATE, "batch already ran");
    const int32_t count = (int32_t)b->plan.probs.size();
    unsigned long long *res = reinterpret_cast<unsigned long long *>(b->arena + b->plan.off_res);
    j3d_status st = refresh_halos(b->plan, b->arena, 0, (int32_t)b->plan.blocks.size(), 0, b->stream);
    if (st != J3D_OK) return st;
    st = hip_status(launch_fill_u64(res, count, 0ull, b->stream), "residual reset");
    if (st != J3D_OK) return st;
    SweepArgs a;
    std::memset(&a, 0, sizeof a);
    a.base = reinterpret_cast<double *>(b->arena);
    a.blocks = reinterpret_cast<const BlockDesc *>(b->arena + b->plan.off_blocks);
    a.probs = reinterpret_cast<const ProbDesc *>(b->arena + b->plan.off_probs);
    a.tiles = reinterpret_cast<const Tile *>(b->arena + b->plan.off_tiles);
    a.res = res;
    a.queue = reinterpret_cast<unsigned int *>(b->arena + b->plan.off_queue);
    a.zchunk = b->zchunk;
    int32_t active = count;
    for (int64_t s = 0; s < b->max_iters; ++s) {
        while (active > 0 && b->plan.probs[b->order[active - 1]].iters <= s) --active;
        a.step = s;
        a.tile_begin = 0;
        a.tile_count = b->prefix_tiles[active];
        a.flags = SW_FUSED | SW_MULTI;
        int grid;
        if (b->tune.blocks_per_cu > 0) {
            a.flags |= SW_PERSIST;
            a.queue_slot = (int)(b->persist_launches++ & 1);
            grid = std::min(a.tile_count, b->cus * b->tune.blocks_per_cu);
        } else {
            grid = xcd_split(b->work, 0, a.tile_count, a.xcut);
        }
        st = hip_status(launch_sweep(b->tune.variant, a, grid, b->stream), "batch sweep launch");
        if (st != J3D_OK) return st;
    }
    b->ran = true;
    b->final_parity.resize(count);
    for (int32_t i = 0; i < count; ++i) b->final_parity[i] = (int)(b->plan.probs[i].iters & 1);
    if (residuals_out) {
        std::vector<unsigned long long> bits(count);
        st = hip_status(hipMemcpyAsync(bits.data(), res, count * sizeof(unsigned long long),
                                       hipMemcpyDeviceToHost, b->stream),
                        "residual readback");
        if (st == J3D_OK) st = hip_status(hipStreamSynchronize(b->stream), "residual readback");
        if (st != J3D_OK) return st;
        for (int32_t i = 0; i < count; ++i) std::memcpy(&residuals_out[i], &bits[i], sizeof(double));
    }
    return J3D_OK;
}

j3d_status j3d_batch_run_two_sweep(j3d_batch *b, double *residuals_out)
{
    if (!b) return set_error(J3D_EINVAL, "batch is NULL");
    if (b->ran) return set_error(J3D_ESTATE, "batch already ran");
    const int32_t count = (int32_t)b->plan.probs.size();
    for (int32_t i = 0; i < count; ++i)
        if (b->plan.probs[i].nblocks != 1)
            return set_error(J3D_EINVAL, "two sweeps per launch need undivided problems (problem %d has %d blocks)",
                             i, b->plan.probs[i].nblocks);
    // two-sweep tiles: problems by pair count, longest first, so the tiles
    // active at pair step s are a prefix of the table
    constexpr int kZchunk = 64;  // measured: 32 and 128 were 3% and 5% slower on the batched workload
    std::vector<int32_t> order(count);
    for (int32_t i = 0; i < count; ++i) order[i] = i;
    std::stable_sort(order.begin(), order.end(), [&](int32_t x, int32_t y) {
        return b->plan.probs[x].iters / 2 > b->plan.probs[y].iters / 2;
    });
    std::vector<Tile> tiles2;
    std::vector<int32_t> prefix2(1, 0);
    for (int32_t k = 0; k < count; ++k) {
        const ProbPlan &pp = b->plan.probs[order[k]];
        twostep_make_tiles(b->plan.blocks.data(), pp.block_begin, pp.block_begin + 1, kZchunk, &tiles2);
        prefix2.push_back((int32_t)tiles2.size());
    }
    if (tiles2.size() > b->plan.tiles_cap)
        return set_error(J3D_EINVAL, "two-sweep tiles (%zu) exceed the tile table (%llu)", tiles2.size(),
                         (unsigned long long)b->plan.tiles_cap);

    unsigned long long *res = reinterpret_cast<unsigned long long *>(b->arena + b->plan.off_res);
    ProbDesc *probs_dev = reinterpret_cast<ProbDesc *>(b->arena + b->plan.off_probs);
    j3d_status st = hip_status(launch_fill_u64(res, count, 0ull, b->stream), "residual reset");
    if (st != J3D_OK) return st;
    auto upload_probs = [&](const std::vector<ProbDesc> &pd) {
        j3d_status r = hip_status(hipMemcpyAsync(probs_dev, pd.data(), pd.size() * sizeof(ProbDesc),
                                                 hipMemcpyHostToDevice, b->stream),
                                  "problem table");
        return r == J3D_OK ? hip_status(hipStreamSynchronize(b->stream), "problem table") : r;
    };
    std::vector<ProbDesc> pd(count);
    // an odd count starts with one ordinary sweep (residual only if it is the last)
    bool any_odd = false;
    for (int32_t i = 0; i < count; ++i) {
        std::memset(&pd[i], 0, sizeof(ProbDesc));
        const int64_t it = b->plan.probs[i].iters;
        pd[i].limit = it & 1;
        pd[i].res_slot = i;
        pd[i].flags = it == 1 ? PF_RES_LAST : 0;
        any_odd = any_odd || (it & 1);
    }
    if (any_odd) {
        st = upload_probs(pd);
        if (st != J3D_OK) return st;
        SweepArgs a;
        std::memset(&a, 0, sizeof a);
        a.base = reinterpret_cast<double *>(b->arena);
        a.blocks = reinterpret_cast<const BlockDesc *>(b->arena + b->plan.off_blocks);
        a.probs = probs_dev;
        a.tiles = reinterpret_cast<const Tile *>(b->arena + b->plan.off_tiles);
        a.res = res;
        a.queue = reinterpret_cast<unsigned int *>(b->arena + b->plan.off_queue);
        a.zchunk = b->zchunk;
        a.step = 0;
        a.tile_count = b->prefix_tiles[count];
        a.flags = SW_FUSED | SW_MULTI;
        int grid;
        if (b->tune.blocks_per_cu > 0) {
            a.flags |= SW_PERSIST;
            a.queue_slot = (int)(b->persist_launches++ & 1);
            grid = std::min(a.tile_count, b->cus * b->tune.blocks_per_cu);
        } else {
            grid = xcd_split(b->work, 0, a.tile_count, a.xcut);
        }
        st = hip_status(launch_sweep(b->tune.variant, a, grid, b->stream), "batch sweep launch");
        if (st != J3D_OK) return st;
    }
    // then iters / 2 two-sweep launches per problem
    for (int32_t i = 0; i < count; ++i) {
        const int64_t it = b->plan.probs[i].iters;
        pd[i].base = it & 1;
        pd[i].limit = it / 2;
        pd[i].flags = 0;
    }
    st = upload_probs(pd);
    if (st == J3D_OK) st = upload_tiles(b->plan, tiles2, b->arena, b->stream);
    if (st != J3D_OK) return st;
    TwoStepArgs a2;
    std::memset(&a2, 0, sizeof a2);
    a2.base = reinterpret_cast<double *>(b->arena);
    a2.blocks = reinterpret_cast<const BlockDesc *>(b->arena + b->plan.off_blocks);
    a2.probs = probs_dev;
    a2.tiles = reinterpret_cast<const Tile *>(b->arena + b->plan.off_tiles);
    a2.res = res;
    a2.zchunk = kZchunk;
    int32_t active = count;
    const int64_t max_pairs = count > 0 ? b->plan.probs[order[0]].iters / 2 : 0;
    for (int64_t s2 = 0; s2 < max_pairs; ++s2) {
        while (active > 0 && b->plan.probs[order[active - 1]].iters / 2 <= s2) --active;
        a2.step = s2;
        a2.tile_begin = 0;
        a2.tile_count = prefix2[active];
        st = hip_status(launch_twostep(a2, b->stream), "two-sweep batch launch");
        if (st != J3D_OK) return st;
    }
    b->ran = true;
    b->final_parity.resize(count);
    for (int32_t i = 0; i < count; ++i) {
        const int64_t it = b->plan.probs[i].iters;
        b->final_parity[i] = (int)(((it & 1) + it / 2) & 1);
    }
    if (residuals_out) {
        std::vector<unsigned long long> bits(count);
        st = hip_status(hipMemcpyAsync(bits.data(), res, count * sizeof(unsigned long long),
                                       hipMemcpyDeviceToHost, b->stream),
                        "residual readback");
        if (st == J3D_OK) st = hip_status(hipStreamSynchronize(b->stream), "residual readback");
        if (st != J3D_OK) return st;
        for (int32_t i = 0; i < count; ++i) std::memcpy(&residuals_out[i], &bits[i], sizeof(double));
    }
    return J3D_OK;
}

j3d_status j3d_batch_get_interior(j3d_batch *b, int32_t i, double *dst, int dst_on_device)
{
    if (!b || !dst) return set_error(J3D_EINVAL, "NULL argument");
    if (i < 0 || i >= (int32_t)b->plan.probs.size()) return set_error(J3D_EINVAL, "problem %d out of range", i);
    const int parity = b->ran ? b->final_parity[i] : 0;
    return copy_dense(b->plan, b->arena, i, parity, dst, dst_on_device, true, b->stream);
}

j3d_status j3d_batch_destroy(j3d_batch *b)
{
    if (!b) return set_error(J3D_EINVAL, "batch is NULL");
    j3d_status st = hip_status(hipStreamSynchronize(b->stream), "batch destroy");
    delete b;
    return st;
}

// ---- measurement helpers --------------------------------------------------------

j3d_status j3d_device_copy(void *dst, const void *src, uint64_t bytes, void *hip_stream)
{
    if (!dst || !src) return set_error(J3D_EINVAL, "NULL argument");
    if (bytes % 16) return set_error(J3D_EINVAL, "bytes must be a multiple of 16");
    if (reinterpret_cast<uintptr_t>(dst) % 16 || reinterpret_cast<uintptr_t>(src) % 16)
        return set_error(J3D_EINVAL, "copy buffers must be 16-byte aligned");
    int dev = 0;
    j3d_status st = require_device(&dev, nullptr);
    if (st != J3D_OK) return st;
    return hip_status(launch_copy(dst, src, bytes, hip_stream), "copy launch");
}

j3d_status j3d_device_cus(int32_t *cus)
{
    if (!cus) return set_error(J3D_EINVAL, "cus is NULL");
    int n = 0;
    j3d_status st = require_device(nullptr, &n);
    if (st != J3D_OK) return st;
    *cus = n;
    return J3D_OK;
}

}  // extern "C"
