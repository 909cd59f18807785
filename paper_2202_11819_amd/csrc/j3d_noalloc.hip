// j3d_noalloc.hip -- a solve that allocates no device memory.
//
// j3d_solve_noalloc runs the fused sweep of j3d_run (strategy C, one launch
// per iteration for all blocks) on fields that live in memory the caller
// passes, and keeps everything else it needs on the device (block and
// problem descriptors, the tile table, the per-axis maps of the dense
// copies, the residual word) in one file-scope device array of fixed size.
// It is for callers that cannot allocate: code under stream capture, tight
// serving loops, harnesses that forbid allocation.  It calls no hipMalloc,
// hipFree, hipHostMalloc, graph or stream creation.
//
// The array is per device: each GPU the library runs on holds its own copy
// until the process ends, and every call on that GPU uses it, so calls that
// overlap on one GPU (two host threads, or two streams) race for it.  Its
// contents persist from call to call; the residual word is cleared by a fill
// kernel before use, and every other table is rewritten by each call.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <mutex>
#include <vector>

#include "j3d_device.hpp"

namespace j3d {

constexpr uint64_t kScratchBytes = 4ull << 20;  // descriptor, tile and map tables

// The scratch array.  In host code this name is only a stand-in for the
// symbol: its device address comes from hipGetSymbolAddress (per device), and
// only that address is passed to kernels and copies.
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};

// Device address of this device's scratch array, looked up once per device
// with that device current.
j3d_status scratch_address(int dev, char **out)
{
    if (dev < 0 || dev >= kMaxDevices) return set_error(J3D_EDEVICE, "device %d out of range", dev);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr) return hip_status(e == hipSuccess ? hipErrorInvalidSymbol : e, "scratch address");
        g_scratch_ptr[dev] = ptr;
    }
    *out = static_cast<char *>(g_scratch_ptr[dev]);
    return J3D_OK;
}

// x-halo arrays of parity p filled from the x neighbours' current iterate
// (their boundary column next to the shared face): the exchange the fused
// sweep needs before its first launch, read straight across the block
// boundary (no send/receive buffers).  x neighbours share ey and ez.
__global__ __launch_bounds__(256) void xhalo_pull_kernel(double *base, const BlockDesc *blocks, int nblocks,
                                                         int parity)
{
    for (int b = blockIdx.y; b < nblocks; b += gridDim.y) {
        const BlockDesc &B = blocks[b];
        const int ey = B.ext[1], ez = B.ext[2];
        const int64_t fx = (int64_t)ey * ez;
        double *X = base + B.xoff[parity];
        for (int side = 0; side < 2; ++side) {
            if (B.nbr[side] < 0) continue;
            const BlockDesc &N = blocks[B.nbr[side]];
            const int64_t nps = plane_stride(N.pitch, N.ext[1]);
            const double *F = base + N.off[parity] + (side == 0 ? N.ext[0] - 1 : 0);
            for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < fx;
                 i += (int64_t)gridDim.x * blockDim.x) {
                const int64_t y = i % ey, z = i / ey;
                X[side * fx + i] = F[(z + 1) * nps + (y + 1) * N.pitch];
            }
        }
    }
}

struct Layout {
    uint64_t off_blocks, off_probs, off_tiles, off_maps, off_res, total;
};

Layout scratch_layout(size_t nblocks, size_t ntiles, size_t nmaps)
{
    Layout l;
    uint64_t o = 0;
    l.off_blocks = o;
    o = align_up(o + nblocks * sizeof(BlockDesc), 256);
    l.off_probs = o;
    o = align_up(o + sizeof(ProbDesc), 256);
    l.off_tiles = o;
    o = align_up(o + ntiles * sizeof(Tile), 256);
    l.off_maps = o;
    o = align_up(o + nmaps * sizeof(int32_t), 256);
    l.off_res = o;
    o = align_up(o + sizeof(uint64_t), 256);
    l.total = o;
    return l;
}

}  // namespace
}  // namespace j3d

using namespace j3d;

extern "C" j3d_status j3d_solve_noalloc(const j3d_problem *p, void *fields, uint64_t fields_bytes,
                                        const double *interior_in, double *interior_out, int64_t iters,
                                        double *residual_out, void *hip_stream)
{
    // ---- validation, before any device work ----
    if (!p || !fields || !interior_out) return set_error(J3D_EINVAL, "NULL argument");
    if (reinterpret_cast<uintptr_t>(fields) % 256) return set_error(J3D_EINVAL, "fields not 256-byte aligned");
    if (iters < 0) return set_error(J3D_EINVAL, "iters %lld < 0", (long long)iters);
    Plan plan;
    j3d_status st = make_plan(1, p, false, &plan);
    if (st != J3D_OK) return st;
    const ProbPlan &pp = plan.probs[0];
    const int64_t *n = pp.d.n;
    // the two iterates of every block, then the x-halo arrays, packed in the
    // caller's buffer (offsets in doubles from `fields`)
    uint64_t o = 0;
    for (int q = 0; q < 2; ++q)
        for (BlockDesc &B : plan.blocks) {
            B.off[q] = (int64_t)o;
            o += (uint64_t)block_field_cells(B.ext[0], B.ext[1], B.ext[2]);
        }
    for (int q = 0; q < 2; ++q)
        for (BlockDesc &B : plan.blocks) {
            B.xoff[q] = (int64_t)o;
            o += 2ull * B.ext[1] * B.ext[2];
        }
    link_halo_sources(plan.blocks.data(), plan.blocks.size());  // from the offsets just set
    if (fields_bytes < o * sizeof(double))
        return set_error(J3D_ENOMEM, "fields hold %llu bytes, %llu needed (j3d_field_bytes)",
                         (unsigned long long)fields_bytes, (unsigned long long)(o * sizeof(double)));
    const uint64_t cells = (uint64_t)(n[0] * n[1] * n[2]);
    const char *fb = static_cast<const char *>(fields), *fe = fb + o * sizeof(double);
    auto overlaps = [&](const void *q) {
        const char *a = static_cast<const char *>(q);
        return q && a < fe && a + cells * sizeof(double) > fb;
    };
    if (overlaps(interior_in) || overlaps(interior_out))
        return set_error(J3D_EINVAL, "interior arrays overlap the fields");
    int dev = 0, cus = 0;
    st = require_device(&dev, &cus);
    if (st != J3D_OK) return st;
    j3d_tune t;
    default_tune(plan, cus, &t);
    std::vector<Tile> tiles;
    make_tiles(plan, 0, (int32_t)plan.blocks.size(), t.variant, t.zchunk, &tiles, nullptr);
    std::vector<int32_t> maps;
    for (int a = 0; a < 3; ++a)
        for (int32_t b = 0; b < pp.d.nb[a]; ++b)
            for (int64_t l = 0; l < pp.d.ext[a][b]; ++l) {
                maps.push_back(b);
                maps.push_back((int32_t)l);
            }
    const Layout lay = scratch_layout(plan.blocks.size(), tiles.size(), maps.size());
    if (lay.total > kScratchBytes)
        return set_error(J3D_EINVAL, "problem needs %llu bytes of tables (%zu blocks, %zu tiles), more than the %llu "
                         "of the static scratch", (unsigned long long)lay.total, plan.blocks.size(), tiles.size(),
                         (unsigned long long)kScratchBytes);
    char *scr = nullptr;
    st = scratch_address(dev, &scr);
    if (st != J3D_OK) return st;

    // ---- tables into the scratch (the host copies are consumed before return) ----
    hipStream_t stream = static_cast<hipStream_t>(hip_stream);
    ProbDesc prob;
    std::memset(&prob, 0, sizeof prob);
    prob.limit = iters;
    prob.flags = PF_RES_LAST;
    st = hip_status(hipMemcpyAsync(scr + lay.off_blocks, plan.blocks.data(), plan.blocks.size() * sizeof(BlockDesc),
                                   hipMemcpyHostToDevice, stream),
                    "table upload");
    if (st == J3D_OK)
        st = hip_status(hipMemcpyAsync(scr + lay.off_probs, &prob, sizeof prob, hipMemcpyHostToDevice, stream),
                        "table upload");
    if (st == J3D_OK && !tiles.empty())
        st = hip_status(hipMemcpyAsync(scr + lay.off_tiles, tiles.data(), tiles.size() * sizeof(Tile),
                                       hipMemcpyHostToDevice, stream),
                        "table upload");
    if (st == J3D_OK)
        st = hip_status(hipMemcpyAsync(scr + lay.off_maps, maps.data(), maps.size() * sizeof(int32_t),
                                       hipMemcpyHostToDevice, stream),
                        "table upload");
    if (st == J3D_OK) st = hip_status(hipStreamSynchronize(stream), "table upload");
    if (st != J3D_OK) return st;

    double *base = static_cast<double *>(fields);
    const BlockDesc *dblocks = reinterpret_cast<const BlockDesc *>(scr + lay.off_blocks);
    const int32_t *dmaps = reinterpret_cast<const int32_t *>(scr + lay.off_maps);
    unsigned long long *res = reinterpret_cast<unsigned long long *>(scr + lay.off_res);
    const int32_t nb = (int32_t)plan.blocks.size();

    // ---- initial iterate: halo storage (Dirichlet values) and the interior ----
    int64_t maxc = 0, maxx = 0;
    for (const BlockDesc &B : plan.blocks) {
        maxc = std::max<int64_t>(maxc, block_field_cells(B.ext[0], B.ext[1], B.ext[2]));
        maxx = std::max<int64_t>(maxx, (int64_t)B.ext[1] * B.ext[2]);
    }
    st = hip_status(launch_init(base, dblocks, 0, nb, (int32_t)maxc, (int32_t)maxx, 0, n, pp.s0, pp.bc,
                                interior_in ? 0 : 1, stream),
                    "init launch");
    if (st == J3D_OK && interior_in)
        st = hip_status(launch_scatter(base, dblocks, 0, pp.d.nb, dmaps, n, 0, n[2], interior_in, 0, stream),
                        "scatter launch");
    if (st == J3D_OK && nb > 1) {
        hipLaunchKernelGGL(xhalo_pull_kernel, dim3((unsigned)std::min<int64_t>((maxx + 255) / 256, 1024),
                                                   (unsigned)std::min<int32_t>(nb, 65535)),
                           dim3(256), 0, stream, base, dblocks, nb, 0);
        st = hip_status(hipGetLastError(), "x-halo launch");
    }
    if (st == J3D_OK && residual_out)
        st = hip_status(launch_fill_u64(res, 1, 0ull, stream), "residual reset");

    // ---- iterations: one fused launch each (strategy C for all blocks) ----
    SweepArgs a;
    std::memset(&a, 0, sizeof a);
    a.base = base;
    a.blocks = dblocks;
    a.probs = reinterpret_cast<const ProbDesc *>(scr + lay.off_probs);
    a.tiles = reinterpret_cast<const Tile *>(scr + lay.off_tiles);
    a.res = res;
    int ezm = 1;  // a z-chunk of 0 means whole blocks, as make_tiles reads it
    for (const BlockDesc &B : plan.blocks) ezm = std::max(ezm, B.ext[2]);
    a.zchunk = t.zchunk > 0 ? t.zchunk : ezm;
    a.tile_count = (int32_t)tiles.size();
    for (int64_t k = 0; k < iters && st == J3D_OK; ++k) {
        a.parity = (int32_t)(k & 1);
        a.flags = SW_FUSED | (residual_out && k + 1 == iters ? SW_RES : 0);
        st = hip_status(launch_sweep(t.variant, a, a.tile_count, stream), "sweep launch");
    }
    if (st == J3D_OK)
        st = hip_status(launch_gather(base, dblocks, 0, pp.d.nb, dmaps, n, 0, n[2], interior_out, (int)(iters & 1),
                                      stream),
                        "gather launch");
    if (st != J3D_OK) return st;
    if (!residual_out) return J3D_OK;
    if (iters == 0) {
        *residual_out = 0.0;
        return J3D_OK;
    }
    unsigned long long bits = 0;
    st = hip_status(hipMemcpyAsync(&bits, res, sizeof bits, hipMemcpyDeviceToHost, stream), "residual readback");
    if (st == J3D_OK) st = hip_status(hipStreamSynchronize(stream), "residual readback");
    if (st != J3D_OK) return st;
    std::memcpy(residual_out, &bits, sizeof bits);
    return J3D_OK;
}
