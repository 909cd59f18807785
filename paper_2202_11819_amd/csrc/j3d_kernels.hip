// j3d_kernels.hip -- gfx950 kernels of the Jacobi3D hot path and their launchers.
//
// The sweep (Jacobi update, fused with the halo hand-off of kernel-fusion
// strategy C, Sec. III-D-1) is the only kernel that runs per iteration in the
// fused and graph modes.  It is bound by HBM bandwidth (7 flops per 16 bytes),
// so it is built for streaming: a workgroup owns an x-y tile of one block and
// marches along z; every cell is read from HBM once (x-contiguous rows, whole
// 64-lane waves per row segment) and written once; the four in-plane
// neighbours come from a double-buffered LDS copy of the current plane with a
// one-cell ring, the two z-neighbours from registers.  Halo values are read
// where the neighbour block wrote them, and a cell on a block face writes its
// new value straight into the neighbour's halo storage of the next iterate
// (pack, exchange and unpack as a single store).  The other kernels here are
// the unfused pack / exchange / unpack of Fig. 1 and Fig. 3, the seeded
// initialisation, and dense <-> block copies.
//
// Arithmetic of the update, fixed for bit-exact results: the 7-term sum in the
// order centre, x-, x+, y-, y+, z-, z+, each addition rounded, then one
// multiplication by fl(1/7); no contraction (built with -ffp-contract=off).
#include <hip/hip_runtime.h>

#include <cstdint>

#include "j3d_internal.hpp"

namespace j3d {
namespace {

constexpr double kW = 1.0 / 7.0;                    // fl(1/7)
constexpr uint64_t kGamma = 0x9E3779B97F4A7C15ull;  // SplitMix64 Weyl increment
constexpr int kXcds = 8;                            // XCDs per MI355X

__device__ __forceinline__ uint64_t splitmix64_mix(uint64_t z)
{
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

// Output g+1 of the SplitMix64 stream that starts in state s0, mapped to [0,1).
__device__ __forceinline__ double seeded_value(uint64_t s0, uint64_t g)
{
    const uint64_t h = splitmix64_mix(s0 + (g + 1) * kGamma);
    return (double)(h >> 11) * (1.0 / 9007199254740992.0);
}

__device__ __forceinline__ unsigned int atomic_add_agent(unsigned int *p, unsigned int v)
{
    return __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ void atomic_store_agent(unsigned int *p, unsigned int v)
{
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ void atomic_max_agent(unsigned long long *p, unsigned long long v)
{
    __hip_atomic_fetch_max(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Workgroups of a launch are dispatched round-robin over the XCDs (workgroup
// i to XCD i % 8).  Give each XCD a contiguous run of tiles so that tiles
// sharing halo rows run together under one L2.
__device__ __forceinline__ int xcd_remap(int i, int n)
{
    const int q = n / kXcds, r = n % kXcds;
    const int x = i % kXcds, j = i / kXcds;
    return x * q + min(x, r) + j;
}

// ---- the sweep ----------------------------------------------------------------

template <int TX, int NTY, int RY>
struct Shape {
    static constexpr int TY = NTY * RY;   // tile rows
    static constexpr int NT = TX * NTY;   // threads
    static constexpr int LX = TX + 2;     // LDS plane with a one-cell ring
    static constexpr int LY = TY + 2;
    static constexpr int LDS = 2 * LX * LY;
    static_assert(NT >= 2 * TX + 2 * TY, "every halo cell of a plane needs a loader thread");
    static_assert(NT % 64 == 0, "whole waves");
};

template <int TX, int NTY, int RY>
__device__ __forceinline__ void sweep_tile(const SweepArgs &a, const Tile tl, double *sm, double *red)
{
    using S = Shape<TX, NTY, RY>;
    const BlockDesc *__restrict__ B = a.blocks + tl.block;
    const ProbDesc *__restrict__ P = a.probs + B->prob;

    int p;
    bool want_res;
    if (a.flags & SW_MULTI) {
        const int64_t t = P->base + a.step;
        if (t >= P->limit) return;  // uniform over the workgroup
        p = (int)(t & 1);
        const int64_t t1 = t + 1;
        want_res = ((P->flags & PF_RES_LAST) && t1 == P->limit) ||
                   (P->check_every > 0 && t1 % P->check_every == 0);
    } else {
        p = a.parity;
        want_res = (a.flags & SW_RES) != 0;
    }
    const bool fused = (a.flags & SW_FUSED) != 0;

    const int ex = B->ext[0], ey = B->ext[1], ez = B->ext[2];
    const int PS = (ey + 2) * ex;  // plane stride of the field
    const double *__restrict__ cur = a.base + B->off[p];
    double *__restrict__ nxt = a.base + B->off[p ^ 1];

    const int x0 = tl.tx * TX, y0 = tl.ty * S::TY, z0 = tl.tz * a.zchunk;
    const int nxv = min(TX, ex - x0), nyv = min(S::TY, ey - y0), nzv = min(a.zchunk, ez - z0);

    const int tid = threadIdx.x;
    const int tx = tid % TX, ty = tid / TX;
    const int x = x0 + tx;
    const bool vx = tx < nxv;

    // Destinations of this block's face values in the neighbours' halo
    // storage of the next iterate (null: global boundary or unfused).
    double *dxm = nullptr, *dxp = nullptr, *dym = nullptr, *dyp = nullptr, *dzm = nullptr,
           *dzp = nullptr;
    int psym = 0, psyp = 0;
    if (fused) {
        const int q = p ^ 1;
        if (B->nbr[0] >= 0) dxm = a.base + a.blocks[B->nbr[0]].xoff[q] + (int64_t)ey * ez;
        if (B->nbr[1] >= 0) dxp = a.base + a.blocks[B->nbr[1]].xoff[q];
        if (B->nbr[2] >= 0) {
            const BlockDesc *N = a.blocks + B->nbr[2];
            psym = (N->ext[1] + 2) * ex;
            dym = a.base + N->off[q] + (int64_t)(N->ext[1] + 1) * ex;
        }
        if (B->nbr[3] >= 0) {
            const BlockDesc *N = a.blocks + B->nbr[3];
            psyp = (N->ext[1] + 2) * ex;
            dyp = a.base + N->off[q];
        }
        if (B->nbr[4] >= 0) {
            const BlockDesc *N = a.blocks + B->nbr[4];
            dzm = a.base + N->off[q] + (int64_t)(N->ext[2] + 1) * PS;
        }
        if (B->nbr[5] >= 0) dzp = a.base + a.blocks[B->nbr[5]].off[q];
    }

    // This thread's cells: rows y0 + ty + NTY*r of column x.
    bool vr[RY];
    int col[RY];  // field offset of (x, y_r) in plane index 0
#pragma unroll
    for (int r = 0; r < RY; ++r) {
        const int ly = ty + NTY * r;
        vr[r] = vx && ly < nyv;
        col[r] = (y0 + ly + 1) * ex + x;
    }

    // Halo loader role: one ring cell of the LDS plane per thread.
    int hl = -1;
    const double *__restrict__ hsrc = nullptr;
    int hstep = 0;
    if (tid < 2 * TX) {
        const int side = tid / TX, xx = tid % TX;
        if (xx < nxv) {
            const int row = side ? (y0 + nyv) : (y0 - 1);  // a halo row when at the block edge
            hsrc = cur + PS + (row + 1) * ex + x0 + xx;
            hstep = PS;
            hl = (side ? (nyv + 1) : 0) * S::LX + xx + 1;
        }
    } else if (tid < 2 * TX + 2 * S::TY) {
        const int u = tid - 2 * TX;
        const int side = u / S::TY, yy = u % S::TY;
        if (yy < nyv) {
            const int y = y0 + yy;
            if (side == 0) {
                if (x0 == 0) {
                    hsrc = a.base + B->xoff[p] + y;
                    hstep = ey;
                } else {
                    hsrc = cur + PS + (y + 1) * ex + x0 - 1;
                    hstep = PS;
                }
                hl = (yy + 1) * S::LX;
            } else {
                const int xr = x0 + nxv;
                if (xr == ex) {
                    hsrc = a.base + B->xoff[p] + (int64_t)ey * ez + y;
                    hstep = ey;
                } else {
                    hsrc = cur + PS + (y + 1) * ex + xr;
                    hstep = PS;
                }
                hl = (yy + 1) * S::LX + nxv + 1;
            }
        }
    }

    double zm[RY], c[RY], zp[RY], zq[RY];
#pragma unroll
    for (int r = 0; r < RY; ++r) {
        zm[r] = c[r] = zp[r] = zq[r] = 0.0;
        if (vr[r]) {
            const double *q = cur + col[r];
            zm[r] = q[z0 * PS];            // plane z0-1 (the z- halo when z0 == 0)
            c[r] = q[(z0 + 1) * PS];       // plane z0
            zp[r] = q[(z0 + 2) * PS];      // plane z0+1 (the z+ halo when z0 == ez-1)
        }
    }
    double h = (hl >= 0) ? hsrc[(int64_t)z0 * hstep] : 0.0;
    double rmax = 0.0;

    for (int kk = 0; kk < nzv; ++kk) {
        const int k = z0 + kk;
        const bool more = kk + 1 < nzv;
        double hn = 0.0;
        if (more) {
#pragma unroll
            for (int r = 0; r < RY; ++r)
                if (vr[r]) zq[r] = cur[col[r] + (k + 3) * PS];  // plane k+2
            if (hl >= 0) hn = hsrc[(int64_t)(k + 1) * hstep];
        }
        double *L = sm + (kk & 1) * (S::LX * S::LY);
#pragma unroll
        for (int r = 0; r < RY; ++r)
            if (vr[r]) L[(ty + NTY * r + 1) * S::LX + tx + 1] = c[r];
        if (hl >= 0) L[hl] = h;
        __syncthreads();
#pragma unroll
        for (int r = 0; r < RY; ++r) {
            if (!vr[r]) continue;
            const int li = (ty + NTY * r + 1) * S::LX + tx + 1;
            double s = c[r];
            s += L[li - 1];
            s += L[li + 1];
            s += L[li - S::LX];
            s += L[li + S::LX];
            s += zm[r];
            s += zp[r];
            const double v = s * kW;
            nxt[col[r] + (k + 1) * PS] = v;
            if (fused) {
                const int y = y0 + ty + NTY * r;
                if (x == 0 && dxm) dxm[y + ey * k] = v;
                if (x == ex - 1 && dxp) dxp[y + ey * k] = v;
                if (y == 0 && dym) dym[(k + 1) * psym + x] = v;
                if (y == ey - 1 && dyp) dyp[(k + 1) * psyp + x] = v;
                if (k == 0 && dzm) dzm[(y + 1) * ex + x] = v;
                if (k == ez - 1 && dzp) dzp[(y + 1) * ex + x] = v;
            }
            if (want_res) {
                const double d = fabs(v - c[r]);
                rmax = d > rmax ? d : rmax;
            }
        }
#pragma unroll
        for (int r = 0; r < RY; ++r) {
            zm[r] = c[r];
            c[r] = zp[r];
            zp[r] = zq[r];
        }
        h = hn;
    }

    if (want_res) {
        // max over the workgroup, then one atomic per tile; the maximum of
        // non-negative doubles orders like their bit patterns, so the result
        // is exact and independent of the order of arrival.
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) {
            const double t = __shfl_xor(rmax, o);
            rmax = t > rmax ? t : rmax;
        }
        if ((tid & 63) == 0) red[tid >> 6] = rmax;
        __syncthreads();
        if (tid == 0) {
            double m = 0.0;
            for (int w = 0; w < S::NT / 64; ++w) m = red[w] > m ? red[w] : m;
            atomic_max_agent(a.res + P->res_slot, (unsigned long long)__double_as_longlong(m));
        }
    }
    __syncthreads();  // the next tile of a persistent workgroup reuses the LDS
}

template <int TX, int NTY, int RY>
__global__ __launch_bounds__(TX *NTY) void sweep_kernel(SweepArgs a)
{
    using S = Shape<TX, NTY, RY>;
    __shared__ double sm[S::LDS];
    __shared__ double red[S::NT / 64];
    __shared__ int next_tile;

    if (a.flags & SW_PERSIST) {
        // Per-XCD queues over contiguous tile ranges; a workgroup drains its
        // own XCD's queue, then helps the others.
        const int xcd = blockIdx.x % kXcds;
        for (int qi = 0; qi < kXcds; ++qi) {
            const int q = (xcd + qi) % kXcds;
            const int beg = (int)((int64_t)a.tile_count * q / kXcds);
            const int end = (int)((int64_t)a.tile_count * (q + 1) / kXcds);
            for (;;) {
                if (threadIdx.x == 0)
                    next_tile = beg + (int)atomic_add_agent(a.queue + a.queue_slot * kXcds + q, 1u);
                __syncthreads();
                const int t = next_tile;
                __syncthreads();
                if (t >= end) break;
                sweep_tile<TX, NTY, RY>(a, a.tiles[a.tile_begin + t], sm, red);
            }
        }
        // Re-arm the other half of the counters for the next persistent launch.
        if (blockIdx.x == 0 && threadIdx.x < kXcds)
            atomic_store_agent(a.queue + (a.queue_slot ^ 1) * kXcds + threadIdx.x, 0u);
    } else {
        const int t = xcd_remap(blockIdx.x, gridDim.x);
        sweep_tile<TX, NTY, RY>(a, a.tiles[a.tile_begin + t], sm, red);
    }
}

// ---- unfused halo kernels (one thread per cell of the largest face) ----------

struct FaceGeom {
    int ex, ey, ez, PS, fx, fy, fz;
    int64_t o[6];  // offsets of the six faces inside S[b] / R[b]
};

__device__ __forceinline__ FaceGeom face_geom(const BlockDesc &B)
{
    FaceGeom g;
    g.ex = B.ext[0];
    g.ey = B.ext[1];
    g.ez = B.ext[2];
    g.PS = (g.ey + 2) * g.ex;
    g.fx = g.ey * g.ez;
    g.fy = g.ex * g.ez;
    g.fz = g.ex * g.ey;
    g.o[0] = 0;
    g.o[1] = g.fx;
    g.o[2] = 2 * (int64_t)g.fx;
    g.o[3] = g.o[2] + g.fy;
    g.o[4] = g.o[3] + g.fy;
    g.o[5] = g.o[4] + g.fz;
    return g;
}

// Field offset (within F) of face f's cell i, for the layer just inside the
// block (interior = true, used by pack) or its halo layer (unpack).  x faces
// are handled through the separate x-halo arrays when !interior.
__device__ __forceinline__ int64_t face_cell(const FaceGeom &g, int f, int i, bool interior)
{
    if (f < 2) {
        const int y = i % g.ey, z = i / g.ey;
        return (int64_t)(z + 1) * g.PS + (y + 1) * g.ex + (f == 0 ? 0 : g.ex - 1);
    }
    if (f < 4) {
        const int x = i % g.ex, z = i / g.ex;
        const int row = interior ? (f == 2 ? 1 : g.ey) : (f == 2 ? 0 : g.ey + 1);
        return (int64_t)(z + 1) * g.PS + row * g.ex + x;
    }
    const int x = i % g.ex, y = i / g.ex;
    const int plane = interior ? (f == 4 ? 1 : g.ez) : (f == 4 ? 0 : g.ez + 1);
    return (int64_t)plane * g.PS + (y + 1) * g.ex + x;
}

__device__ __forceinline__ int face_size(const FaceGeom &g, int f)
{
    return f < 2 ? g.fx : (f < 4 ? g.fy : g.fz);
}

__global__ __launch_bounds__(256) void pack_kernel(double *base, const BlockDesc *blocks,
                                                   int block_begin, int nblocks, int parity,
                                                   int face_mask)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    for (int bb = blockIdx.y; bb < nblocks; bb += gridDim.y) {
        const BlockDesc &B = blocks[block_begin + bb];
        const FaceGeom g = face_geom(B);
        const double *cur = base + B.off[parity];
        double *S = base + B.sr_off;
        for (int f = 0; f < 6; ++f) {
            if (!((face_mask >> f) & 1) || B.nbr[f] < 0 || i >= face_size(g, f)) continue;
            S[g.o[f] + i] = cur[face_cell(g, f, i, true)];
        }
    }
}

__global__ __launch_bounds__(256) void exchange_kernel(double *base, const BlockDesc *blocks,
                                                       int block_begin, int nblocks)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    for (int bb = blockIdx.y; bb < nblocks; bb += gridDim.y) {
        const BlockDesc &B = blocks[block_begin + bb];
        const FaceGeom g = face_geom(B);
        const double *S = base + B.sr_off;
        for (int f = 0; f < 6; ++f) {
            if (B.nbr[f] < 0 || i >= face_size(g, f)) continue;
            const BlockDesc &N = blocks[B.nbr[f]];
            const FaceGeom gn = face_geom(N);
            double *R = base + N.sr_off + N.face_total;
            R[gn.o[f ^ 1] + i] = S[g.o[f] + i];
        }
    }
}

__global__ __launch_bounds__(256) void unpack_kernel(double *base, const BlockDesc *blocks,
                                                     int block_begin, int nblocks, int parity,
                                                     int face_mask)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    for (int bb = blockIdx.y; bb < nblocks; bb += gridDim.y) {
        const BlockDesc &B = blocks[block_begin + bb];
        const FaceGeom g = face_geom(B);
        double *cur = base + B.off[parity];
        double *X = base + B.xoff[parity];
        const double *R = base + B.sr_off + B.face_total;
        for (int f = 0; f < 6; ++f) {
            if (!((face_mask >> f) & 1) || B.nbr[f] < 0 || i >= face_size(g, f)) continue;
            const double v = R[g.o[f] + i];
            if (f < 2)
                X[(f == 0 ? 0 : g.fx) + i] = v;
            else
                cur[face_cell(g, f, i, false)] = v;
        }
    }
}

// ---- initialisation and dense <-> block copies -----------------------------

__global__ __launch_bounds__(256) void init_kernel(double *base, const BlockDesc *blocks,
                                                   int block_begin, int nblocks, int parity,
                                                   int64_t n0, int64_t n1, uint64_t s0, double bc0,
                                                   double bc1, double bc2, double bc3, double bc4,
                                                   double bc5, int write_interior)
{
    const double bc[6] = {bc0, bc1, bc2, bc3, bc4, bc5};
    const double qnan = __builtin_nan("");
    for (int bb = blockIdx.y; bb < nblocks; bb += gridDim.y) {
        const BlockDesc &B = blocks[block_begin + bb];
        const int ex = B.ext[0], ey = B.ext[1], ez = B.ext[2];
        const int64_t cells = (int64_t)ex * (ey + 2) * (ez + 2);
        double *F0 = base + B.off[0];
        double *F1 = base + B.off[1];
        double *Fp = parity ? F1 : F0;
        const int64_t stride = (int64_t)gridDim.x * blockDim.x;
        for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < cells; idx += stride) {
            const int x = (int)(idx % ex);
            const int64_t rr = idx / ex;
            const int yy = (int)(rr % (ey + 2)), zz = (int)(rr / (ey + 2));
            const bool oy = (yy == 0 || yy == ey + 1), oz = (zz == 0 || zz == ez + 1);
            if (!oy && !oz) {
                if (write_interior) {
                    const uint64_t g = (uint64_t)(B.org[0] + x) +
                                       (uint64_t)n0 * ((uint64_t)(B.org[1] + yy - 1) +
                                                       (uint64_t)n1 * (uint64_t)(B.org[2] + zz - 1));
                    Fp[idx] = seeded_value(s0, g);
                }
                continue;
            }
            double v = qnan;  // halo of an interior face (filled by the exchange) or an edge
            if (oy && !oz) {
                const int f = yy == 0 ? 2 : 3;
                if (B.nbr[f] < 0) v = bc[f];
            } else if (oz && !oy) {
                const int f = zz == 0 ? 4 : 5;
                if (B.nbr[f] < 0) v = bc[f];
            }
            F0[idx] = v;
            F1[idx] = v;
        }
        const int64_t fx = (int64_t)ey * ez;
        for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < fx; idx += stride) {
            for (int q = 0; q < 2; ++q) {
                double *X = base + B.xoff[q];
                X[idx] = B.nbr[0] < 0 ? bc[0] : qnan;
                X[fx + idx] = B.nbr[1] < 0 ? bc[1] : qnan;
            }
        }
    }
}

struct DenseMap {
    const int32_t *mx, *my, *mz;  // (block coordinate, local coordinate) per global coordinate
    int32_t nb0, nb1, nb2;
};

// Arena offset (in doubles) of global interior cell (i, j, k) in parity `parity`.
__device__ __forceinline__ int64_t dense_to_block(const BlockDesc *blocks, int block_base,
                                                  const DenseMap &m, int64_t i, int64_t j,
                                                  int64_t k, int parity)
{
    const int bx = m.mx[2 * i], lx = m.mx[2 * i + 1];
    const int by = m.my[2 * j], ly = m.my[2 * j + 1];
    const int bz = m.mz[2 * k], lz = m.mz[2 * k + 1];
    const BlockDesc &B = blocks[block_base + bx + m.nb0 * (by + m.nb1 * bz)];
    const int ex = B.ext[0], ey = B.ext[1];
    return B.off[parity] + (int64_t)(lz + 1) * (ey + 2) * ex + (int64_t)(ly + 1) * ex + lx;
}

__global__ __launch_bounds__(256) void scatter_kernel(double *base, const BlockDesc *blocks,
                                                      int block_base, DenseMap m, int64_t n0,
                                                      int64_t n1, int64_t z0, int64_t count,
                                                      const double *src, int parity)
{
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; g < count; g += stride) {
        const int64_t i = g % n0, j = (g / n0) % n1, k = z0 + g / (n0 * n1);
        base[dense_to_block(blocks, block_base, m, i, j, k, parity)] = src[g];
    }
}

__global__ __launch_bounds__(256) void gather_kernel(const double *base, const BlockDesc *blocks,
                                                     int block_base, DenseMap m, int64_t n0,
                                                     int64_t n1, int64_t z0, int64_t count,
                                                     double *dst, int parity)
{
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; g < count; g += stride) {
        const int64_t i = g % n0, j = (g / n0) % n1, k = z0 + g / (n0 * n1);
        dst[g] = base[dense_to_block(blocks, block_base, m, i, j, k, parity)];
    }
}

__global__ __launch_bounds__(256) void set_face_kernel(double *base, const BlockDesc *blocks,
                                                       int block_base, DenseMap m, int64_t n0,
                                                       int64_t n1, int64_t n2, int face,
                                                       const double *src)
{
    const int axis = face / 2;
    const int64_t count = axis == 0 ? n1 * n2 : (axis == 1 ? n0 * n2 : n0 * n1);
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; g < count; g += stride) {
        int bx, by, bz, lx = 0, ly = 0, lz = 0;
        if (axis == 0) {
            const int64_t j = g % n1, k = g / n1;
            bx = face == 0 ? 0 : m.nb0 - 1;
            by = m.my[2 * j];
            ly = m.my[2 * j + 1];
            bz = m.mz[2 * k];
            lz = m.mz[2 * k + 1];
        } else if (axis == 1) {
            const int64_t i = g % n0, k = g / n0;
            by = face == 2 ? 0 : m.nb1 - 1;
            bx = m.mx[2 * i];
            lx = m.mx[2 * i + 1];
            bz = m.mz[2 * k];
            lz = m.mz[2 * k + 1];
        } else {
            const int64_t i = g % n0, j = g / n0;
            bz = face == 4 ? 0 : m.nb2 - 1;
            bx = m.mx[2 * i];
            lx = m.mx[2 * i + 1];
            by = m.my[2 * j];
            ly = m.my[2 * j + 1];
        }
        const BlockDesc &B = blocks[block_base + bx + m.nb0 * (by + m.nb1 * bz)];
        const int ex = B.ext[0], ey = B.ext[1], ez = B.ext[2];
        const int64_t PS = (int64_t)(ey + 2) * ex;
        const double v = src[g];
        for (int q = 0; q < 2; ++q) {
            if (axis == 0) {
                base[B.xoff[q] + (face == 1 ? (int64_t)ey * ez : 0) + ly + (int64_t)ey * lz] = v;
            } else if (axis == 1) {
                base[B.off[q] + (lz + 1) * PS + (int64_t)(face == 2 ? 0 : ey + 1) * ex + lx] = v;
            } else {
                base[B.off[q] + (face == 4 ? 0 : (int64_t)(ez + 1)) * PS + (int64_t)(ly + 1) * ex + lx] = v;
            }
        }
    }
}

__global__ __launch_bounds__(256) void gather_block_kernel(const double *base,
                                                           const BlockDesc *blocks, int block,
                                                           int parity, double *dst)
{
    const BlockDesc &B = blocks[block];
    const int ex = B.ext[0], ey = B.ext[1], ez = B.ext[2];
    const int64_t count = (int64_t)ex * ey * ez;
    const int64_t PS = (int64_t)(ey + 2) * ex;
    const double *F = base + B.off[parity];
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; g < count; g += stride) {
        const int64_t x = g % ex, y = (g / ex) % ey, z = g / ((int64_t)ex * ey);
        dst[g] = F[(z + 1) * PS + (y + 1) * ex + x];
    }
}

__global__ __launch_bounds__(256) void fill_u64_kernel(unsigned long long *p, int64_t count,
                                                       unsigned long long v)
{
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += stride) p[i] = v;
}

__global__ __launch_bounds__(256) void fill_u32_kernel(unsigned int *p, int64_t count, unsigned int v)
{
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += stride) p[i] = v;
}

// Streaming copy, 16 bytes per thread per iteration.
__global__ __launch_bounds__(256) void copy_kernel(uint4 *__restrict__ dst,
                                                   const uint4 *__restrict__ src, int64_t n16)
{
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n16; i += stride)
        dst[i] = src[i];
}

int grid_for(int64_t work, int per_block, int cap)
{
    int64_t g = (work + per_block - 1) / per_block;
    if (g < 1) g = 1;
    if (g > cap) g = cap;
    return (int)g;
}

constexpr int kMaxGridY = 65535;

// Variant table: (TX, NTY, RY).  Tile = TX x (NTY*RY) cells, TX*NTY threads.
#define J3D_VARIANTS(X) \
    X(64, 16, 4)        \
    X(64, 8, 8)         \
    X(64, 4, 4)         \
    X(64, 8, 4)         \
    X(128, 8, 4)        \
    X(128, 4, 8)        \
    X(128, 4, 4)        \
    X(256, 4, 4)        \
    X(32, 8, 4)         \
    X(64, 4, 8)

struct VariantEntry {
    int tx, nty, ry;
    void (*fn)(SweepArgs);
};

#define J3D_ENTRY(TX, NTY, RY) {TX, NTY, RY, sweep_kernel<TX, NTY, RY>},
const VariantEntry kVariants[] = {J3D_VARIANTS(J3D_ENTRY)};
#undef J3D_ENTRY
constexpr int kVariantCount = sizeof(kVariants) / sizeof(kVariants[0]);

}  // namespace

int variant_count() { return kVariantCount; }

VariantInfo variant_info(int v)
{
    const VariantEntry &e = kVariants[v];
    return VariantInfo{e.tx, e.nty * e.ry, e.tx * e.nty};
}

int launch_sweep(int variant, const SweepArgs &a, int grid, void *stream)
{
    if (variant < 0 || variant >= kVariantCount || grid < 1) return (int)hipErrorInvalidValue;
    const VariantEntry &e = kVariants[variant];
    hipLaunchKernelGGL(e.fn, dim3(grid), dim3(e.tx * e.nty), 0, (hipStream_t)stream, a);
    return (int)hipGetLastError();
}

int launch_init(double *base, const BlockDesc *blocks, int32_t block_begin, int32_t nblocks,
                int32_t max_cells, int32_t max_xface, int parity, const int64_t n[3], uint64_t s0,
                const double bc[6], int write_interior, void *stream)
{
    (void)max_xface;
    const dim3 grid(grid_for(max_cells, 256, 8192), nblocks < kMaxGridY ? nblocks : kMaxGridY);
    hipLaunchKernelGGL(init_kernel, grid, dim3(256), 0, (hipStream_t)stream, base, blocks,
                       block_begin, nblocks, parity, n[0], n[1], s0, bc[0], bc[1], bc[2], bc[3],
                       bc[4], bc[5], write_interior);
    return (int)hipGetLastError();
}

int launch_pack(double *base, const BlockDesc *blocks, int32_t block_begin, int32_t nblocks,
                int32_t max_face, int parity, int face_mask, void *stream)
{
    const dim3 grid(grid_for(max_face, 256, 1 << 30), nblocks < kMaxGridY ? nblocks : kMaxGridY);
    hipLaunchKernelGGL(pack_kernel, grid, dim3(256), 0, (hipStream_t)stream, base, blocks,
                       block_begin, nblocks, parity, face_mask);
    return (int)hipGetLastError();
}

int launch_exchange(double *base, const BlockDesc *blocks, int32_t block_begin, int32_t nblocks,
                    int32_t max_face, void *stream)
{
    const dim3 grid(grid_for(max_face, 256, 1 << 30), nblocks < kMaxGridY ? nblocks : kMaxGridY);
    hipLaunchKernelGGL(exchange_kernel, grid, dim3(256), 0, (hipStream_t)stream, base, blocks,
                       block_begin, nblocks);
    return (int)hipGetLastError();
}

int launch_unpack(double *base, const BlockDesc *blocks, int32_t block_begin, int32_t nblocks,
                  int32_t max_face, int parity, int face_mask, void *stream)
{
    const dim3 grid(grid_for(max_face, 256, 1 << 30), nblocks < kMaxGridY ? nblocks : kMaxGridY);
    hipLaunchKernelGGL(unpack_kernel, grid, dim3(256), 0, (hipStream_t)stream, base, blocks,
                       block_begin, nblocks, parity, face_mask);
    return (int)hipGetLastError();
}

int launch_scatter(double *base, const BlockDesc *blocks, int32_t block_base, const int32_t nb[3],
                   const int32_t *maps, const int64_t n[3], int64_t z0, int64_t z1,
                   const double *src, int parity, void *stream)
{
    const DenseMap m{maps, maps + 2 * n[0], maps + 2 * (n[0] + n[1]), nb[0], nb[1], nb[2]};
    const int64_t count = n[0] * n[1] * (z1 - z0);
    hipLaunchKernelGGL(scatter_kernel, dim3(grid_for(count, 256, 65536)), dim3(256), 0,
                       (hipStream_t)stream, base, blocks, block_base, m, n[0], n[1], z0, count,
                       src, parity);
    return (int)hipGetLastError();
}

int launch_gather(const double *base, const BlockDesc *blocks, int32_t block_base,
                  const int32_t nb[3], const int32_t *maps, const int64_t n[3], int64_t z0,
                  int64_t z1, double *dst, int parity, void *stream)
{
    const DenseMap m{maps, maps + 2 * n[0], maps + 2 * (n[0] + n[1]), nb[0], nb[1], nb[2]};
    const int64_t count = n[0] * n[1] * (z1 - z0);
    hipLaunchKernelGGL(gather_kernel, dim3(grid_for(count, 256, 65536)), dim3(256), 0,
                       (hipStream_t)stream, base, blocks, block_base, m, n[0], n[1], z0, count,
                       dst, parity);
    return (int)hipGetLastError();
}

int launch_set_face(double *base, const BlockDesc *blocks, int32_t block_base, const int32_t nb[3],
                    const int32_t *maps, const int64_t n[3], int face, const double *src,
                    void *stream)
{
    const DenseMap m{maps, maps + 2 * n[0], maps + 2 * (n[0] + n[1]), nb[0], nb[1], nb[2]};
    const int axis = face / 2;
    const int64_t count = axis == 0 ? n[1] * n[2] : (axis == 1 ? n[0] * n[2] : n[0] * n[1]);
    hipLaunchKernelGGL(set_face_kernel, dim3(grid_for(count, 256, 65536)), dim3(256), 0,
                       (hipStream_t)stream, base, blocks, block_base, m, n[0], n[1], n[2], face,
                       src);
    return (int)hipGetLastError();
}

int launch_gather_block(const double *base, const BlockDesc *blocks, int32_t block, int parity,
                        double *dst, void *stream)
{
    hipLaunchKernelGGL(gather_block_kernel, dim3(4096), dim3(256), 0, (hipStream_t)stream, base,
                       blocks, block, parity, dst);
    return (int)hipGetLastError();
}

int launch_fill_u64(unsigned long long *p, int64_t count, unsigned long long value, void *stream)
{
    hipLaunchKernelGGL(fill_u64_kernel, dim3(grid_for(count, 256, 4096)), dim3(256), 0,
                       (hipStream_t)stream, p, count, value);
    return (int)hipGetLastError();
}

int launch_fill_u32(unsigned int *p, int64_t count, unsigned int value, void *stream)
{
    hipLaunchKernelGGL(fill_u32_kernel, dim3(grid_for(count, 256, 4096)), dim3(256), 0,
                       (hipStream_t)stream, p, count, value);
    return (int)hipGetLastError();
}

int launch_copy(void *dst, const void *src, uint64_t bytes, void *stream)
{
    const int64_t n16 = (int64_t)(bytes / 16);
    hipLaunchKernelGGL(copy_kernel, dim3(grid_for(n16, 256, 256 * 64)), dim3(256), 0,
                       (hipStream_t)stream, (uint4 *)dst, (const uint4 *)src, n16);
    return (int)hipGetLastError();
}

}  // namespace j3d
