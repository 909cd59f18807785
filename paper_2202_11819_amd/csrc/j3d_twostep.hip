// j3d_twostep.hip -- two Jacobi sweeps per launch on an undivided grid.
//
// Temporal blocking along the marching axis: a workgroup owns an x-y tile of
// the grid and walks up z.  For each plane it first computes the intermediate
// iterate v = u^{t+1} over the tile and a one-cell ring around it, from u^t
// over the tile and a two-cell ring, and then the result w = u^{t+2} over the
// tile, one plane behind.  u^t is read from HBM once and u^{t+2} written
// once, so a cell update costs 8 bytes of HBM traffic instead of 16; the
// intermediate iterate lives only in LDS.  Each value of v and w is the
// 7-term sum of the same operands in the same order as a single sweep
// (centre, x-, x+, y-, y+, z-, z+, each addition rounded, then one
// multiplication by fl(1/7); built with -ffp-contract=off), so the result is
// bit-identical to two separate sweeps.
//
// Only a grid of one block is handled here: every halo value is then a
// Dirichlet value held in the block's own ghost rows, ghost planes and x-halo
// arrays, which never change.  Ring cells of v that lie on the boundary
// layer keep their Dirichlet value.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "j3d_internal.hpp"

namespace j3d {
namespace {

constexpr double kW2 = 1.0 / 7.0;  // fl(1/7)
constexpr int kXcds2 = 8;          // XCDs per MI355X

constexpr int NB = 3;   // planes of u held in registers per lane

// Tile shapes: TX x TY cells of w, NT threads.  u^t covers the tile with a
// two-cell ring, v the tile with a one-cell ring; each LDS plane ends in one
// sink cell that takes the writes of lanes past the region.
template <int TX_, int TY_, int NT_>
struct Shape {
    static constexpr int TX = TX_, TY = TY_, NT = NT_;
    static constexpr int UX = TX + 4, UY = TY + 4, UP = UX * UY;
    static constexpr int VX = TX + 2, VY = TY + 2, VP = VX * VY;
    static constexpr int US = (UP + NT - 1) / NT;  // u cells per thread and plane
    static constexpr int VS = (VP + NT - 1) / NT;  // v cells per thread and plane
    static constexpr int WS = TX * TY / NT;        // w cells per thread and plane
    static constexpr int USLOT = UP + 2, VSLOT = VP + 2;
    static_assert(TX * TY % NT == 0, "whole w rows per thread");
    static_assert(US == 3 && VS == 3 && WS == 2, "slot counts assumed below");
    static_assert((USLOT + VSLOT) * 4 * 8 <= 160 * 1024 - 1024, "LDS of one workgroup");
};

// LDS-only barrier (the loop hands data between waves through LDS alone, so
// outstanding global loads of later planes need not complete).
__device__ __forceinline__ void lds_barrier2()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

__device__ __forceinline__ int xcd_remap2(int i, int n)
{
    const int q = n / kXcds2, r = n % kXcds2;
    const int x = i % kXcds2, j = i / kXcds2;
    return x * q + min(x, r) + j;
}

}  // namespace

template <class S>
__global__ __launch_bounds__(S::NT) void twostep_kernel(TwoStepArgs a)
{
    constexpr int TX = S::TX, TY = S::TY, NT = S::NT, UX = S::UX, UP = S::UP, VX = S::VX, VP = S::VP;
    constexpr int US = S::US, VS = S::VS, WS = S::WS, USLOT = S::USLOT, VSLOT = S::VSLOT;
    __shared__ double Us[4 * USLOT];
    __shared__ double Vs[4 * VSLOT];
    __shared__ double red[NT / 64];

    const int tid = threadIdx.x;
    const int t = xcd_remap2(blockIdx.x, gridDim.x);
    // Tile geometry and buffers: the launch's single grid, or (multi-problem
    // launch) the tile's block and problem from the tables.
    const double *cur, *xh;
    double *nxt;
    unsigned long long *resp;
    int ex, ey, ez, pitch, tx, ty, tz, nty, ntz;
    bool want_res;
    if (a.blocks) {
        const Tile tl = a.tiles[a.tile_begin + t];
        const BlockDesc *__restrict__ B = a.blocks + tl.block;
        const ProbDesc *__restrict__ P = a.probs + B->prob;
        if (a.step >= P->limit) return;  // uniform over the workgroup: no barrier reached
        const int p = (int)((P->base + a.step) & 1);
        ex = B->ext[0];
        ey = B->ext[1];
        ez = B->ext[2];
        pitch = B->pitch;
        cur = a.base + B->off[p];
        nxt = a.base + B->off[p ^ 1];
        xh = a.base + B->xoff[p];
        resp = a.res + P->res_slot;
        want_res = a.step + 1 == P->limit;
        tx = tl.tx;
        ty = tl.ty;
        tz = tl.tz;
        nty = (ey + TY - 1) / TY;
        ntz = (ez + a.zchunk - 1) / a.zchunk;
    } else {
        ex = a.ex;
        ey = a.ey;
        ez = a.ez;
        pitch = a.pitch;
        cur = a.cur;
        nxt = a.nxt;
        xh = a.xh;
        resp = a.res;
        want_res = a.want_res != 0;
        tx = t % a.ntx;
        ty = (t / a.ntx) % a.nty;
        tz = t / (a.ntx * a.nty);
        nty = a.nty;
        ntz = a.ntz;
    }
    const int x0 = tx * TX, nxv = min(TX, ex - x0);
    const int y0 = (int)((int64_t)ty * ey / nty), nyv = (int)((int64_t)(ty + 1) * ey / nty) - y0;
    const int z0 = (int)((int64_t)tz * ez / ntz), nzv = (int)((int64_t)(tz + 1) * ez / ntz) - z0;
    const int64_t ps = plane_stride(pitch, ey);  // plane stride of the field, doubles

    // u^t sources.  Cell (gx, gy) of the tile's two-cell ring, plane z:
    //   inside the grid in x and y: the field, planes -1 .. ez (the ghost
    //   planes hold the z faces);
    //   one row outside in y: the field's ghost row, planes 0 .. ez-1;
    //   one column outside in x: the x-halo array, planes 0 .. ez-1;
    //   anything else is never an operand of a needed value and reads as 0.
    const double *ub[US];
    int64_t ust[US];
    int uzl[US], uzh[US];
#pragma unroll
    for (int r = 0; r < US; ++r) {
        const int i = tid + r * NT;
        const int lx = i % UX, ly = i / UX;
        const int gx = x0 - 2 + lx, gy = y0 - 2 + ly;
        const bool in_tile = i < UP && lx < nxv + 4 && ly < nyv + 4;
        const bool inx = gx >= 0 && gx < ex, iny = gy >= 0 && gy < ey;
        ub[r] = cur;
        ust[r] = 0;
        uzl[r] = 1;
        uzh[r] = 0;  // empty range: no load
        if (in_tile) {
            if (inx && (iny || gy == -1 || gy == ey)) {
                ub[r] = cur + ps + (int64_t)(gy + 1) * pitch + gx;
                ust[r] = ps;
                uzl[r] = iny ? -1 : 0;
                uzh[r] = iny ? ez : ez - 1;
            } else if (iny && (gx == -1 || gx == ex)) {
                ub[r] = xh + (gx < 0 ? 0 : (int64_t)ey * ez) + gy;
                ust[r] = ey;
                uzl[r] = 0;
                uzh[r] = ez - 1;
            }
        }
    }
    // Plain (temporal) loads: the ring cells of a tile are the edge cells of
    // its neighbours, which run at about the same planes; a non-temporal hint
    // evicts those lines before the neighbour reads them (measured 1.53x
    // instead of 1.15x the algorithmic read bytes, 517 instead of 598 GLUP/s).
    auto load_plane = [&](int z, double (&dst)[US]) __attribute__((always_inline)) {
#pragma unroll
        for (int r = 0; r < US; ++r) {
            const bool ok = z >= uzl[r] && z <= uzh[r];
            const double *p = ok ? ub[r] + (int64_t)z * ust[r] : cur;
            const double v = *p;
            dst[r] = ok ? v : 0.0;
        }
    };

    // v cells: (vx, vy) of the one-cell ring region.  kind 1: inside the grid
    // in x and y (computed inside the z range, Dirichlet on the z faces);
    // kind 2: on an x or y face of the boundary layer (keeps its Dirichlet
    // value inside the z range); kind 0: not needed.
    int vc[VS], vkind[VS];
#pragma unroll
    for (int r = 0; r < VS; ++r) {
        const int i = tid + r * NT;
        const int vx = i % VX, vy = i / VX;
        const bool in_tile = i < VP && vx < nxv + 2 && vy < nyv + 2;
        const int gx = x0 - 1 + vx, gy = y0 - 1 + vy;
        const bool inx = gx >= 0 && gx < ex, iny = gy >= 0 && gy < ey;
        vc[r] = in_tile ? (vy + 1) * UX + vx + 1 : UX + 1;
        vkind[r] = !in_tile ? 0 : (inx && iny) ? 1 : ((inx && (gy == -1 || gy == ey)) ||
                                                     (iny && (gx == -1 || gx == ex))) ? 2 : 0;
    }

    // w cells: the tile; wc is the cell's index in the v region.
    int wc[WS];
    bool wok[WS];
    int64_t wo[WS];
#pragma unroll
    for (int r = 0; r < WS; ++r) {
        const int i = tid + r * NT;
        const int wx = i % TX, wy = i / TX;
        wok[r] = wx < nxv && wy < nyv;
        wc[r] = (wy + 1) * VX + wx + 1;
        wo[r] = (int64_t)(y0 + wy + 1) * pitch + x0 + wx;
    }

    // Step j writes u plane z0-2+j into LDS, computes v on plane z0-3+j and
    // w on plane z0-5+j (whose v operands were all written before this step's
    // barrier).  Four LDS slots per iterate keep every slot's last reader a
    // barrier ahead of its next writer.
    const int nsteps = nzv + 5;
    double R[NB][US];
#pragma unroll
    for (int k = 0; k < NB; ++k) load_plane(z0 - 2 + k, R[k]);
    double rmax = 0.0;

    auto step = [&](const int j, double (&Rk)[US]) __attribute__((always_inline)) {
        double *Uw = Us + (j & 3) * USLOT;
        if (j < nzv + 4) {
#pragma unroll
            for (int r = 0; r < US; ++r) Uw[min(tid + r * NT, UP)] = Rk[r];
        }
        load_plane(z0 - 2 + j + NB, Rk);
        lds_barrier2();
        const int zv = z0 - 3 + j;
        if (j >= 2 && j <= nzv + 3) {
            const double *Uc = Us + ((j - 1) & 3) * USLOT;
            const double *Um = Us + ((j - 2) & 3) * USLOT;
            const double *Up = Uw;
            double *Vw = Vs + (j & 3) * VSLOT;
            const bool inz = zv >= 0 && zv < ez;
            const bool zface = zv == -1 || zv == ez;
#pragma unroll
            for (int r = 0; r < VS; ++r) {
                const int c = vc[r];
                double s = Uc[c];
                s += Uc[c - 1];
                s += Uc[c + 1];
                s += Uc[c - UX];
                s += Uc[c + UX];
                s += Um[c];
                s += Up[c];
                const double keep = Uc[c];
                const double v = (vkind[r] == 1 && inz) ? s * kW2
                                 : ((vkind[r] == 1 && zface) || (vkind[r] == 2 && inz)) ? keep : 0.0;
                Vw[min(tid + r * NT, VP)] = v;
            }
        }
        if (j >= 5) {
            const int zw = z0 - 5 + j;
            const double *Vc = Vs + ((j - 2) & 3) * VSLOT;
            const double *Vm = Vs + ((j - 3) & 3) * VSLOT;
            const double *Vp = Vs + ((j - 1) & 3) * VSLOT;
            double *outp = nxt + (int64_t)(zw + 1) * ps;
#pragma unroll
            for (int r = 0; r < WS; ++r) {
                const int vi = wc[r];
                double s = Vc[vi];
                s += Vc[vi - 1];
                s += Vc[vi + 1];
                s += Vc[vi - VX];
                s += Vc[vi + VX];
                s += Vm[vi];
                s += Vp[vi];
                const double w = s * kW2;
                if (wok[r]) __builtin_nontemporal_store(w, outp + wo[r]);
                if (want_res && wok[r]) {
                    const double d = fabs(w - Vc[vi]);
                    rmax = d > rmax ? d : rmax;
                }
            }
        }
    };

    for (int jb = 0; jb < nsteps; jb += NB) {
        step(jb, R[0]);
        if (jb + 1 < nsteps) step(jb + 1, R[1]);
        if (jb + 2 < nsteps) step(jb + 2, R[2]);
    }

    if (want_res) {
        double m = rmax;
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) {
            const double q = __shfl_xor(m, o);
            m = q > m ? q : m;
        }
        if ((tid & 63) == 0) red[tid >> 6] = m;
        __syncthreads();
        if (tid == 0) {
            double w = 0.0;
            for (int i = 0; i < NT / 64; ++i) w = red[i] > w ? red[i] : w;
            __hip_atomic_fetch_max(resp, (unsigned long long)__double_as_longlong(w), __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_AGENT);
        }
    }
}

// 64 x 16 tiles of 512 threads: two workgroups share a compute unit.  Measured
// alternatives: a 64 x 32 tile of 1024 threads, alone on its compute unit, 20%
// slower; a 32 x 32 tile of 512 threads 5-7% slower on 512^3 and 1024^3 grids
// (1% faster on the batched mix of small problems).
using Tile16 = Shape<64, 16, 512>;

int twostep_tiles(int ex, int ey, int ez, int zchunk, int *ntx, int *nty, int *ntz)
{
    *ntx = (ex + Tile16::TX - 1) / Tile16::TX;
    *nty = (ey + Tile16::TY - 1) / Tile16::TY;
    const int zc = zchunk > 0 && zchunk < ez ? zchunk : ez;
    *ntz = (ez + zc - 1) / zc;
    return *ntx * *nty * *ntz;
}

void twostep_make_tiles(const BlockDesc *blocks, int32_t b0, int32_t b1, int zchunk, std::vector<Tile> *tiles)
{
    for (int32_t b = b0; b < b1; ++b) {
        int ntx = 0, nty = 0, ntz = 0;
        twostep_tiles(blocks[b].ext[0], blocks[b].ext[1], blocks[b].ext[2], zchunk, &ntx, &nty, &ntz);
        for (int tz = 0; tz < ntz; ++tz)
            for (int ty = 0; ty < nty; ++ty)
                for (int tx = 0; tx < ntx; ++tx) {
                    Tile t{};  // the two-sweep kernel cuts its own rectangle from tx, ty, tz
                    t.block = b;
                    t.tx = tx;
                    t.ty = ty;
                    t.tz = tz;
                    tiles->push_back(t);
                }
    }
}

int launch_twostep(const TwoStepArgs &a, void *stream)
{
    const int grid = a.blocks ? a.tile_count : a.ntx * a.nty * a.ntz;
    hipLaunchKernelGGL(twostep_kernel<Tile16>, dim3(grid), dim3(Tile16::NT), 0, static_cast<hipStream_t>(stream),
                       a);
    return (int)hipGetLastError();
}

}  // namespace j3d
