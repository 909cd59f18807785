// j3d_kernels.hip -- gfx950 kernels of the Jacobi3D hot path and their launchers.
//
// The sweep (Jacobi update, fused with the halo hand-off of kernel-fusion
// strategy C, Sec. III-D-1) is the only kernel that runs per iteration in the
// fused and graph modes.  It is bound by HBM bandwidth (7 flops per 16 bytes),
// so it is built for streaming: a workgroup owns an x-y tile of one block and
// marches along z; every cell is read from HBM once (x-contiguous rows, whole
// 64-lane waves per row segment) and written once; the four in-plane
// neighbours come from a double-buffered LDS copy of the current plane with a
// one-cell ring, the two z-neighbours from registers.  In the fused sweep the
// y and z halos are read straight from the neighbour blocks' current iterate
// (pack, exchange and unpack become one read across the block boundary), and
// a block's x faces, which a neighbour could only read one double per row,
// are handed to the neighbour's x-halo array of the next iterate as two
// coalesced stores per plane.  The other kernels here are the unfused pack /
// exchange / unpack of Fig. 1 and Fig. 3, the seeded initialisation, and
// dense <-> block copies.
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
constexpr int kXcds = kXcdCount;

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

// Barrier that orders LDS only.  __syncthreads() is a workgroup release /
// acquire over all address spaces, which makes every wave wait for its
// outstanding global loads and stores (including the prefetch of the next
// plane) before the barrier; the sweep exchanges data between waves through
// LDS only, so only LDS operations need to complete.
__device__ __forceinline__ void lds_barrier()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// ---- the sweep ----------------------------------------------------------------
//
// Addressing: every global access is a uniform (scalar) 64-bit base pointer
// for the current plane plus a 32-bit per-lane byte offset inside that plane,
// so the hardware's scalar-base + vector-offset form is used and each thread
// keeps one offset per row instead of one 64-bit address per row and plane.

#ifndef J3D_NT_LOAD
#define J3D_NT_LOAD 1   // interior cells are read once per sweep: stream them
#endif
#ifndef J3D_NT_STORE
#define J3D_NT_STORE 1  // the next iterate is not read again within the sweep
#endif

// Raw buffer accesses: a 128-bit resource (base, byte range) in scalar
// registers plus a 32-bit per-lane byte offset.  Every streaming access of the
// sweep goes through a resource that spans exactly one plane (or one halo
// row), so an offset outside it reads 0 and drops the store instead of
// touching other memory.
typedef int i32x2 __attribute__((ext_vector_type(2)));
constexpr int kRsrcWord3 = 0x00020000;  // gfx9-family raw buffer, 32-bit elements
constexpr int kAuxNT = 2;               // non-temporal (streaming) cache policy
constexpr int kAuxLoad = J3D_NT_LOAD ? kAuxNT : 0;
constexpr int kAuxStore = J3D_NT_STORE ? kAuxNT : 0;

__device__ __forceinline__ __amdgpu_buffer_rsrc_t rsrc(const void *p, uint64_t bytes)
{
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(p), 0,
                                             (int)(bytes > 0x7fffffffull ? 0x7fffffffull : bytes),
                                             kRsrcWord3);
}

// A resource of at most 2 GiB - 1 (a plane or a face row): no clamp needed.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t rsrc32(const void *p, uint32_t bytes)
{
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(p), 0, (int)bytes, kRsrcWord3);
}

template <int AUX>
__device__ __forceinline__ double bload(__amdgpu_buffer_rsrc_t r, uint32_t off)
{
    return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, (int)off, 0, AUX));
}

template <int AUX>
__device__ __forceinline__ void bstore(__amdgpu_buffer_rsrc_t r, uint32_t off, double v)
{
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(i32x2, v), r, (int)off, 0, AUX);
}

// ---- tile layouts ------------------------------------------------------------
//
// A tile is a rectangle of one block's x-y plane (x0.., y0.., nxv x nyv cells)
// streamed over a range of planes.  A layout decides which cell of the
// rectangle each thread owns in each of its RY rows, and which cell of the
// rectangle's one-cell halo ring it loads.  The LDS holds the current plane
// of the rectangle with its ring: row length lx = width + 2.

// Occupancy.  More streams per compute unit were measured slower: two
// 512-thread workgroups per CU (4 waves per SIMD) sweep 3-15% slower than one,
// the HBM sees more concurrent, scattered streams for the same bytes.  So a
// workgroup of 512 threads or more reserves enough LDS to be alone on its CU,
// and a 256-thread one to share it with at most one other.  The reservation
// is the tail of the plane buffer, never touched.
constexpr int kLdsPerCu = 160 * 1024;
constexpr int smem_doubles(int nt, int used_doubles)
{
    const int cap = nt >= 512 ? 1 : 2;                    // workgroups per CU
    const int need = (kLdsPerCu / (cap + 1) + 1024) / 8;  // more than 1/(cap+1) of the LDS
    return used_doubles > need ? used_doubles : need;
}

// Fixed tiles: TX x TY, thread (tx, ty) owns column tx of rows ty + NTY*r.
// x tiles start on multiples of TX; the last one in a row may be ragged.
template <int TX, int NTY, int RY_, int PF_>
struct Tiled {
    static constexpr int NT = TX * NTY, RY = RY_, PF = PF_;
    static constexpr int TY = NTY * RY;
    static constexpr int LXC = TX + 2;
    static constexpr int SINK = LXC * (TY + 2);    // masked lanes write after the plane
    static constexpr int PLANE = SINK + 64;
    static constexpr int XROWS = TY;               // rows of a tile, at most
    static constexpr int SMEM = smem_doubles(NT, 2 * PLANE);
    static_assert(NT >= 2 * TX + 2 * TY, "every halo cell of a plane needs a loader thread");
    static_assert(NT % 64 == 0, "whole waves");
    static_assert(PF >= 1 && PF <= 4, "prefetch depth");
    __device__ static int lx(int) { return LXC; }
    __device__ static bool full(int nxv, int nyv) { return nxv == TX && nyv == TY; }
    template <bool FULL>
    __device__ static bool cell(int tid, int r, int nxv, int nyv, int, int &cx, int &cy)
    {
        cx = tid % TX;
        cy = tid / TX + NTY * r;
        return FULL || (cx < nxv && cy < nyv);
    }
    // ring cell of this thread: kind 0/1 = y-/y+ row (c = column), 2/3 = x-/x+ column (c = row)
    __device__ static bool ring(int tid, int nxv, int nyv, int &kind, int &c)
    {
        if (tid < 2 * TX) {
            kind = tid / TX;
            c = tid % TX;
            return c < nxv;
        }
        const int u = tid - 2 * TX;
        kind = 2 + u / TY;
        c = u % TY;
        return u < 2 * TY && c < nyv;
    }
};

// Flattened tiles: the rectangle's cells, numbered x fastest, are dealt to
// the threads in order (slot f goes to thread f % NT, row f / NT); the
// rectangle is sized per block by flat_shape, so only the lanes of the last
// partial wave idle.  With whole rows (the usual case) a plane of the tile is
// one contiguous run of memory and every wave reads 64 consecutive doubles.
template <int NT_, int RY_, int PF_>
struct Flat {
    static constexpr int NT = NT_, RY = RY_, PF = PF_;
    static constexpr int CAP = NT * RY;
    // (nxv+2)(nyv+2) <= nxv*nyv + 2(nxv+nyv) + 4 <= CAP + NT + 4
    static constexpr int SINK = CAP + NT + 4;
    static constexpr int PLANE = SINK + 64;
    static constexpr int XROWS = NT / 2;
    static constexpr int SMEM = smem_doubles(NT, 2 * PLANE);
    static_assert(NT % 64 == 0 && NT >= 256, "whole waves, room for a halo ring");
    static_assert(PF >= 1 && PF <= 4, "prefetch depth");
    __device__ static int lx(int nxv) { return nxv + 2; }
    // every slot of every thread holds a cell (no idle tail, no shift)
    __device__ static bool full(int nxv, int nyv) { return nxv * nyv == CAP; }
    // shift: slots before the tile's first cell (aligns waves to lines)
    template <bool FULL>
    __device__ static bool cell(int tid, int r, int nxv, int nyv, int shift, int &cx, int &cy)
    {
        const int f = tid + r * NT - shift;
        const int q = f / nxv, x = f - q * nxv;
        const bool v = FULL || (f >= 0 && q < nyv);
        cy = v ? q : 0;
        cx = v ? x : 0;
        return v;
    }
    __device__ static bool ring(int tid, int nxv, int nyv, int &kind, int &c)
    {
        int h = tid;
        kind = 0;
        if (h >= nxv) { h -= nxv; kind = 1; }
        if (kind == 1 && h >= nxv) { h -= nxv; kind = 2; }
        if (kind == 2 && h >= nyv) { h -= nyv; kind = 3; }
        c = h;
        return kind < 3 || h < nyv;
    }
};

// Uniform description of one tile (lives in scalar registers).
struct TileGeo {
    const char *cur;   // input field, byte address of plane index 0 (the z- ghost plane)
    char *nxt;         // output field
    const char *zlo;   // plane read as z = -1: the own ghost plane, or in the fused
    const char *zhi;   // sweep the z neighbour's nearest interior plane; likewise z = ez
    char *dxm, *dxp;   // x-halo arrays (plane index 0) that take this block's x- / x+ face
    uint32_t xrm, xrp; // bytes of one plane of those arrays (0: no neighbour, nothing stored)
    uint64_t psb;      // plane stride of this block's field, bytes
    int ex, ey, ez, pitch;  // pitch: row stride in doubles (>= ex)
    int x0, y0, z0, nxv, nyv, nzv;
    int shift;         // flattened tiles of whole rows: slots before the first cell
    bool want_res;
};

template <class K, bool FULL, bool RES>
__device__ __forceinline__ double sweep_planes(const TileGeo &g, const double *__restrict__ hsrc0,
                                               uint64_t hstep, int hl, double *sm, double *xf)
{
    constexpr int RY = K::RY;
    // Register ring of NB planes: while plane k is computed from planes
    // k-1, k, k+1, the loads of planes k+2 .. k+1+PF are in flight.  The loop
    // is unrolled NB times so every ring index is a compile-time constant and
    // a load lands in its register without any copy; the slot of plane k-1 is
    // refilled with plane k+PF+2 right after its last use.
    //
    // Every global load and store of a step is issued by every lane, without
    // branches (lanes with nothing to do address outside the resource), and
    // the steady-state loop is entered only after one peeled round: the
    // compiler's memory-counter waits then see the same instruction stream on
    // every path and wait only for the plane that is about to be used, never
    // for the stores of the previous step.
    constexpr int NB = K::PF + 3;
    const int tid = threadIdx.x;
    const int lx = K::lx(g.nxv);
    const uint32_t rowb = (uint32_t)g.pitch * 8u;
    // Lanes without a cell stay in lock-step with the others: their buffer
    // offset lies outside every resource, so their loads return 0 and their
    // stores are dropped; their LDS writes go to a sink after the plane and
    // their LDS reads to a valid cell.
    constexpr uint32_t kOutside = 0x80000000u;
    bool vr[RY];
    uint32_t off[RY];  // byte offset of this thread's cell of row r inside a plane
    int lw[RY];        // LDS slot this thread writes for row r
    int li[RY];        // LDS slot of the cell (its four in-plane neighbours are +-1, +-lx)
    int ly[RY];        // row of the cell inside the tile
    bool fxm[RY], fxp[RY];  // cell on the block's x- / x+ face with a neighbour there (fused)
#pragma unroll
    for (int r = 0; r < RY; ++r) {
        int cx, cy;
        vr[r] = K::template cell<FULL>(tid, r, g.nxv, g.nyv, g.shift, cx, cy);
        off[r] = vr[r] ? (uint32_t)(g.y0 + cy + 1) * rowb + (uint32_t)(g.x0 + cx) * 8u : kOutside;
        li[r] = vr[r] ? (cy + 1) * lx + cx + 1 : lx + 1;
        lw[r] = vr[r] ? li[r] : K::SINK + (tid & 63);
        ly[r] = cy;
        fxm[r] = vr[r] && g.xrm != 0 && g.x0 + cx == 0;
        fxp[r] = vr[r] && g.xrp != 0 && g.x0 + cx == g.ex - 1;
    }
    // x faces (fused sweep): a cell of the block's first / last column puts its
    // new value into xf; after the next barrier the first 2*nyv threads store
    // one face cell each, so a plane's face goes out as two coalesced stores.
    const int xs = tid < g.nyv ? tid : (tid < 2 * g.nyv ? K::XROWS + tid - g.nyv : 0);
    uint32_t xom = kOutside, xop = kOutside;
    if (tid < g.nyv) {
        if (g.x0 == 0) xom = (uint32_t)(g.y0 + tid) * 8u;
    } else if (tid < 2 * g.nyv) {
        if (g.x0 + g.nxv == g.ex) xop = (uint32_t)(g.y0 + tid - g.nyv) * 8u;
    }
    const uint64_t psb = g.psb;
    const uint32_t psz = (uint32_t)psb;  // a plane is far below 2 GiB (checked by the planner)
    const int zend = g.z0 + g.nzv;  // last plane read: the z+ neighbour of the last one computed
    auto plane = [&](int z) -> const char * {
        return z < 0 ? g.zlo : (z >= g.ez ? g.zhi : g.cur + (uint64_t)(z + 1) * psb);
    };

    double R[NB][RY];
    double H[NB];
    // slot of interior plane z is (z - z0 + 1) mod NB
#pragma unroll
    for (int j = 0; j < NB; ++j) {
        const int z = g.z0 - 1 + j;
        const bool live = z <= zend;
        const __amdgpu_buffer_rsrc_t rz = rsrc32(plane(live ? z : zend), live ? psz : 0u);
#pragma unroll
        for (int r = 0; r < RY; ++r) R[j][r] = bload<kAuxLoad>(rz, off[r]);
        const int zh = z < g.z0 ? g.z0 : (z < zend ? z : zend - 1);
        H[j] = hsrc0[(uint64_t)zh * hstep];
    }
    double rmax = 0.0;

    // Addresses that move by one plane per step, kept as running values (the
    // step is short of scalar issue slots when every wave recomputes them).
    char *op = g.nxt + (uint64_t)(g.z0 + 1) * psb;        // output plane z0+kk
    int zn = g.z0 - 1 + NB;                                // plane refilled by step kk
    const char *lp = g.cur + (uint64_t)(zn + 1) * psb;    // ... its address inside the field
    const double *hp = hsrc0 + (uint64_t)(zn < zend ? zn : zend - 1) * hstep;  // its halo value
    const uint64_t xstep = (uint64_t)g.ey * 8u;
    uint64_t xo = (uint64_t)(int64_t)(g.z0 - 1) * xstep;  // x-face plane z0+kk-1 (unused at kk = 0)

    auto step = [&](const int kk, const int j) __attribute__((always_inline)) {
        const int jm = j, jc = (j + 1) % NB, jp = (j + 2) % NB;
        double *L = sm + (kk & 1) * K::PLANE;
#pragma unroll
        for (int r = 0; r < RY; ++r) L[lw[r]] = R[jc][r];
        if (hl >= 0) L[hl] = H[jc];
        lds_barrier();
        {   // x faces of plane k-1 (none before the first step)
            const bool any = kk > 0;
            const double xv = xf[((kk + 1) & 1) * 2 * K::XROWS + xs];
            bstore<0>(rsrc32(g.dxm + xo, any ? g.xrm : 0u), xom, xv);
            bstore<0>(rsrc32(g.dxp + xo, any ? g.xrp : 0u), xop, xv);
        }

        const __amdgpu_buffer_rsrc_t ro = rsrc32(op, psz);
        double *XF = xf + (kk & 1) * 2 * K::XROWS;
#pragma unroll
        for (int r = 0; r < RY; ++r) {
            const int c = li[r];
            double s = R[jc][r];
            s += L[c - 1];
            s += L[c + 1];
            s += L[c - lx];
            s += L[c + lx];
            s += R[jm][r];
            s += R[jp][r];
            const double v = s * kW;
            bstore<kAuxStore>(ro, off[r], v);
            if (fxm[r]) XF[ly[r]] = v;
            if (fxp[r]) XF[K::XROWS + ly[r]] = v;
            if (RES) {
                const double d = vr[r] ? fabs(v - R[jc][r]) : 0.0;
                rmax = d > rmax ? d : rmax;
            }
        }
        // refill the slot of plane k-1 with plane k-1+NB; past the tile's
        // last plane the resource is empty (loads return 0)
        {
            const bool live = zn <= zend;
            const __amdgpu_buffer_rsrc_t rn = rsrc32(zn < g.ez ? lp : g.zhi, live ? psz : 0u);
#pragma unroll
            for (int r = 0; r < RY; ++r) R[jm][r] = bload<kAuxLoad>(rn, off[r]);
            H[jm] = *hp;
        }
        op += psb;
        lp += psb;
        ++zn;
        hp += zn < zend ? hstep : 0;
        xo += xstep;
    };
    int kk = 0;
    if (g.nzv >= NB) {
        // one peeled round, then the steady state
#pragma unroll
        for (int j = 0; j < NB; ++j) step(j, j);
        for (kk = NB; kk + NB <= g.nzv; kk += NB) {
#pragma unroll
            for (int j = 0; j < NB; ++j) step(kk + j, j);
        }
    }
#pragma unroll
    for (int j = 0; j < NB - 1; ++j)
        if (kk + j < g.nzv) step(kk + j, j);
    lds_barrier();
    {   // x faces of the last plane
        const double xv = xf[((g.nzv - 1) & 1) * 2 * K::XROWS + xs];
        const uint64_t fo = (uint64_t)(zend - 1) * xstep;
        bstore<0>(rsrc32(g.dxm + fo, g.xrm), xom, xv);
        bstore<0>(rsrc32(g.dxp + fo, g.xrp), xop, xv);
    }
    return rmax;
}

template <class K>
__device__ __forceinline__ void sweep_tile(const SweepArgs &a, const Tile tl, double *sm, double *red,
                                           double *xf)
{
    // The descriptor tables are read-only while kernels run: reading them
    // through the constant address space keeps every field a scalar load,
    // whatever the compiler can prove about the pointers (a vector load would
    // queue behind the planes' streams).
    typedef const __attribute__((address_space(4))) BlockDesc KBlockDesc;
    typedef const __attribute__((address_space(4))) ProbDesc KProbDesc;
    KBlockDesc *B = (KBlockDesc *)(a.blocks + tl.block);
    KProbDesc *P = (KProbDesc *)(a.probs + B->prob);

    TileGeo g;
    int p;
    if (a.flags & SW_MULTI) {
        const int64_t t = P->base + a.step;
        if (t >= P->limit) return;  // uniform over the workgroup
        p = (int)(t & 1);
        const int64_t t1 = t + 1;
        g.want_res = ((P->flags & PF_RES_LAST) && t1 == P->limit) ||
                     (P->check_every > 0 && t1 % P->check_every == 0);
    } else {
        p = a.parity;
        g.want_res = (a.flags & SW_RES) != 0;
    }
    const bool fused = (a.flags & SW_FUSED) != 0;
    g.ex = B->ext[0];
    g.ey = B->ext[1];
    g.ez = B->ext[2];
    g.pitch = B->pitch;
    const int ex = g.ex, ey = g.ey, ez = g.ez, pitch = g.pitch;
    g.psb = (uint64_t)plane_stride(pitch, ey) * 8u;
    char *base = reinterpret_cast<char *>(a.base);
    g.cur = base + B->off[p] * 8;
    g.nxt = base + B->off[p ^ 1] * 8;
    // the tile's cells, as the host cut them (flat_shape / fixed columns,
    // near-equal pieces along y and z)
    g.x0 = tl.x0;
    g.nxv = tl.nxv;
    g.y0 = tl.y0;
    g.nyv = tl.nyv;
    g.z0 = tl.z0;
    g.nzv = tl.nzv;
    if (a.flags & SW_INNER) {
        // Fig. 1's interior update: the cells that read no halo, i.e. the tile
        // clipped to [1, e-1) along every axis (uniform over the workgroup)
        const int x1 = min(g.x0 + g.nxv, ex - 1), y1 = min(g.y0 + g.nyv, ey - 1), z1 = min(g.z0 + g.nzv, ez - 1);
        g.x0 = max(g.x0, 1);
        g.y0 = max(g.y0, 1);
        g.z0 = max(g.z0, 1);
        g.nxv = x1 - g.x0;
        g.nyv = y1 - g.y0;
        g.nzv = z1 - g.z0;
        if (g.nxv <= 0 || g.nyv <= 0 || g.nzv <= 0) return;
    }

    // Halo sources.  The unfused sweep reads the block's own ghost layer,
    // which the unpack step has filled.  The fused sweep reads the y and z
    // halos straight from the neighbours' current iterate (their rows / planes
    // next to the shared face: the exchange is a read across the block
    // boundary, nothing is copied), and hands its x faces, which would be
    // strided reads for the neighbour, to the neighbours' x-halo arrays of the
    // next iterate.  Global-boundary faces always come from the own ghost
    // layer, which holds the Dirichlet values.
    g.zlo = g.cur;
    g.zhi = g.cur + (uint64_t)(ez + 1) * g.psb;
    g.dxm = g.dxp = g.nxt;
    g.xrm = g.xrp = 0;
    const uint64_t ps = (uint64_t)plane_stride(pitch, ey);  // plane stride, doubles
    const double *curd = a.base + B->off[p];
    const double *ym_src = curd + ps + (uint64_t)g.y0 * pitch;                 // row y0-1, plane 0
    const double *yp_src = curd + ps + (uint64_t)(g.y0 + g.nyv + 1) * pitch;  // row y0+nyv, plane 0
    uint64_t ym_step = ps, yp_step = ps;
    if (fused) {  // the neighbours' places, precomputed in the block's descriptor
        const int q = p ^ 1;
        const int64_t xm = B->fx_m[q], xp = B->fx_p[q], ym = B->fy_m[p], yp = B->fy_p[p];
        const int64_t zm = B->fz_m[p], zp = B->fz_p[p];
        if (xm >= 0) {
            g.dxm = base + xm * 8;
            g.xrm = (uint32_t)ey * 8u;
        }
        if (xp >= 0) {
            g.dxp = base + xp * 8;
            g.xrp = (uint32_t)ey * 8u;
        }
        if (g.y0 == 0 && ym >= 0) {
            ym_src = a.base + ym;
            ym_step = (uint64_t)B->fy_step[0];
        }
        if (g.y0 + g.nyv == ey && yp >= 0) {
            yp_src = a.base + yp;
            yp_step = (uint64_t)B->fy_step[1];
        }
        if (zm >= 0) g.zlo = base + zm * 8;
        if (zp >= 0) g.zhi = base + zp * 8;
    }

    const int64_t xh = B->xoff[p];  // own x-halo arrays of iterate p (before any per-lane branch)
    // Halo loader role: at most one ring cell of the LDS plane per thread.
    // hsrc0 points at plane index 0's value; plane k adds k*hstep doubles.
    const int tid = threadIdx.x;
    const int lx = K::lx(g.nxv);
    int hl = -1;
    const double *hsrc0 = curd;  // lanes without a halo role read a valid cell
    uint64_t hstep = 0;
    {
        int kind, c;
        if (K::ring(tid, g.nxv, g.nyv, kind, c)) {
            if (kind < 2) {
                hsrc0 = (kind ? yp_src : ym_src) + g.x0 + c;
                hstep = kind ? yp_step : ym_step;
                hl = (kind ? (g.nyv + 1) : 0) * lx + c + 1;
            } else {
                const int y = g.y0 + c;
                if (kind == 2) {
                    if (g.x0 == 0) {
                        hsrc0 = a.base + xh + y;
                        hstep = ey;
                    } else {
                        hsrc0 = curd + ps + (uint64_t)(y + 1) * pitch + g.x0 - 1;
                        hstep = ps;
                    }
                    hl = (c + 1) * lx;
                } else {
                    const int xr = g.x0 + g.nxv;
                    if (xr == ex) {
                        hsrc0 = a.base + xh + (int64_t)ey * ez + y;
                        hstep = ey;
                    } else {
                        hsrc0 = curd + ps + (uint64_t)(y + 1) * pitch + xr;
                        hstep = ps;
                    }
                    hl = (c + 1) * lx + g.nxv + 1;
                }
            }
        }
    }

    // a tile of whole rows starts its slots on the line that holds its first
    // cell (planes start on lines), so every wave reads and writes whole lines
    g.shift = g.nxv == pitch ? (int)(((int64_t)(g.y0 + 1) * pitch) & 15) : 0;
    const bool full = K::full(g.nxv, g.nyv) && g.shift == 0;
    // the residual's compare-and-select code only in the sweeps that want it
    const double rmax = full ? (g.want_res ? sweep_planes<K, true, true>(g, hsrc0, hstep, hl, sm, xf)
                                           : sweep_planes<K, true, false>(g, hsrc0, hstep, hl, sm, xf))
                             : (g.want_res ? sweep_planes<K, false, true>(g, hsrc0, hstep, hl, sm, xf)
                                           : sweep_planes<K, false, false>(g, hsrc0, hstep, hl, sm, xf));

    if (g.want_res) {
        // max over the workgroup, then one atomic per tile; the maximum of
        // non-negative doubles orders like their bit patterns, so the result
        // is exact and independent of the order of arrival.
        double m = rmax;
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) {
            const double t = __shfl_xor(m, o);
            m = t > m ? t : m;
        }
        if ((tid & 63) == 0) red[tid >> 6] = m;
        __syncthreads();
        if (tid == 0) {
            double w = 0.0;
            for (int i = 0; i < K::NT / 64; ++i) w = red[i] > w ? red[i] : w;
            atomic_max_agent(a.res + P->res_slot, (unsigned long long)__double_as_longlong(w));
        }
    }
}

template <class K>
__global__ __launch_bounds__(K::NT) void sweep_kernel(SweepArgs a)
{
    __shared__ double sm[K::SMEM];
    __shared__ double red[K::NT / 64];
    __shared__ double xf[4 * K::XROWS];
    // Workgroups are dispatched round-robin over the XCDs (workgroup i to XCD
    // i mod 8).  XCD x runs the contiguous run of tiles xcut[x] ..
    // xcut[x+1]-1 in order, so tiles sharing halo rows run together under one
    // L2.
    // (xcut[x], xcut[x+1]) come straight from the launch arguments by index:
    // one load, issued with the others, instead of a chain of selects that
    // every wave would run.
    const int x = blockIdx.x % kXcds, j = blockIdx.x / kXcds;
    typedef const __attribute__((address_space(4))) int32_t kint32;
    typedef const __attribute__((address_space(4))) char kchar;
    const kint32 *xc = (const kint32 *)((kchar *)__builtin_amdgcn_kernarg_segment_ptr() + offsetof(SweepArgs, xcut));
    const int lo = xc[x], hi = xc[x + 1];
    // A workgroup past its XCD's run (runs differ in length) exits.  The test
    // reads the tile's descriptor and the block table's address (never null),
    // so that every launch argument the tile needs is fetched ahead of it
    // rather than after it.
    const int t = lo + j;
    const Tile tl = a.tiles[a.tile_begin + min(t, a.tile_count - 1)];
    if ((t >= hi ? -1 : tl.block) < 0 || a.blocks == nullptr) return;  // uniform
    sweep_tile<K>(a, tl, sm, red, xf);
}

// Persistent form: a grid of a few workgroups per compute unit; per-XCD
// queues over contiguous tile ranges; a workgroup drains its own XCD's
// queue, then helps the others.
template <class K>
__global__ __launch_bounds__(K::NT) void sweep_kernel_persistent(SweepArgs a)
{
    __shared__ double sm[K::SMEM];
    __shared__ double red[K::NT / 64];
    __shared__ double xf[4 * K::XROWS];
    __shared__ int next_tile;
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
            sweep_tile<K>(a, a.tiles[a.tile_begin + t], sm, red, xf);
            __syncthreads();  // the next tile reuses the LDS
        }
    }
    // Re-arm the other half of the counters for the next persistent launch.
    if (blockIdx.x == 0 && threadIdx.x < kXcds)
        atomic_store_agent(a.queue + (a.queue_slot ^ 1) * kXcds + threadIdx.x, 0u);
}

// ---- unfused halo kernels (one thread per cell of the largest face) ----------

struct FaceGeom {
    int ex, ey, ez, pitch, PS, fx, fy, fz;
    int64_t o[6];  // offsets of the six faces inside S[b] / R[b]
};

__device__ __forceinline__ FaceGeom face_geom(const BlockDesc &B)
{
    FaceGeom g;
    g.ex = B.ext[0];
    g.ey = B.ext[1];
    g.ez = B.ext[2];
    g.pitch = B.pitch;
    g.PS = (int)plane_stride(g.pitch, g.ey);
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
        return (int64_t)(z + 1) * g.PS + (int64_t)(y + 1) * g.pitch + (f == 0 ? 0 : g.ex - 1);
    }
    if (f < 4) {
        const int x = i % g.ex, z = i / g.ex;
        const int row = interior ? (f == 2 ? 1 : g.ey) : (f == 2 ? 0 : g.ey + 1);
        return (int64_t)(z + 1) * g.PS + (int64_t)row * g.pitch + x;
    }
    const int x = i % g.ex, y = i / g.ex;
    const int plane = interior ? (f == 4 ? 1 : g.ez) : (f == 4 ? 0 : g.ez + 1);
    return (int64_t)plane * g.PS + (int64_t)(y + 1) * g.pitch + x;
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

// ---- block shell update -------------------------------------------------------
//
// The cells of a block that read a halo (its outer one-cell shell) updated from
// the current halo storage, with the same expression and order as the sweep:
// Fig. 1's exterior update, run once the halos have been unpacked, after the
// interior update (a sweep clipped to the halo-free cells, SW_INNER) ran
// while they were in transit.

__device__ __forceinline__ int64_t shell_cells(int ex, int ey, int ez)
{
    const int64_t plane = (int64_t)ex * ey;
    const int64_t ring = (ex <= 2 || ey <= 2) ? plane : 2 * (int64_t)ex + 2 * (int64_t)(ey - 2);
    return (ez >= 2 ? 2 : 1) * plane + (int64_t)(ez > 2 ? ez - 2 : 0) * ring;
}

__global__ __launch_bounds__(256) void shell_kernel(double *base, const BlockDesc *blocks, int block_begin,
                                                    int nblocks, int parity)
{
    for (int bb = blockIdx.y; bb < nblocks; bb += gridDim.y) {
        const BlockDesc &B = blocks[block_begin + bb];
        const int ex = B.ext[0], ey = B.ext[1], ez = B.ext[2], pitch = B.pitch;
        const int64_t n = shell_cells(ex, ey, ez);
        const int64_t plane = (int64_t)ex * ey;
        const int64_t full = (ez >= 2 ? 2 : 1) * plane;
        const int64_t ring = (ex <= 2 || ey <= 2) ? plane : 2 * (int64_t)ex + 2 * (int64_t)(ey - 2);
        const int64_t ps = plane_stride(pitch, ey);
        const double *cur = base + B.off[parity];
        double *nxt = base + B.off[parity ^ 1];
        const double *X = base + B.xoff[parity];
        const int64_t stride = (int64_t)gridDim.x * blockDim.x;
        for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
            int x, y, z;
            if (i < full) {
                z = i < plane ? 0 : ez - 1;
                const int64_t r = i % plane;
                x = (int)(r % ex);
                y = (int)(r / ex);
            } else {
                const int64_t j = i - full, r = j % ring;
                z = 1 + (int)(j / ring);
                if (ex <= 2 || ey <= 2) {
                    x = (int)(r % ex);
                    y = (int)(r / ex);
                } else if (r < ex) {
                    x = (int)r;
                    y = 0;
                } else if (r < 2 * (int64_t)ex) {
                    x = (int)(r - ex);
                    y = ey - 1;
                } else {
                    const int64_t q = r - 2 * (int64_t)ex;
                    y = 1 + (int)(q / 2);
                    x = (q & 1) ? ex - 1 : 0;
                }
            }
            const int64_t c = (int64_t)(z + 1) * ps + (int64_t)(y + 1) * pitch + x;
            double s = cur[c];
            s += x > 0 ? cur[c - 1] : X[(int64_t)z * ey + y];
            s += x < ex - 1 ? cur[c + 1] : X[(int64_t)ey * ez + (int64_t)z * ey + y];
            s += cur[c - pitch];
            s += cur[c + pitch];
            s += cur[c - ps];
            s += cur[c + ps];
            nxt[c] = s * kW;
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
        const int ey = B.ext[1], ez = B.ext[2], pitch = B.pitch;
        const int64_t ps = plane_stride(pitch, ey), rows = (int64_t)(ey + 2) * pitch;
        const int64_t cells = ps * (ez + 2);
        double *F0 = base + B.off[0];
        double *F1 = base + B.off[1];
        double *Fp = parity ? F1 : F0;
        const int64_t stride = (int64_t)gridDim.x * blockDim.x;
        for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < cells; idx += stride) {
            const int zz = (int)(idx / ps);
            const int64_t w = idx - (int64_t)zz * ps;
            if (w >= rows) {  // padding at the end of a plane: never read as data
                F0[idx] = 0.0;
                F1[idx] = 0.0;
                continue;
            }
            const int x = (int)(w % pitch), yy = (int)(w / pitch);
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
    const int pitch = B.pitch, ey = B.ext[1];
    return B.off[parity] + (int64_t)(lz + 1) * plane_stride(pitch, ey) + (int64_t)(ly + 1) * pitch + lx;
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
        const int pitch = B.pitch, ey = B.ext[1], ez = B.ext[2];
        const int64_t PS = plane_stride(pitch, ey);
        const double v = src[g];
        for (int q = 0; q < 2; ++q) {
            if (axis == 0) {
                base[B.xoff[q] + (face == 1 ? (int64_t)ey * ez : 0) + ly + (int64_t)ey * lz] = v;
            } else if (axis == 1) {
                base[B.off[q] + (lz + 1) * PS + (int64_t)(face == 2 ? 0 : ey + 1) * pitch + lx] = v;
            } else {
                base[B.off[q] + (face == 4 ? 0 : (int64_t)(ez + 1)) * PS + (int64_t)(ly + 1) * pitch + lx] = v;
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
    const int64_t PS = plane_stride(B.pitch, ey);
    const double *F = base + B.off[parity];
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; g < count; g += stride) {
        const int64_t x = g % ex, y = (g / ex) % ey, z = g / ((int64_t)ex * ey);
        dst[g] = F[(z + 1) * PS + (y + 1) * B.pitch + x];
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

// Streaming copy: each workgroup moves one 16 KiB chunk in a single pass
// (four 16-byte loads per thread in flight, then four stores), the fastest
// shape measured for a 1:1 read/write stream on MI355X.  The last chunk's
// resource is clipped to the buffer, so the tail needs no branch.
constexpr int kCopyChunk = 16384;

__global__ __launch_bounds__(256) void copy_kernel(char *__restrict__ dst, const char *__restrict__ src,
                                                   uint64_t bytes)
{
    const uint64_t base = (uint64_t)blockIdx.x * kCopyChunk;
    const uint64_t left = bytes - base;
    const int len = (int)(left < (uint64_t)kCopyChunk ? left : (uint64_t)kCopyChunk);
    const __amdgpu_buffer_rsrc_t rs = rsrc(src + base, (uint64_t)len);
    const __amdgpu_buffer_rsrc_t rd = rsrc(dst + base, (uint64_t)len);
    typedef int i32x4 __attribute__((ext_vector_type(4)));
    i32x4 v[4];
#pragma unroll
    for (int u = 0; u < 4; ++u)
        v[u] = __builtin_amdgcn_raw_buffer_load_b128(rs, (int)((threadIdx.x + u * 256) * 16), 0, kAuxNT);
#pragma unroll
    for (int u = 0; u < 4; ++u)
        __builtin_amdgcn_raw_buffer_store_b128(v[u], rd, (int)((threadIdx.x + u * 256) * 16), 0, kAuxNT);
}

int grid_for(int64_t work, int per_block, int cap)
{
    int64_t g = (work + per_block - 1) / per_block;
    if (g < 1) g = 1;
    if (g > cap) g = cap;
    return (int)g;
}

constexpr int kMaxGridY = 65535;

// Variant table.  Fixed tiles (TX, NTY, RY, PF): TX x (NTY*RY) cells, TX*NTY
// threads, loads of PF planes beyond the next one in flight.  Flattened tiles
// (NT, RY, PF): NT threads, up to NT*RY cells of whole row segments.  The
// indices are part of the tuning interface: append, never reorder.
#define J3D_VARIANTS(X, F) \
    X(64, 16, 4, 1)        \
    X(64, 8, 8, 1)         \
    X(64, 4, 4, 1)         \
    X(64, 8, 4, 1)         \
    X(128, 8, 4, 1)        \
    X(128, 4, 8, 1)        \
    X(128, 4, 4, 1)        \
    X(256, 4, 4, 1)        \
    X(32, 8, 4, 1)         \
    X(64, 4, 8, 1)         \
    X(64, 16, 2, 3)        \
    X(64, 8, 4, 2)         \
    X(64, 16, 2, 1)        \
    X(64, 16, 2, 2)        \
    X(64, 4, 8, 2)         \
    X(128, 4, 4, 2)        \
    X(128, 8, 2, 3)        \
    X(160, 4, 4, 1)        \
    X(192, 4, 4, 1)        \
    X(64, 8, 2, 2)         \
    X(64, 4, 4, 2)         \
    X(64, 4, 4, 4)         \
    X(64, 8, 4, 3)         \
    X(128, 4, 4, 3)        \
    X(128, 4, 4, 4)        \
    F(512, 4, 1)           \
    F(512, 4, 2)           \
    F(256, 8, 1)           \
    F(1024, 2, 2)          \
    F(512, 2, 2)           \
    F(256, 4, 1)           \
    F(512, 2, 1)           \
    F(512, 2, 3)           \
    F(512, 1, 2)           \
    F(1024, 1, 2)          \
    F(256, 2, 2)           \
    F(1024, 1, 3)          \
    F(512, 1, 3)

struct VariantEntry {
    int tile_x, tile_y, threads;  // tile_x 0: flattened, tile_y its cell capacity
    int prefetch;
    void (*fn)(SweepArgs);
    void (*persistent)(SweepArgs);
};

#define J3D_TILED(TX, NTY, RY, PF)                                                          \
    {TX, NTY * RY, TX * NTY, PF, sweep_kernel<Tiled<TX, NTY, RY, PF>>,                      \
     sweep_kernel_persistent<Tiled<TX, NTY, RY, PF>>},
#define J3D_FLAT(NT, RY, PF) \
    {0, NT * RY, NT, PF, sweep_kernel<Flat<NT, RY, PF>>, sweep_kernel_persistent<Flat<NT, RY, PF>>},
const VariantEntry kVariants[] = {J3D_VARIANTS(J3D_TILED, J3D_FLAT)};
#undef J3D_TILED
#undef J3D_FLAT
constexpr int kVariantCount = sizeof(kVariants) / sizeof(kVariants[0]);

}  // namespace

int variant_count() { return kVariantCount; }

VariantInfo variant_info(int v)
{
    const VariantEntry &e = kVariants[v];
    return VariantInfo{e.tile_x, e.tile_y, e.threads, e.prefetch};
}

int launch_sweep(int variant, const SweepArgs &a, int grid, void *stream)
{
    if (variant < 0 || variant >= kVariantCount || grid < 1) return (int)hipErrorInvalidValue;
    const VariantEntry &e = kVariants[variant];
    if (a.flags & SW_PERSIST) {
        hipLaunchKernelGGL(e.persistent, dim3(grid), dim3(e.threads), 0, (hipStream_t)stream, a);
        return (int)hipGetLastError();
    }
    SweepArgs b = a;
    if (b.xcut[kXcds] == 0) {
        // equal counts: XCD x takes q or q+1 tiles, which a grid of one
        // workgroup per tile covers exactly
        if (grid != b.tile_count) return (int)hipErrorInvalidValue;
        const int q = b.tile_count / kXcds, r = b.tile_count % kXcds;
        for (int x = 0; x <= kXcds; ++x) b.xcut[x] = x * q + (x < r ? x : r);
    }
    hipLaunchKernelGGL(e.fn, dim3(grid), dim3(e.threads), 0, (hipStream_t)stream, b);
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

int launch_shell(double *base, const BlockDesc *blocks, int32_t block_begin, int32_t nblocks, int64_t max_shell,
                 int parity, void *stream)
{
    const dim3 grid(grid_for(max_shell, 256, 4096), nblocks < kMaxGridY ? nblocks : kMaxGridY);
    hipLaunchKernelGGL(shell_kernel, grid, dim3(256), 0, (hipStream_t)stream, base, blocks, block_begin, nblocks,
                       parity);
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
    const uint64_t chunks = (bytes + kCopyChunk - 1) / kCopyChunk;
    if (chunks == 0) return 0;
    if (chunks > 0x7fffffffull) return (int)hipErrorInvalidValue;
    hipLaunchKernelGGL(copy_kernel, dim3((unsigned)chunks), dim3(256), 0, (hipStream_t)stream, (char *)dst,
                       (const char *)src, bytes);
    return (int)hipGetLastError();
}

}  // namespace j3d
