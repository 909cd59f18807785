// j3d_plan.cpp -- host-only planning and the host-only C-ABI queries.
#include <algorithm>
#include <climits>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>

#include "j3d_host.hpp"

namespace j3d {

namespace {
thread_local std::string g_last_error;
}

j3d_status set_error(j3d_status st, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return st;
}

void clear_error() { g_last_error.clear(); }

const char *last_error_text() { return g_last_error.c_str(); }

uint64_t stream_start(uint64_t seed, uint64_t pid)
{
    // SplitMix64 (Steele, Lea, Flood 2014): state advances by the golden gamma,
    // the output is the mixed state.  Output number m from state s mixes
    // s + m*gamma.
    uint64_t z = seed + (pid + 1) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

j3d_status auto_split(const int64_t n[3], int32_t parts, int32_t nb[3])
{
    if (parts < 1) return set_error(J3D_EINVAL, "auto split: parts must be >= 1 (got %d)", parts);
    if (parts > (1 << 22)) return set_error(J3D_EINVAL, "auto split: %d blocks, more than 2^22", parts);
    bool found = false;
    unsigned __int128 best = 0;
    int32_t bc[3] = {0, 0, 0};
    for (int32_t a = 1; a <= parts && a <= n[0]; ++a) {
        if (parts % a) continue;
        for (int32_t b = 1; b <= parts / a; ++b) {
            if ((parts / a) % b) continue;
            const int32_t c = parts / a / b;
            if (a > n[0] || b > n[1] || c > n[2]) continue;
            // total area of the cuts between blocks (the communication volume)
            const unsigned __int128 cost =
                (unsigned __int128)(a - 1) * (uint64_t)(n[1] * n[2]) +
                (unsigned __int128)(b - 1) * (uint64_t)(n[0] * n[2]) +
                (unsigned __int128)(c - 1) * (uint64_t)(n[0] * n[1]);
            const bool better = !found || cost < best ||
                                (cost == best && (c > bc[2] || (c == bc[2] && b > bc[1])));
            if (better) {
                found = true;
                best = cost;
                bc[0] = a;
                bc[1] = b;
                bc[2] = c;
            }
        }
    }
    if (!found)
        return set_error(J3D_EINVAL, "auto split: no factorisation of %d blocks fits %lldx%lldx%lld",
                         parts, (long long)n[0], (long long)n[1], (long long)n[2]);
    nb[0] = bc[0];
    nb[1] = bc[1];
    nb[2] = bc[2];
    return J3D_OK;
}

j3d_status resolve_decomp(const j3d_problem *p, Decomp *d)
{
    if (!p) return set_error(J3D_EINVAL, "problem is NULL");
    for (int a = 0; a < 3; ++a) {
        if (p->n[a] < 1 || p->n[a] > INT32_MAX)
            return set_error(J3D_EINVAL, "n[%d] = %lld out of range [1, 2^31-1]", a, (long long)p->n[a]);
        d->n[a] = p->n[a];
    }
    for (int f = 0; f < 6; ++f)
        if (!std::isfinite(p->bc[f])) return set_error(J3D_EINVAL, "bc[%d] is not finite", f);
    const bool all_zero = p->nblk[0] == 0 && p->nblk[1] == 0 && p->nblk[2] == 0;
    if (all_zero) {
        if (p->split[0] || p->split[1] || p->split[2])
            return set_error(J3D_EINVAL, "explicit splits need explicit block counts");
        const int32_t parts = p->auto_parts == 0 ? 1 : p->auto_parts;
        j3d_status st = auto_split(d->n, parts, d->nb);
        if (st != J3D_OK) return st;
        for (int a = 0; a < 3; ++a) {
            d->ext[a].assign(d->nb[a], d->n[a] / d->nb[a]);
            for (int64_t i = 0; i < d->n[a] % d->nb[a]; ++i) d->ext[a][i] += 1;
        }
    } else {
        for (int a = 0; a < 3; ++a) {
            const int32_t nb = p->nblk[a];
            if (nb < 1 || nb > d->n[a])
                return set_error(J3D_EINVAL, "nblk[%d] = %d out of range [1, n[%d]]", a, nb, a);
            d->nb[a] = nb;
            if (p->split[a]) {
                int64_t sum = 0;
                d->ext[a].resize(nb);
                for (int32_t i = 0; i < nb; ++i) {
                    const int64_t e = p->split[a][i];
                    if (e < 1) return set_error(J3D_EINVAL, "split[%d][%d] = %lld < 1", a, i, (long long)e);
                    d->ext[a][i] = e;
                    sum += e;
                }
                if (sum != d->n[a])
                    return set_error(J3D_EINVAL, "split[%d] sums to %lld, not n[%d] = %lld", a,
                                     (long long)sum, a, (long long)d->n[a]);
            } else {
                if (d->n[a] % nb)
                    return set_error(J3D_EINVAL, "even split needs n[%d] %% nblk[%d] == 0 (%lld %% %d)",
                                     a, a, (long long)d->n[a], nb);
                d->ext[a].assign(nb, d->n[a] / nb);
            }
        }
    }
    for (int a = 0; a < 3; ++a) {
        d->org[a].resize(d->nb[a]);
        int64_t o = 0;
        for (int32_t i = 0; i < d->nb[a]; ++i) {
            d->org[a][i] = o;
            o += d->ext[a][i];
        }
    }
    const int64_t nblocks = (int64_t)d->nb[0] * d->nb[1] * d->nb[2];
    if (nblocks > (1 << 22)) return set_error(J3D_EINVAL, "%lld blocks: more than 2^22", (long long)nblocks);
    for (int32_t bz = 0; bz < d->nb[2]; ++bz)
        for (int32_t by = 0; by < d->nb[1]; ++by)
            for (int32_t bx = 0; bx < d->nb[0]; ++bx) {
                const int64_t ex = d->ext[0][bx], ey = d->ext[1][by], ez = d->ext[2][bz];
                if (block_field_cells(ex, ey, ez) > INT32_MAX || ey * ez > INT32_MAX / 2 ||
                    ex * ez > INT32_MAX || ex * ey > INT32_MAX)
                    return set_error(J3D_EINVAL, "block %lldx%lldx%lld exceeds 2^31 cells with halos",
                                     (long long)ex, (long long)ey, (long long)ez);
                // the sweep addresses one plane (with its ghost rows) by 32-bit byte offsets
                if (plane_stride(row_pitch(ex), ey) * 8 > INT32_MAX)
                    return set_error(J3D_EINVAL, "block %lldx%lldx%lld: an x-y plane exceeds 2^28 cells",
                                     (long long)ex, (long long)ey, (long long)ez);
            }
    return J3D_OK;
}

namespace {

struct Bump {
    uint64_t off = 0;
    uint64_t take(uint64_t bytes, uint64_t align = 256)
    {
        off = align_up(off, align);
        const uint64_t at = off;
        off += bytes;
        return at;
    }
};

int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }

int max_ez(const Plan &plan, int32_t b0, int32_t b1)
{
    int m = 1;
    for (int32_t b = b0; b < b1; ++b) m = plan.blocks[b].ext[2] > m ? plan.blocks[b].ext[2] : m;
    return m;
}

}  // namespace

int find_variant(int tile_x, int tile_y, int threads)
{
    for (int v = 0; v < variant_count(); ++v) {
        const VariantInfo vi = variant_info(v);
        if (vi.tile_x == tile_x && vi.tile_y == tile_y && vi.threads == threads) return v;
    }
    return -1;
}

int find_flat_variant(int threads, int cells, int prefetch)
{
    for (int v = 0; v < variant_count(); ++v) {
        const VariantInfo vi = variant_info(v);
        if (vi.tile_x == 0 && vi.tile_y == cells && vi.threads == threads && vi.prefetch == prefetch) return v;
    }
    return -1;
}

uint64_t count_tiles(const Plan &plan, int variant, int zchunk)
{
    const VariantInfo vi = variant_info(variant);
    const int zc = zchunk > 0 ? zchunk : max_ez(plan, 0, (int32_t)plan.blocks.size());
    uint64_t n = 0;
    for (const BlockDesc &B : plan.blocks) {
        int64_t ntx, nty;
        tiles_xy(vi, B.ext[0], B.ext[1], &ntx, &nty);
        n += (uint64_t)(ntx * nty * ceil_div(B.ext[2], zc));
    }
    return n;
}

j3d_status make_plan(int32_t count, const j3d_problem *probs, bool with_sr, Plan *plan)
{
    if (count < 1 || !probs) return set_error(J3D_EINVAL, "need at least one problem");
    plan->blocks.clear();
    plan->probs.assign(count, ProbPlan{});
    plan->with_sr = with_sr;
    plan->max_face = 0;
    plan->max_cells = 0;
    for (int32_t i = 0; i < count; ++i) {
        ProbPlan &pp = plan->probs[i];
        j3d_status st = resolve_decomp(&probs[i], &pp.d);
        if (st != J3D_OK) return st;
        for (int f = 0; f < 6; ++f) pp.bc[f] = probs[i].bc[f];
        pp.s0 = stream_start(probs[i].seed, probs[i].pid);
        pp.block_begin = (int32_t)plan->blocks.size();
        const Decomp &d = pp.d;
        pp.nblocks = d.nb[0] * d.nb[1] * d.nb[2];
        if ((int64_t)plan->blocks.size() + pp.nblocks > (1 << 22))
            return set_error(J3D_EINVAL, "more than 2^22 blocks in total");
        auto index = [&](int32_t bx, int32_t by, int32_t bz) {
            return pp.block_begin + bx + d.nb[0] * (by + d.nb[1] * bz);
        };
        for (int32_t bz = 0; bz < d.nb[2]; ++bz)
            for (int32_t by = 0; by < d.nb[1]; ++by)
                for (int32_t bx = 0; bx < d.nb[0]; ++bx) {
                    BlockDesc B;
                    std::memset(&B, 0, sizeof B);
                    B.ext[0] = (int32_t)d.ext[0][bx];
                    B.ext[1] = (int32_t)d.ext[1][by];
                    B.ext[2] = (int32_t)d.ext[2][bz];
                    B.org[0] = (int32_t)d.org[0][bx];
                    B.org[1] = (int32_t)d.org[1][by];
                    B.org[2] = (int32_t)d.org[2][bz];
                    B.pitch = (int32_t)row_pitch(B.ext[0]);
                    B.prob = i;
                    B.nbr[0] = bx > 0 ? index(bx - 1, by, bz) : -1;
                    B.nbr[1] = bx + 1 < d.nb[0] ? index(bx + 1, by, bz) : -1;
                    B.nbr[2] = by > 0 ? index(bx, by - 1, bz) : -1;
                    B.nbr[3] = by + 1 < d.nb[1] ? index(bx, by + 1, bz) : -1;
                    B.nbr[4] = bz > 0 ? index(bx, by, bz - 1) : -1;
                    B.nbr[5] = bz + 1 < d.nb[2] ? index(bx, by, bz + 1) : -1;
                    const int64_t ex = B.ext[0], ey = B.ext[1], ez = B.ext[2];
                    B.face_total = 2 * (ey * ez + ex * ez + ex * ey);
                    const int64_t mf = std::max(ey * ez, std::max(ex * ez, ex * ey));
                    plan->max_face = (int32_t)std::max<int64_t>(plan->max_face, mf);
                    plan->max_cells = (int32_t)std::max<int64_t>(plan->max_cells, block_field_cells(ex, ey, ez));
                    plan->blocks.push_back(B);
                }
    }

    Bump bump;
    const uint64_t nb = plan->blocks.size();
    plan->off_blocks = bump.take(nb * sizeof(BlockDesc));
    plan->off_probs = bump.take((uint64_t)count * sizeof(ProbDesc));
    uint64_t cap = 0;
    for (int v = 0; v < variant_count(); ++v) cap = std::max(cap, count_tiles(*plan, v, kMinZchunk));
    plan->tiles_cap = cap;
    plan->off_tiles = bump.take(cap * sizeof(Tile));
    for (ProbPlan &pp : plan->probs)
        pp.maps_off = bump.take((uint64_t)(pp.d.n[0] + pp.d.n[1] + pp.d.n[2]) * 2 * sizeof(int32_t));
    plan->off_res = bump.take((uint64_t)(count + 1) * sizeof(uint64_t));
    plan->off_queue = bump.take(16 * sizeof(uint32_t));
    for (int q = 0; q < 2; ++q)
        for (ProbPlan &pp : plan->probs) {
            pp.f_off[q] = align_up(bump.off, 4096);
            uint64_t cells = 0;
            for (int32_t b = pp.block_begin; b < pp.block_begin + pp.nblocks; ++b) {
                BlockDesc &B = plan->blocks[b];
                const uint64_t c = (uint64_t)block_field_cells(B.ext[0], B.ext[1], B.ext[2]);
                B.off[q] = (int64_t)(bump.take(c * sizeof(double), 4096) / sizeof(double));
                cells += c;
            }
            pp.field_cells = cells;
        }
    for (int q = 0; q < 2; ++q)
        for (BlockDesc &B : plan->blocks)
            B.xoff[q] = (int64_t)(bump.take(2 * (uint64_t)B.ext[1] * B.ext[2] * sizeof(double)) /
                                  sizeof(double));
    if (with_sr)
        for (BlockDesc &B : plan->blocks)
            B.sr_off = (int64_t)(bump.take(2 * (uint64_t)B.face_total * sizeof(double)) / sizeof(double));
    link_halo_sources(plan->blocks.data(), plan->blocks.size());
    uint64_t bounce = 0;
    for (const ProbPlan &pp : plan->probs) {
        const int64_t n0 = pp.d.n[0], n1 = pp.d.n[1], n2 = pp.d.n[2];
        uint64_t need = (uint64_t)std::max(n0 * n1, std::max(n1 * n2, n0 * n2));
        need = std::max<uint64_t>(need, std::min<uint64_t>((uint64_t)(n0 * n1 * n2), 1ull << 22));
        bounce = std::max(bounce, need);
    }
    plan->bounce_doubles = bounce;
    plan->off_bounce = bump.take(bounce * sizeof(double), 4096);
    plan->total = align_up(bump.off, 4096);
    return J3D_OK;
}

void make_tiles(const Plan &plan, int32_t b0, int32_t b1, int variant, int zchunk,
                std::vector<Tile> *tiles, std::vector<int32_t> *block_first)
{
    const VariantInfo vi = variant_info(variant);
    const int zc = zchunk > 0 ? zchunk : max_ez(plan, 0, (int32_t)plan.blocks.size());
    if (block_first) block_first->clear();
    for (int32_t b = b0; b < b1; ++b) {
        const BlockDesc &B = plan.blocks[b];
        if (block_first) block_first->push_back((int32_t)tiles->size());
        int64_t ntx, nty;
        tiles_xy(vi, B.ext[0], B.ext[1], &ntx, &nty);
        const int ex = B.ext[0], ey = B.ext[1], ez = B.ext[2];
        const int ntz = (int)ceil_div(ez, zc);
        // z is cut into ntz near-equal pieces, so no tile is a thin remainder
        for (int tz = 0; tz < ntz; ++tz)
            for (int ty = 0; ty < (int)nty; ++ty)
                for (int tx = 0; tx < (int)ntx; ++tx) {
                    Tile t{};
                    t.block = b;
                    t.tx = tx;
                    t.ty = ty;
                    t.tz = tz;
                    if (vi.tile_x == 0) {  // flattened: x pieces on 16-column boundaries, y near-equal
                        const FlatShape f = flat_shape(ex, ey, vi.threads, vi.tile_y);
                        t.x0 = flat_x0(ex, f.tnx, tx);
                        t.nxv = flat_x0(ex, f.tnx, tx + 1) - t.x0;
                    } else {  // fixed: TX-wide columns, y near-equal
                        t.x0 = tx * vi.tile_x;
                        t.nxv = std::min(vi.tile_x, ex - t.x0);
                    }
                    t.y0 = (int32_t)((int64_t)ty * ey / nty);
                    t.nyv = (int32_t)((int64_t)(ty + 1) * ey / nty) - t.y0;
                    t.z0 = (int32_t)((int64_t)tz * ez / ntz);
                    t.nzv = (int32_t)((int64_t)(tz + 1) * ez / ntz) - t.z0;
                    tiles->push_back(t);
                }
    }
    if (block_first) block_first->push_back((int32_t)tiles->size());
}

void tile_work(const std::vector<Tile> &tiles, std::vector<uint64_t> *prefix)
{
    // A tile's time is set by the planes it streams, whatever share of its
    // lanes hold a cell (measured: weighting by cells balanced the batched
    // workload worse than equal counts), plus a fixed cost of about one plane
    // for its first memory latency.
    constexpr uint64_t kTileFixed = 1;  // planes
    prefix->assign(tiles.size() + 1, 0);
    uint64_t acc = 0;
    for (size_t i = 0; i < tiles.size(); ++i) {
        acc += (uint64_t)(tiles[i].nzv + 2) + kTileFixed;
        (*prefix)[i + 1] = acc;
    }
}

void default_tune(const Plan &plan, int cus, j3d_tune *t)
{
    // Shapes measured fastest on MI355X (one workgroup per tile; the
    // persistent schedule never won for a single problem):
    //   <= 64 wide:         flattened tiles of 512 threads, 2 cells each (64 x 16
    //                       on 64-wide blocks), through 64 planes;
    //   widths not a multiple of 16 (rows ending inside a cache line), or
    //   129..192 wide:      flattened tiles of 512 threads, 4 cells each, which
    //                       write whole lines at row ends, z-chunks of 32;
    //   <= 128:             128 x 16 tiles of 512 threads, z-chunks of 32;
    //   wider:              128 x 32 tiles of 1024 threads, z-chunks of 64.
    int exm = 1;
    bool ragged = false;
    for (const BlockDesc &B : plan.blocks) {
        exm = std::max(exm, B.ext[0]);
        ragged = ragged || B.ext[0] % 16 != 0;
    }
    int v, zc;
    if (exm <= 64) {
        v = find_flat_variant(512, 1024, 3);
        zc = 64;
    } else if (ragged || (exm > 128 && exm <= 192)) {
        v = find_flat_variant(512, 2048, 1);
        zc = 32;
    } else if (exm <= 128) {
        v = find_variant(128, 16, 512);
        zc = 32;
    } else {
        v = find_variant(128, 32, 1024);
        zc = 64;
    }
    if (v < 0) v = 0;  // a shape missing from the table: any variant is correct, only slower
    t->variant = v;
    t->blocks_per_cu = 0;
    // a shallower chunk if the launch would otherwise have too few workgroups
    // to fill the chip
    const int ezm = max_ez(plan, 0, (int32_t)plan.blocks.size());
    while (zc > 16 && count_tiles(plan, v, zc) < (uint64_t)(2 * (cus > 0 ? cus : 256))) zc = (zc + 1) / 2;
    t->zchunk = zc >= ezm ? 0 : zc;
}

j3d_status check_tune(const Plan &plan, const j3d_tune *t, int *zchunk_eff)
{
    if (t->variant < 0 || t->variant >= variant_count())
        return set_error(J3D_EINVAL, "tune variant %d out of range [0, %d)", t->variant, variant_count());
    if (t->zchunk < 0) return set_error(J3D_EINVAL, "tune zchunk %d < 0", t->zchunk);
    if (t->blocks_per_cu < 0 || t->blocks_per_cu > 32)
        return set_error(J3D_EINVAL, "tune blocks_per_cu %d out of range [0, 32]", t->blocks_per_cu);
    const uint64_t n = count_tiles(plan, t->variant, t->zchunk);
    if (n > plan.tiles_cap || n > INT32_MAX)
        return set_error(J3D_EINVAL, "tune gives %llu tiles, more than the table holds (%llu)",
                         (unsigned long long)n, (unsigned long long)plan.tiles_cap);
    *zchunk_eff = t->zchunk > 0 ? t->zchunk : max_ez(plan, 0, (int32_t)plan.blocks.size());
    return J3D_OK;
}

}  // namespace j3d

using namespace j3d;

extern "C" {

const char *j3d_last_error(void) { return last_error_text(); }

const char *j3d_version(void) { return "j3d 0.1 (gfx950)"; }

j3d_status j3d_auto_split(const int64_t n[3], int32_t parts, int32_t nblk_out[3])
{
    if (!n || !nblk_out) return set_error(J3D_EINVAL, "NULL argument");
    for (int a = 0; a < 3; ++a)
        if (n[a] < 1) return set_error(J3D_EINVAL, "n[%d] < 1", a);
    int32_t nb[3];
    j3d_status st = auto_split(n, parts, nb);
    if (st != J3D_OK) return st;
    for (int a = 0; a < 3; ++a) nblk_out[a] = nb[a];
    return J3D_OK;
}

j3d_status j3d_block_extents(const j3d_problem *p, int32_t nblk_out[3], int64_t *extents_out,
                             int64_t cap)
{
    if (!nblk_out) return set_error(J3D_EINVAL, "nblk_out is NULL");
    Decomp d;
    j3d_status st = resolve_decomp(p, &d);
    if (st != J3D_OK) return st;
    const int64_t need = (int64_t)d.nb[0] + d.nb[1] + d.nb[2];
    if (extents_out && cap < need)
        return set_error(J3D_EINVAL, "extents_out holds %lld values, %lld needed", (long long)cap,
                         (long long)need);
    for (int a = 0; a < 3; ++a) nblk_out[a] = d.nb[a];
    if (extents_out) {
        int64_t k = 0;
        for (int a = 0; a < 3; ++a)
            for (int64_t e : d.ext[a]) extents_out[k++] = e;
    }
    return J3D_OK;
}

j3d_status j3d_arena_bytes(const j3d_problem *p, uint64_t *bytes)
{
    if (!bytes) return set_error(J3D_EINVAL, "bytes is NULL");
    Plan plan;
    j3d_status st = make_plan(1, p, true, &plan);
    if (st != J3D_OK) return st;
    *bytes = plan.total;
    return J3D_OK;
}

j3d_status j3d_field_bytes(const j3d_problem *p, uint64_t *bytes)
{
    if (!bytes) return set_error(J3D_EINVAL, "bytes is NULL");
    Plan plan;
    j3d_status st = make_plan(1, p, true, &plan);
    if (st != J3D_OK) return st;
    uint64_t b = 0;
    for (const BlockDesc &B : plan.blocks)
        b += 2 * sizeof(double) *
             ((uint64_t)block_field_cells(B.ext[0], B.ext[1], B.ext[2]) + 2ull * B.ext[1] * B.ext[2]);
    *bytes = b;
    return J3D_OK;
}

j3d_status j3d_variant_info(int32_t variant, int32_t *tile_x, int32_t *tile_y, int32_t *threads)
{
    if (variant < 0 || variant >= variant_count())
        return set_error(J3D_EINVAL, "variant %d out of range [0, %d)", variant, variant_count());
    const VariantInfo vi = variant_info(variant);
    if (tile_x) *tile_x = vi.tile_x;
    if (tile_y) *tile_y = vi.tile_y;
    if (threads) *threads = vi.threads;
    return J3D_OK;
}

j3d_status j3d_batch_arena_bytes(int32_t count, const j3d_problem *probs, uint64_t *bytes)
{
    if (!bytes) return set_error(J3D_EINVAL, "bytes is NULL");
    Plan plan;
    j3d_status st = make_plan(count, probs, true, &plan);
    if (st != J3D_OK) return st;
    *bytes = plan.total;
    return J3D_OK;
}

}  // extern "C"
