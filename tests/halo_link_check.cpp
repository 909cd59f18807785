// Host check of the fused sweep's precomputed halo sources and x-face
// targets (link_halo_sources): on random block grids with random offsets,
// every field equals the neighbour-descriptor formula it stands for, a face
// without a neighbour gives -1 (the own ghost layer), and a lone block built
// field by field from a zeroed descriptor (as the pool builds a request's)
// ends with every source at -1.  Exit status 0 when every case holds.
#include <cstdio>
#include <cstring>
#include <random>
#include <vector>

#include "j3d_host.hpp"

using namespace j3d;

int main()
{
    std::mt19937_64 rng(7);
    long bad = 0, n = 0;
    for (int rep = 0; rep < 300; ++rep) {
        const int nb[3] = {1 + (int)(rng() % 4), 1 + (int)(rng() % 4), 1 + (int)(rng() % 4)};
        std::vector<int> ext[3];
        for (int a = 0; a < 3; ++a)
            for (int i = 0; i < nb[a]; ++i) ext[a].push_back(1 + (int)(rng() % 70));
        std::vector<BlockDesc> blocks;
        auto index = [&](int x, int y, int z) { return x + nb[0] * (y + nb[1] * z); };
        for (int z = 0; z < nb[2]; ++z)
            for (int y = 0; y < nb[1]; ++y)
                for (int x = 0; x < nb[0]; ++x) {
                    BlockDesc B;
                    std::memset(&B, 0, sizeof B);
                    B.ext[0] = ext[0][x];
                    B.ext[1] = ext[1][y];
                    B.ext[2] = ext[2][z];
                    B.pitch = (int32_t)row_pitch(B.ext[0]);
                    B.nbr[0] = x > 0 ? index(x - 1, y, z) : -1;
                    B.nbr[1] = x + 1 < nb[0] ? index(x + 1, y, z) : -1;
                    B.nbr[2] = y > 0 ? index(x, y - 1, z) : -1;
                    B.nbr[3] = y + 1 < nb[1] ? index(x, y + 1, z) : -1;
                    B.nbr[4] = z > 0 ? index(x, y, z - 1) : -1;
                    B.nbr[5] = z + 1 < nb[2] ? index(x, y, z + 1) : -1;
                    for (int q = 0; q < 2; ++q) {
                        B.off[q] = (int64_t)(rng() % (1ull << 30));
                        B.xoff[q] = (int64_t)(rng() % (1ull << 30));
                    }
                    blocks.push_back(B);
                }
        link_halo_sources(blocks.data(), blocks.size());
        for (const BlockDesc &B : blocks) {
            ++n;
            bool ok = true;
            const int64_t ey = B.ext[1], ez = B.ext[2], pitch = B.pitch, ps = plane_stride(pitch, ey);
            for (int q = 0; q < 2; ++q) {
                const BlockDesc *N;
                N = B.nbr[0] >= 0 ? &blocks[B.nbr[0]] : nullptr;
                ok = ok && B.fx_m[q] == (N ? N->xoff[q] + ey * ez : -1);
                N = B.nbr[1] >= 0 ? &blocks[B.nbr[1]] : nullptr;
                ok = ok && B.fx_p[q] == (N ? N->xoff[q] : -1);
                N = B.nbr[2] >= 0 ? &blocks[B.nbr[2]] : nullptr;
                ok = ok && B.fy_m[q] == (N ? N->off[q] + plane_stride(pitch, N->ext[1]) + (int64_t)N->ext[1] * pitch : -1);
                if (N) ok = ok && B.fy_step[0] == plane_stride(pitch, N->ext[1]);
                N = B.nbr[3] >= 0 ? &blocks[B.nbr[3]] : nullptr;
                ok = ok && B.fy_p[q] == (N ? N->off[q] + plane_stride(pitch, N->ext[1]) + pitch : -1);
                if (N) ok = ok && B.fy_step[1] == plane_stride(pitch, N->ext[1]);
                N = B.nbr[4] >= 0 ? &blocks[B.nbr[4]] : nullptr;
                ok = ok && B.fz_m[q] == (N ? N->off[q] + (int64_t)N->ext[2] * ps : -1);
                N = B.nbr[5] >= 0 ? &blocks[B.nbr[5]] : nullptr;
                ok = ok && B.fz_p[q] == (N ? N->off[q] + ps : -1);
            }
            if (!ok) {
                if (bad < 5) std::printf("bad block %dx%dx%d\n", B.ext[0], B.ext[1], B.ext[2]);
                ++bad;
            }
        }
    }
    // a lone block built from a zeroed descriptor
    BlockDesc B;
    std::memset(&B, 0, sizeof B);
    B.ext[0] = B.ext[1] = B.ext[2] = 40;
    B.pitch = 40;
    for (int f = 0; f < 6; ++f) B.nbr[f] = -1;
    link_halo_sources(&B, 1);
    ++n;
    for (int q = 0; q < 2; ++q)
        if (B.fx_m[q] != -1 || B.fx_p[q] != -1 || B.fy_m[q] != -1 || B.fy_p[q] != -1 || B.fz_m[q] != -1 ||
            B.fz_p[q] != -1) {
            std::printf("bad lone block\n");
            ++bad;
            break;
        }
    std::printf("%ld cases, %ld bad\n", n, bad);
    return bad ? 1 : 0;
}
