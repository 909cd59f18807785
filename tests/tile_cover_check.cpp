// Host check of the sweep tile tables (make_tiles, linked from libj3d.so): for
// many block shapes, every kernel variant and several z-chunks, the tiles of a
// block lie inside it, fit their variant, carry the block's index, and cover
// every cell exactly once; count_tiles agrees with the table.  Exit status 0
// when every case holds.
#include <cstdio>
#include <vector>

#include "j3d_host.hpp"

using namespace j3d;

int main()
{
    const int widths[] = {1, 2, 15, 16, 17, 33, 63, 64, 65, 100, 127, 128, 129, 160, 192, 193, 255, 256, 300};
    const int heights[] = {1, 3, 16, 31, 129};
    const int depths[] = {1, 5, 33};
    const int zchunks[] = {0, 4, 7, 16, 32, 64};
    long bad = 0, n = 0;
    std::vector<unsigned char> seen;
    for (int ex : widths)
        for (int ey : heights)
            for (int ez : depths) {
                Plan plan;
                BlockDesc B{};
                B.ext[0] = ex;
                B.ext[1] = ey;
                B.ext[2] = ez;
                B.pitch = ex;
                B.prob = 0;
                plan.blocks.assign(1, B);
                for (int v = 0; v < variant_count(); ++v) {
                    const VariantInfo vi = variant_info(v);
                    for (int zc : zchunks) {
                        ++n;
                        std::vector<Tile> tiles;
                        std::vector<int32_t> first;
                        make_tiles(plan, 0, 1, v, zc, &tiles, &first);
                        long fail = 0;
                        if (first.size() != 2 || first[0] != 0 || first[1] != (int32_t)tiles.size()) ++fail;
                        if (count_tiles(plan, v, zc) != tiles.size()) ++fail;
                        seen.assign((size_t)ex * ey * ez, 0);
                        for (const Tile &t : tiles) {
                            if (t.block != 0 || t.nxv < 1 || t.nyv < 1 || t.nzv < 1 || t.x0 < 0 || t.y0 < 0 ||
                                t.z0 < 0 || t.x0 + t.nxv > ex || t.y0 + t.nyv > ey || t.z0 + t.nzv > ez) {
                                ++fail;
                                continue;
                            }
                            if (vi.tile_x > 0 ? (t.nxv > vi.tile_x || t.nyv > vi.tile_y)
                                              : (t.nxv * t.nyv > vi.tile_y))
                                ++fail;
                            if (zc > 0 && t.nzv > zc) ++fail;
                            for (int z = t.z0; z < t.z0 + t.nzv; ++z)
                                for (int y = t.y0; y < t.y0 + t.nyv; ++y)
                                    for (int x = t.x0; x < t.x0 + t.nxv; ++x) ++seen[((size_t)z * ey + y) * ex + x];
                        }
                        for (unsigned char c : seen)
                            if (c != 1) {
                                ++fail;
                                break;
                            }
                        if (fail) {
                            if (bad < 20)
                                printf("block %dx%dx%d variant %d zchunk %d: %ld failures\n", ex, ey, ez, v, zc, fail);
                            ++bad;
                        }
                    }
                }
            }
    printf("tile tables: %ld cases, %ld bad\n", n, bad);
    return bad == 0 ? 0 : 1;
}
