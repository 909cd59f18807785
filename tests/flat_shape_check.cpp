// Host check of the flattened-tile shape rule (flat_shape, flat_x0) shared by
// the planner and the sweep kernel: for every block width and height and every
// thread count / capacity a variant can have, each tile fits its variant (cells
// plus the line-alignment shift of a whole-row tile within the capacity, one
// halo-ring loader thread per ring cell, rows within the x-face buffer) and the
// tiles cover the plane.  Exit status 0 when every case holds.
#include <cstdio>

#include "j3d_internal.hpp"

using namespace j3d;

int main()
{
    const int nts[] = {256, 512, 1024};
    const int rys[] = {1, 2, 3, 4, 8};
    long bad = 0, n = 0;
    for (int nt : nts)
        for (int ry : rys) {
            const int cap = nt * ry;
            for (int ex = 1; ex <= 1200; ++ex)
                for (int ey = 1; ey <= 700; ey += (ey < 64 ? 1 : 7)) {
                    const FlatShape s = flat_shape(ex, ey, nt, cap);
                    ++n;
                    int covered_x = 0;
                    for (int tx = 0; tx < s.tnx; ++tx) {
                        const int w = flat_x0(ex, s.tnx, tx + 1) - flat_x0(ex, s.tnx, tx);
                        if (w < 1 || flat_x0(ex, s.tnx, tx) != covered_x) ++bad;
                        covered_x += w;
                        for (int ty = 0; ty < s.tny; ++ty) {
                            const int y0 = (int)((long)ty * ey / s.tny), y1 = (int)((long)(ty + 1) * ey / s.tny);
                            const int h = y1 - y0;
                            const int shift = w == ex ? (int)(((long)(y0 + 1) * ex) & 15) : 0;
                            if (h < 1 || w > s.wx || h > s.hy || w * h + shift > cap || 2 * (w + h) > nt ||
                                h > nt / 2) {
                                if (bad < 10)
                                    std::printf("ex %d ey %d nt %d cap %d: tile %dx%d shift %d (tnx %d wx %d hy %d)\n",
                                                ex, ey, nt, cap, w, h, shift, s.tnx, s.wx, s.hy);
                                ++bad;
                            }
                        }
                    }
                    if (covered_x != ex) ++bad;
                }
        }
    std::printf("checked %ld shapes, %ld bad\n", n, bad);
    return bad != 0;
}
