// Host check of the per-XCD tile ranges (xcd_split) that the one-workgroup-
// per-tile sweep launch uses: for random tile work and launch windows, the
// ranges partition the window in order, each XCD's work is within one tile of
// an equal share, and the kernel's mapping of the returned grid (workgroup b
// runs tile xcut[b % 8] + b / 8 when that is below xcut[b % 8 + 1]) runs every
// tile of the window exactly once.  Small launches keep equal counts (all cuts
// zero, grid = tile count).  Exit status 0 when every case holds.
#include <cstdio>
#include <random>

#include "j3d_host.hpp"

using namespace j3d;

int main()
{
    std::mt19937_64 rng(12345);
    long bad = 0, n = 0;
    for (int rep = 0; rep < 4000; ++rep) {
        const int ntiles = 1 + (int)(rng() % 40000);
        std::vector<uint64_t> prefix(ntiles + 1, 0);
        const int spread = 1 + (int)(rng() % 3);  // uniform, mixed, heavy-tailed tile work
        uint64_t maxw = 0;
        for (int i = 0; i < ntiles; ++i) {
            uint64_t w = 2048 + rng() % 70000;
            if (spread == 2 && rng() % 4 == 0) w *= 8;
            if (spread == 3 && rng() % 50 == 0) w *= 60;
            prefix[i + 1] = prefix[i] + w;
        }
        const int32_t t0 = (int32_t)(rng() % ntiles);
        const int32_t cnt = 1 + (int32_t)(rng() % (ntiles - t0));
        int32_t cut[kXcdCount + 1];
        const int grid = xcd_split(prefix, t0, cnt, cut);
        ++n;
        bool ok = true;
        if (cnt < 4 * 256) {
            for (int x = 0; x <= kXcdCount; ++x) ok = ok && cut[x] == 0;
            ok = ok && grid == cnt;
        } else {
            ok = ok && cut[0] == 0 && cut[kXcdCount] == cnt;
            int longest = 0;
            for (int x = 0; x < kXcdCount; ++x) {
                ok = ok && cut[x] <= cut[x + 1];
                longest = std::max(longest, cut[x + 1] - cut[x]);
            }
            ok = ok && grid == kXcdCount * std::max(longest, 1);
            for (int i = t0; i < t0 + cnt; ++i) maxw = std::max(maxw, prefix[i + 1] - prefix[i]);
            const double share = (double)(prefix[t0 + cnt] - prefix[t0]) / kXcdCount;
            for (int x = 0; x < kXcdCount; ++x) {
                const double w = (double)(prefix[t0 + cut[x + 1]] - prefix[t0 + cut[x]]);
                ok = ok && w <= share + 1.0 * maxw && w >= share - 1.0 * maxw;
            }
            std::vector<int> runs(cnt, 0);
            for (int b = 0; b < grid; ++b) {
                const int x = b % kXcdCount, j = b / kXcdCount;
                if (cut[x] + j < cut[x + 1]) ++runs[cut[x] + j];
            }
            for (int i = 0; i < cnt; ++i) ok = ok && runs[i] == 1;
        }
        if (!ok) {
            if (bad < 10)
                std::printf("bad: ntiles %d t0 %d cnt %d grid %d cuts %d %d %d %d %d %d %d %d %d\n", ntiles, t0, cnt,
                            grid, cut[0], cut[1], cut[2], cut[3], cut[4], cut[5], cut[6], cut[7], cut[8]);
            ++bad;
        }
    }
    std::printf("%ld cases, %ld bad\n", n, bad);
    return bad ? 1 : 0;
}
