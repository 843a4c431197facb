// Host checks of the persistent served launch's tile and counter layout
// (vdi_internal.h): which XCD group takes which tile, how many tiles each
// group has in a job, where each completion counter lives, and a simulation
// of one job's tiles finishing in random order across the groups, counted the
// way the kernel counts them (one counter per group, then a count of
// finished groups), which must report the job finished exactly once, at its
// last tile.
#include <stddef.h>
#include <stdint.h>

#include <random>
#include <vector>

#include "vdi_internal.h"

extern "C" int persist_layout_check(int max_tiles, int trials, unsigned seed)
{
    using namespace vdi;
    if (sizeof(PCounter) != 128 || sizeof(PJob) % 256 != 0) return 1;
    if (offsetof(PQueue, tail) % 128 || offsetof(PQueue, stop) % 128 || offsetof(PHost, stop) % 128) return 2;
    // Counters: distinct, each on its own 128-byte line, inside the job's block.
    std::vector<int> seen;
    for (int part = 0; part < 2; ++part)
        for (int x = 0; x <= kXcds; ++x) {
            const int w = done_word(part, x);
            if (w < 0 || w + 32 > kDoneWords || w % 32) return 3;
            for (int o : seen)
                if (o == w) return 4;
            seen.push_back(w);
        }
    for (int n = 0; n <= max_tiles; ++n) {
        uint32_t sum = 0, groups = 0;
        for (uint32_t x = 0; x < (uint32_t)kXcds; ++x) {
            sum += group_tiles((uint32_t)n, x);
            groups += group_tiles((uint32_t)n, x) > 0;
        }
        if (sum != (uint32_t)n || groups != (uint32_t)(n < kXcds ? n : kXcds)) return 5;
    }
    std::mt19937 rng(seed);
    for (int t = 0; t < trials; ++t) {
        const uint32_t n = 1 + rng() % (uint32_t)max_tiles;
        const uint64_t t0 = (uint64_t)kXcds * (rng() % 1000);  // a job starts at a multiple of the XCD count
        std::vector<uint64_t> order(n);
        for (uint32_t i = 0; i < n; ++i) order[i] = t0 + i;
        std::shuffle(order.begin(), order.end(), rng);
        std::vector<uint32_t> D(kDoneWords, 0u);
        int finished = 0;
        for (uint32_t i = 0; i < n; ++i) {
            const uint32_t x = (uint32_t)(order[i] % kXcds);  // the group that takes global tile order[i]
            const uint32_t c = ++D[done_word(0, (int)x)];
            bool last = false;
            if (c == group_tiles(n, x)) last = ++D[done_word(0, kXcds)] == (n < (uint32_t)kXcds ? n : (uint32_t)kXcds);
            if (last) {
                if (i + 1 != n) return 6;  // reported before the last tile
                ++finished;
            }
        }
        if (finished != 1) return 7;
    }
    return 0;
}
