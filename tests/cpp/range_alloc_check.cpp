// Host-logic check of the serving engine's pool allocator: random alloc /
// release sequences never hand out overlapping or out-of-range blocks, usage
// is accounted exactly, and releasing everything coalesces to one block.
#include <cstdio>
#include <random>
#include <vector>

#include "range_alloc.h"

int main() {
    int bad = 0;
    std::mt19937_64 rng(12345);
    for (int trial = 0; trial < 200; ++trial) {
        btas::RangeAllocator a;
        const size_t size = 256 * (1 + rng() % 4096);
        a.reset(size);
        struct Blk { size_t off, len; };
        std::vector<Blk> live;
        size_t used = 0;
        for (int op = 0; op < 400; ++op) {
            if (live.empty() || rng() % 3 != 0) {
                const size_t want = 1 + rng() % (size / 4 + 1);
                const size_t off = a.alloc(want);
                if (off == SIZE_MAX) continue;
                const size_t len = btas::RangeAllocator::round(want);
                if (off % 256 || off + len > a.size()) ++bad;
                for (const Blk& b : live)
                    if (off < b.off + b.len && b.off < off + len) ++bad;
                live.push_back({off, len});
                used += len;
            } else {
                const size_t i = rng() % live.size();
                a.release(live[i].off, live[i].len);
                used -= live[i].len;
                live.erase(live.begin() + i);
            }
            if (a.used() != used || a.peak() < used) ++bad;
        }
        for (const Blk& b : live) a.release(b.off, b.len);
        if (a.used() != 0 || a.free_blocks() != 1 || a.alloc(a.size()) != 0) ++bad;
    }
    std::printf("range allocator failures: %d\n", bad);
    return bad != 0;
}
