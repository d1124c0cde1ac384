// Host-logic check: every tile plan of the grouped APSP kernels covers each
// output element of an n x n matrix exactly once, with tile origins in range.
#include <cstdio>
#include <vector>

#include "batched.h"

int main() {
    int bad = 0;
    for (int n = 1; n <= 1100; ++n)
        for (int s = 0; s < btas::NUM_SHAPES; ++s) {
            std::vector<int> cov((size_t)n * n, 0);
            for (const btas::TileRef& t : btas::tile_plan(n, s)) {
                const int sz = t.kind == btas::BATCH_TILE_128 ? 128 : 64;
                if (t.m0 < 0 || t.n0 < 0 || t.m0 >= n || t.n0 >= n) {
                    ++bad;
                    continue;
                }
                for (int i = t.m0; i < t.m0 + sz && i < n; ++i)
                    for (int j = t.n0; j < t.n0 + sz && j < n; ++j) cov[(size_t)i * n + j]++;
            }
            for (int c : cov)
                if (c != 1) {
                    std::printf("n=%d shape=%d: an element is covered %d times\n", n, s, c);
                    ++bad;
                    break;
                }
        }
    std::printf("tile plan failures: %d\n", bad);
    return bad != 0;
}
