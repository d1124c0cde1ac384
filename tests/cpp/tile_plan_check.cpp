// Host-logic check: every tile plan of the grouped APSP kernels covers each
// output element of an n x n matrix exactly once, with tile origins in range
// and tile kinds of the shape's family only (one kernel per launch).
#include <cstdio>
#include <vector>

#include "batched.h"

int main() {
    int bad = 0;
    for (int n = 1; n <= 1100; ++n)
        for (int s = 0; s < btas::NUM_SHAPES; ++s) {
            std::vector<int> cov((size_t)n * n, 0);
            for (const btas::TileRef& t : btas::tile_plan(n, s)) {
                const int rows = btas::tile_rows(t.kind), cols = btas::tile_cols(t.kind);
                if (btas::tile_family(t.kind) != btas::shape_family(s)) ++bad;
                if (t.m0 < 0 || t.n0 < 0 || t.m0 >= n || t.n0 >= n) {
                    ++bad;
                    continue;
                }
                for (int i = t.m0; i < t.m0 + rows && i < n; ++i)
                    for (int j = t.n0; j < t.n0 + cols && j < n; ++j) cov[(size_t)i * n + j]++;
                // a direct-load tile stays inside the buffer padded to 64
                if (btas::tile_family(t.kind) == 2 &&
                    (t.m0 + rows > btas::padded_edge(n) || t.n0 + cols > btas::padded_edge(n) ||
                     t.m0 % 32 || t.n0 % 32))
                    ++bad;
            }
            for (int c : cov)
                if (c != 1) {
                    std::printf("n=%d shape=%d: an element is covered %d times\n", n, s, c);
                    ++bad;
                    break;
                }
        }
    // XCD ordering: a permutation of the items plus placeholders, and every
    // graph with at most 1/16 of the items stays on one XCD (position mod 8).
    {
        std::vector<btas::BatchItem> items;
        std::vector<int> graph_n;
        for (int g = 0; g < 300; ++g) {
            const int n = g == 3 ? 12000 : 16 + (g * 37) % 1500;  // one graph large enough to band
            graph_n.push_back(n);
            for (const btas::TileRef& t : btas::tile_plan(n, g % btas::NUM_SHAPES))
                items.push_back({g, t.m0, t.n0, t.kind, 1, 0});
        }
        const auto out = btas::order_for_xcds(items, graph_n);
        if (out.size() % 8) ++bad;
        std::vector<int> seen(items.size(), 0), xcd(graph_n.size(), -1);
        std::vector<int> count(graph_n.size(), 0);
        for (const auto& it : items) count[it.graph]++;
        for (size_t p = 0; p < out.size(); ++p) {
            const auto& it = out[p];
            if (it.kind == btas::BATCH_TILE_NONE) continue;
            size_t idx = 0;
            for (; idx < items.size(); ++idx)
                if (!seen[idx] && items[idx].graph == it.graph && items[idx].m0 == it.m0 &&
                    items[idx].n0 == it.n0 && items[idx].kind == it.kind)
                    break;
            if (idx == items.size()) { ++bad; continue; }
            seen[idx] = 1;
            if (count[it.graph] * 16 <= (int)items.size()) {
                if (xcd[it.graph] < 0) xcd[it.graph] = (int)(p % 8);
                else if (xcd[it.graph] != (int)(p % 8)) ++bad;
            }
        }
        for (int s : seen)
            if (!s) ++bad;
        // both placements occur in this mix: some graphs whole, some banded
        int whole = 0, banded = 0;
        for (size_t g = 0; g < graph_n.size(); ++g) (count[g] * 16 <= (int)items.size() ? whole : banded)++;
        if (whole == 0 || banded == 0) {
            std::printf("xcd order mix not exercised: whole=%d banded=%d\n", whole, banded);
            ++bad;
        }
    }
    std::printf("tile plan failures: %d\n", bad);
    return bad != 0;
}
