// Descriptors and launchers for the grouped APSP kernels (internal).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>
#include <vector>

#include "btas.h"

namespace btas {

// One graph's device state: two padded n x n buffers (ld % 4 == 0, 16-byte
// aligned); squaring s (1-based) reads buf[(parity + s - 1) & 1] and writes
// buf[(parity + s) & 1]; D_0 lives in buf[parity & 1]; T squarings in total.
struct BatchGraph {
    void* buf[2];
    int n;
    int ld;
    int T;
    int parity;
};

enum { BATCH_TILE_128 = 0, BATCH_TILE_64 = 1, BATCH_TILE_NONE = -1 };

// One output tile of one squaring of one graph.
struct BatchItem {
    int graph;
    int m0, n0;  // first output row / column of the tile
    int kind;    // BATCH_TILE_128 (128x128 outputs), BATCH_TILE_64 (64x64), or
                 // BATCH_TILE_NONE (placeholder: the workgroup exits at once)
    int step;    // squaring index s >= 1
    int pad;
};

// How a graph's n x n output is cut into tiles.
enum { SHAPE_128 = 0, SHAPE_64 = 1, SHAPE_MIXED = 2, NUM_SHAPES = 3 };

struct TileRef {
    int m0, n0, kind;
};

// Tiles covering [0,n)^2.  SHAPE_MIXED uses 128x128 tiles on the
// floor(n/128)*128 core and 64x64 tiles on the remainder strips, which keeps
// most work on the larger tile while padding the ragged edge only to 64.
inline std::vector<TileRef> tile_plan(int n, int shape) {
    std::vector<TileRef> out;
    if (n <= 0) return out;
    if (shape == SHAPE_128 || shape == SHAPE_64) {
        const int t = shape == SHAPE_128 ? 128 : 64;
        const int kind = shape == SHAPE_128 ? BATCH_TILE_128 : BATCH_TILE_64;
        for (int i = 0; i < n; i += t)
            for (int j = 0; j < n; j += t) out.push_back({i, j, kind});
        return out;
    }
    const int core = n / 128 * 128;
    // 64-wide segments: the core split in halves plus the remainder
    for (int i = 0; i < core; i += 128)
        for (int j = 0; j < core; j += 128) out.push_back({i, j, BATCH_TILE_128});
    for (int i = 0; i < n; i += 64)
        for (int j = 0; j < n; j += 64)
            if (i >= core || j >= core) out.push_back({i, j, BATCH_TILE_64});
    return out;
}

// Padded output area of a plan, 64x64 tiles weighted by `w64` (their lower
// efficiency per element); the model used when tiles are not timed.
inline double tile_plan_cost(int n, int shape, double w64 = 1.15) {
    double c = 0;
    for (const TileRef& t : tile_plan(n, shape)) c += t.kind == BATCH_TILE_128 ? 16384.0 : 4096.0 * w64;
    return c;
}

// Reorder one launch's items so that workgroup i, which the hardware places
// on XCD i % 8 (each XCD has its own L2), works on tiles whose graph lives on
// that XCD: graphs with fewer than 64 tiles go whole to the XCD with the least
// work so far (largest first), larger graphs are cut into 8 bands of
// consecutive tiles, one per XCD.  Queues of unequal length are padded with
// placeholder items.  `items` must be grouped by graph.
inline std::vector<BatchItem> order_for_xcds(const std::vector<BatchItem>& items,
                                             const std::vector<int>& graph_n) {
    constexpr int X = 8;
    std::vector<std::vector<BatchItem>> q(X);
    double load[X] = {0};
    size_t i = 0;
    while (i < items.size()) {
        size_t j = i;
        while (j < items.size() && items[j].graph == items[i].graph) ++j;
        const size_t cnt = j - i;
        const double n = graph_n[items[i].graph];
        auto work = [&](const BatchItem& it) { return (it.kind == BATCH_TILE_128 ? 16384.0 : 4096.0) * n; };
        if (cnt >= 64) {
            for (int x = 0; x < X; ++x)
                for (size_t t = i + cnt * x / X; t < i + cnt * (x + 1) / X; ++t) {
                    q[x].push_back(items[t]);
                    load[x] += work(items[t]);
                }
        } else {
            int best = 0;
            for (int x = 1; x < X; ++x)
                if (load[x] < load[best]) best = x;
            for (size_t t = i; t < j; ++t) {
                q[best].push_back(items[t]);
                load[best] += work(items[t]);
            }
        }
        i = j;
    }
    size_t len = 0;
    for (auto& v : q) len = std::max(len, v.size());
    std::vector<BatchItem> out;
    out.reserve(len * X);
    const BatchItem none{0, 0, 0, BATCH_TILE_NONE, 1, 0};
    for (size_t r = 0; r < len; ++r)
        for (int x = 0; x < X; ++x) out.push_back(r < q[x].size() ? q[x][r] : none);
    return out;
}

inline int model_shape(int n) {
    int best = SHAPE_128;
    for (int s : {SHAPE_64, SHAPE_MIXED})
        if (tile_plan_cost(n, s) < tile_plan_cost(n, best)) best = s;
    return best;
}

// An external matrix (the caller's W or D) paired with a graph.  Jobs of one
// launch own consecutive ranges of workgroups: [first_block, first_block + nblocks).
struct BatchCopy {
    int graph;
    int first_block;
    int nblocks;
    int pad;
    long ld_ext;
    const void* ext;
};

// Squarings for items[0, nitems): one workgroup of 256 threads per item.
// maxabs (int32 only, may be null): per-graph max |finite weight| recorded by
// launch_grouped_init.  changed (may be null): per-graph flag set to 1 when a
// squaring changed some entry.
hipError_t launch_grouped_step(int dt, const BatchGraph* graphs, const BatchItem* items,
                               int nitems, const int* maxabs, int* changed, hipStream_t s);
// buf[parity] <- I (+) W for each job; int32: maxabs[graph] <- max |finite W|
// (maxabs must be zeroed first).
// total_blocks = sum of the jobs' nblocks.
hipError_t launch_grouped_init(int dt, const BatchGraph* graphs, const BatchCopy* jobs, int njobs,
                               int total_blocks, int* maxabs, hipStream_t s);
// D_ext <- buf[(parity + T) & 1] for each job.
hipError_t launch_grouped_copy_out(const BatchGraph* graphs, const BatchCopy* jobs, int njobs,
                                   int total_blocks, hipStream_t s);
// Workgroups an n x n copy job should get (about 4096 elements each, <= 256).
inline int copy_blocks_for(int n) {
    long b = ((long)n * n + 4095) / 4096;
    return (int)(b < 1 ? 1 : (b > 256 ? 256 : b));
}
hipError_t launch_clear_ints(int* p, int count, hipStream_t s);
// D (n x n, leading dimension ld) <- I (+) W for a COO edge list W given by
// device arrays rows/cols/w of length nnz (indices already range-checked);
// duplicate edges keep the smallest weight.
hipError_t launch_densify(int dt, void* D, int n, int ld, int nnz, const int32_t* rows,
                          const int32_t* cols, const void* w, hipStream_t s);



}  // namespace btas
