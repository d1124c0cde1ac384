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
    int np;  // > 0: the buffers are np x np (np = ld, a multiple of 64) and rows /
             // columns n..np-1 hold the absent value (BATCH_TILE_W64D items)
};

// Tile kinds.  The block kinds run in the 256-thread grouped kernel, the wave
// kinds in the 64-thread one (one wave per tile); a launch holds kinds of one
// family only.
enum {
    BATCH_TILE_128 = 0,   // 128x128 outputs, 4 waves, 8x8 per thread
    BATCH_TILE_64 = 1,    // 64x64 outputs, 4 waves, 4x4 per thread
    BATCH_TILE_W64 = 2,   // 64x64 outputs, 1 wave, 8x8 per thread
    BATCH_TILE_W32 = 3,   // 32x32 outputs, 1 wave, 4x4 per thread
    BATCH_TILE_W64D = 4,  // 64x64 outputs of the padded matrix, 1 wave, direct LDS loads
    BATCH_TILE_W64x32D = 5,  // the same, 64 rows x 32 columns (edge strips, see tile_plan)
    BATCH_TILE_W32x64D = 6,  // 32 rows x 64 columns
    BATCH_TILE_W32D = 7,     // 32 x 32
    BATCH_TILE_NONE = -1  // placeholder: the workgroup exits at once
};

inline int tile_rows(int kind) {
    return kind == BATCH_TILE_128 ? 128
           : (kind == BATCH_TILE_W32 || kind == BATCH_TILE_W32x64D || kind == BATCH_TILE_W32D) ? 32 : 64;
}
inline int tile_cols(int kind) {
    return kind == BATCH_TILE_128 ? 128
           : (kind == BATCH_TILE_W32 || kind == BATCH_TILE_W64x32D || kind == BATCH_TILE_W32D) ? 32 : 64;
}
// Kernel family of a tile kind: 0 = four-wave blocks, 1 = one-wave tiles,
// 2 = one-wave direct-load tiles of padded matrices.
inline int tile_family(int kind) {
    return kind >= BATCH_TILE_W64D ? 2 : (kind == BATCH_TILE_W64 || kind == BATCH_TILE_W32) ? 1 : 0;
}
inline bool tile_is_wave(int kind) { return tile_family(kind) == 1; }
// Storage edge of a graph's padded buffers.
inline int padded_edge(int n) { return (n + 63) / 64 * 64; }
// Batches of at most this many graphs, all within the automatic single-launch
// size, are solved one single launch per graph instead of by a batched plan.
constexpr int BATCH_DIRECT_MAX_COUNT = 2;

// One output tile of one squaring of one graph.
struct BatchItem {
    int graph;
    int m0, n0;  // first output row / column of the tile
    int kind;    // BATCH_TILE_*
    int step;    // squaring index s >= 1
    int pad;
};

// How a graph's n x n output is cut into tiles.  SHAPE_128/64/MIXED use the
// block kinds, SHAPE_W64/WMIX the wave kinds, SHAPE_W64D the direct kind.
enum {
    SHAPE_128 = 0, SHAPE_64 = 1, SHAPE_MIXED = 2, SHAPE_W64 = 3, SHAPE_WMIX = 4, SHAPE_W64D = 5,
    NUM_SHAPES = 6
};
constexpr int NUM_FAMILIES = 3;
inline int shape_family(int shape) {
    return shape == SHAPE_W64D ? 2 : (shape == SHAPE_W64 || shape == SHAPE_WMIX) ? 1 : 0;
}
inline bool shape_is_wave(int shape) { return shape_family(shape) == 1; }

struct TileRef {
    int m0, n0, kind;
};

// Tiles covering [0,n)^2.  The mixed shapes use the large tile on the
// floor(n/big)*big core and the small one on the remainder strips, which keeps
// most work on the larger tile while padding the ragged edge only to the
// small edge (SHAPE_MIXED: 128 + 64, SHAPE_WMIX: 64 + 32).  SHAPE_W64D covers
// [0, n rounded up to 32)^2: 64x64 tiles, and when n mod 64 is 1..32, a last
// column strip of 64x32 tiles, a last row strip of 32x64 and a 32x32 corner
// (the padding work of those graphs halves; the whole 4096-graph workload's
// padded over useful terms goes from 1.20 to 1.10).
inline std::vector<TileRef> tile_plan(int n, int shape) {
    std::vector<TileRef> out;
    if (n <= 0) return out;
    if (shape == SHAPE_W64D) {
        const int r = n % 64;
        const int core = (r == 0 || r > 32) ? (n + 63) / 64 * 64 : n / 64 * 64;
        for (int i = 0; i < core; i += 64)
            for (int j = 0; j < core; j += 64) out.push_back({i, j, BATCH_TILE_W64D});
        if (core < n) {
            for (int i = 0; i < core; i += 64) out.push_back({i, core, BATCH_TILE_W64x32D});
            for (int j = 0; j < core; j += 64) out.push_back({core, j, BATCH_TILE_W32x64D});
            out.push_back({core, core, BATCH_TILE_W32D});
        }
        return out;
    }
    if (shape == SHAPE_128 || shape == SHAPE_64 || shape == SHAPE_W64) {
        const int kind = shape == SHAPE_128 ? BATCH_TILE_128
                         : shape == SHAPE_64 ? BATCH_TILE_64 : BATCH_TILE_W64;
        const int t = tile_rows(kind);
        for (int i = 0; i < n; i += t)
            for (int j = 0; j < n; j += t) out.push_back({i, j, kind});
        return out;
    }
    const bool wave = shape == SHAPE_WMIX;
    const int big = wave ? 64 : 128, small = big / 2;
    const int kbig = wave ? BATCH_TILE_W64 : BATCH_TILE_128;
    const int ksmall = wave ? BATCH_TILE_W32 : BATCH_TILE_64;
    const int core = n / big * big;
    for (int i = 0; i < core; i += big)
        for (int j = 0; j < core; j += big) out.push_back({i, j, kbig});
    for (int i = 0; i < n; i += small)
        for (int j = 0; j < n; j += small)
            if (i >= core || j >= core) out.push_back({i, j, ksmall});
    return out;
}

// Output elements a tile covers (padding included).
inline double tile_area(int kind) {
    return (double)tile_rows(kind) * tile_cols(kind);
}

// Padded output area of a plan, small tiles weighted by `w_small` (their
// lower efficiency per element); the model used when tiles are not timed.
inline double tile_plan_cost(int n, int shape, double w_small = 1.15) {
    double c = 0;
    for (const TileRef& t : tile_plan(n, shape))
        c += tile_area(t.kind) * (t.kind == BATCH_TILE_64 || t.kind == BATCH_TILE_W32 ? w_small : 1.0);
    return c;
}

// Reorder one launch's items so that workgroup i, which the hardware places
// on XCD i % 8 (each XCD has its own L2), works on tiles whose graph lives on
// that XCD: a graph goes whole to the XCD with the least work so far (largest
// first), unless it holds more than half of one XCD's share of the launch's
// items; such a graph is cut into 8 bands of consecutive tiles, one per XCD.
// Queues of unequal length are padded with placeholder items.  `items` must
// be grouped by graph.
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
        auto work = [&](const BatchItem& it) { return tile_area(it.kind) * n; };
        if (cnt * 2 * X > items.size()) {
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

static_assert(SHAPE_128 == BTAS_TILES_128 && SHAPE_64 == BTAS_TILES_64 &&
                  SHAPE_MIXED == BTAS_TILES_MIXED && SHAPE_W64 == BTAS_TILES_W64 &&
                  SHAPE_WMIX == BTAS_TILES_WMIX && SHAPE_W64D == BTAS_TILES_W64_DIRECT,
              "internal shape codes are the ABI's");

// Cheapest block-family shape by the padded-area model.
inline int model_shape(int n) {
    int best = SHAPE_128;
    for (int s : {SHAPE_64, SHAPE_MIXED})
        if (tile_plan_cost(n, s) < tile_plan_cost(n, best)) best = s;
    return best;
}

// Cheapest wave-family shape by the padded-area model (a 32x32 wave tile
// costs about 1.3x a 64x64 one per element: half the register tile).
inline int model_wave_shape(int n) {
    return tile_plan_cost(n, SHAPE_WMIX, 1.3) < tile_plan_cost(n, SHAPE_W64) ? SHAPE_WMIX : SHAPE_W64;
}

// An external matrix (the caller's W or D) paired with a graph.  Jobs of one
// launch own consecutive ranges of workgroups: [first_block, first_block + nblocks).
// The copy launchers take an optional table block_job[workgroup] -> job
// (else each workgroup finds its job by binary search over first_block).
struct BatchCopy {
    int graph;
    int first_block;
    int nblocks;
    int pad;
    long ld_ext;
    const void* ext;
};

// Squarings for items[0, nitems): one workgroup per item, 256 threads for the
// block kinds, 64 for the wave and direct kinds (`family` selects the kernel:
// 0 block, 1 wave, 2 direct; every item of the launch must belong to it,
// placeholders aside; direct items need graphs with padded buffers, np > 0).  maxabs (int32 only, may
// be null): per-graph max |finite element of D_0|; an int32 graph with
// 2^T * maxabs <= 2^23-1 is computed on the binary32 pipeline, reading int32
// storage with conversions, or (float_storage) buffers that
// launch_grouped_init filled with binary32 values.  changed (may be null):
// with early_stride == 0, changed[graph] is set to 1 when a squaring changed
// some entry; with early_stride > 0 (early exit), squaring s sets
// changed[s * early_stride + graph] and an item of squaring s >= 2 whose graph
// left squaring s-1 unchanged returns at once (from then on both buffers
// hold the fixpoint, so skipping is exact).
hipError_t launch_grouped_step(int dt, const BatchGraph* graphs, const BatchItem* items,
                               int nitems, const int* maxabs, int* changed, hipStream_t s,
                               int family = 0, bool float_storage = false, int early_stride = 0);
// int32: maxabs[graph] <- max |finite element of I (+) W| (maxabs zeroed
// first); the first pass of the float-storage mode.
hipError_t launch_grouped_maxabs(const BatchGraph* graphs, const BatchCopy* jobs, int njobs,
                                 int total_blocks, int* maxabs, hipStream_t s,
                                 const int* block_job = nullptr);
// buf[parity] <- I (+) W for each job (graphs with np > 0: rows and columns
// n..np-1 of that buffer <- the absent value).  int32 without float_storage:
// maxabs[graph] <- max |finite element| (maxabs zeroed first).  int32 with
// float_storage: maxabs is complete (launch_grouped_maxabs) and graphs in the
// binary32-exact range are stored as binary32.  total_blocks = sum of the
// jobs' nblocks.
hipError_t launch_grouped_init(int dt, const BatchGraph* graphs, const BatchCopy* jobs, int njobs,
                               int total_blocks, int* maxabs, hipStream_t s,
                               bool float_storage = false, const int* block_job = nullptr);
// D_ext <- buf[(parity + T) & 1] for each job; float_maxabs (int32
// float-storage mode, else null) converts the graphs stored as binary32 back.
hipError_t launch_grouped_copy_out(const BatchGraph* graphs, const BatchCopy* jobs, int njobs,
                                   int total_blocks, hipStream_t s,
                                   const int* float_maxabs = nullptr,
                                   const int* block_job = nullptr);
// Workgroups an n x n copy job should get (about 16384 elements each, <= 256;
// with 4096 the 4096-graph workload's max-scan took 268 instead of 160 us,
// init and copy-out unchanged).
inline int copy_blocks_for(int n) {
    long b = ((long)n * n + 16383) / 16384;
    return (int)(b < 1 ? 1 : (b > 256 ? 256 : b));
}
hipError_t launch_clear_ints(int* p, int count, hipStream_t s);

// Graphs of at most BATCH_LDS_MAX_N vertices can be solved whole, one
// workgroup each, with both ping-pong matrices in LDS: straight from the
// caller's W to the caller's D, no internal buffers and no grid-wide launch
// boundary between squarings (opt-in, BTAS_BATCH_LDS=1).
constexpr int BATCH_LDS_MAX_N = 64;
struct BatchSmall {
    int n, T;
    long ldw, ldd;
    const void* W;
    void* D;
};
hipError_t launch_batched_lds_solve(int dt, const BatchSmall* jobs, int njobs, bool early,
                                    hipStream_t s);
// D (n x n, leading dimension ld) <- I (+) W for a COO edge list W given by
// device arrays rows/cols/w of length nnz (indices already range-checked);
// duplicate edges keep the smallest weight.
hipError_t launch_densify(int dt, void* D, int n, int ld, int nnz, const int32_t* rows,
                          const int32_t* cols, const void* w, hipStream_t s);



}  // namespace btas
