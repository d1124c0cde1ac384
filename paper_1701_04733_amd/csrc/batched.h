// Descriptors and launchers for the grouped APSP kernels (internal).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

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

enum { BATCH_TILE_128 = 0, BATCH_TILE_64 = 1 };

// One output tile of one squaring of one graph.
struct BatchItem {
    int graph;
    int tm, tn;  // tile coordinates in units of the tile shape
    int kind;    // BATCH_TILE_128 or BATCH_TILE_64
    int step;    // squaring index s >= 1
    int pad;
};

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

inline int batch_tiles_of(int n, int kind) {
    const int t = kind == BATCH_TILE_128 ? 128 : 64;
    return (n + t - 1) / t;
}

}  // namespace btas
