// Grouped kernels for many independent APSP solves (batched and served).
//
// Each graph g owns two padded n_g x n_g buffers (leading dimension a multiple
// of 4, 256-byte aligned) and squares back and forth between them, as in the
// single-solve driver (Sec. III: D_t = D_{t-1} (+) D_{t-1} (.) D_{t-1}).  One
// launch of the grouped step kernel performs one squaring for a whole list of
// output tiles drawn from many graphs; work items name (graph, tile row, tile
// column, tile shape) and each graph carries its own step parity, so graphs
// at different steps (served requests) can share a launch.  Small elementwise
// kernels map W -> I (+) W into the internal buffer and copy the final matrix
// out to the caller's layout.
#include <hip/hip_runtime.h>

#include <type_traits>

#include "batched.h"
#include "lds_solve.h"
#include "gemm_tile.h"
#include "flat_index.h"

namespace btas {

// One-wave 64x64 tile (8x8 per lane, 8-deep k-blocks) of the direct-load step
// kernel: operands go straight into LDS, so no staging registers; 8 KB of LDS
// per workgroup.
using CfgWD = GemmCfg<64, 64, 8, 8, 8>;
// Edge strips of graphs with n mod 64 in 1..32 (one wave each as well):
// 64x32, 32x64 and 32x32 outputs, 8x4 / 4x8 / 4x4 per lane.
using CfgWD64x32 = GemmCfg<64, 32, 8, 8, 4>;
using CfgWD32x64 = GemmCfg<32, 64, 8, 4, 8>;
using CfgWD32 = GemmCfg<32, 32, 8, 4, 4>;

// int32 graphs whose finite weights satisfy 2^T * max|w| <= FP32_EXACT_MAX
// keep every finite distance of every step inside the binary32-exact range
// (a step's entries are sums of at most 2^t weights), so their squarings run
// on the binary32 pipeline.  The init kernel records max|w| per graph.
template <typename T>
__device__ __forceinline__ bool graph_is_narrow(const BatchGraph& g, const int* maxabs, int gi) {
    if constexpr (std::is_same_v<T, int32_t>) {
        if (maxabs == nullptr) return false;
        const long bound = (long)FP32_EXACT_MAX >> (g.T < 31 ? g.T : 31);
        return (long)maxabs[gi] <= bound;
    } else {
        return false;
    }
}

// Float view of an int32 graph's buffers when they hold binary32 values.
struct FloatView {
    const float* src;
    float* dst;
};

// The change flag an item writes (null: none); false when the item is to be
// skipped because its graph reached the fixpoint at the previous squaring
// (early exit; uniform over the workgroup).
__device__ __forceinline__ bool step_flag(int* changed, const BatchItem& it, int early_stride,
                                          int*& flag) {
    flag = nullptr;
    if (changed == nullptr) return true;
    if (early_stride == 0) {
        flag = changed + it.graph;
        return true;
    }
    if (it.step >= 2 && changed[(it.step - 1) * early_stride + it.graph] == 0) return false;
    flag = changed + it.step * early_stride + it.graph;
    return true;
}

template <typename T, int SR>
__global__ __launch_bounds__(256) void grouped_step_kernel(const BatchGraph* __restrict__ graphs,
                                                            const BatchItem* __restrict__ items,
                                                            const int* __restrict__ maxabs,
                                                            int* __restrict__ changed,
                                                            int float_storage, int early_stride) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const BatchItem it = items[blockIdx.x];
    if (it.kind == BATCH_TILE_NONE) return;
    const BatchGraph g = graphs[it.graph];
    const bool odd = ((g.parity + it.step) & 1) != 0;  // squaring it.step writes buf[odd]
    const T* src = (const T*)(odd ? g.buf[0] : g.buf[1]);
    T* dst = (T*)(odd ? g.buf[1] : g.buf[0]);
    int* chg;
    if (!step_flag(changed, it, early_stride, chg)) return;
    TileArgs<T> a{g.n, g.n, g.n, src, g.ld, src, g.ld, src, g.ld, dst, g.ld, chg, nullptr};
    const bool narrow = graph_is_narrow<T>(g, maxabs, it.graph);
    if constexpr (std::is_same_v<T, int32_t>) {
        if (narrow && float_storage) {
            // the buffers hold binary32 values: the plain fp32 kernel, no conversions
            TileArgs<float> f{g.n, g.n, g.n, (const float*)src, g.ld, (const float*)src, g.ld,
                              (const float*)src, g.ld, (float*)dst, g.ld, chg, nullptr};
            if (it.kind == BATCH_TILE_128) GemmTile<CfgL, float, float, SR, true>::run(f, it.m0, it.n0, smem_raw);
            else GemmTile<CfgM, float, float, SR, true>::run(f, it.m0, it.n0, smem_raw);
            return;
        }
        if (narrow) {
            if (it.kind == BATCH_TILE_128) GemmTile<CfgL, T, float, SR, true>::run(a, it.m0, it.n0, smem_raw);
            else GemmTile<CfgM, T, float, SR, true>::run(a, it.m0, it.n0, smem_raw);
            return;
        }
    }
    if (it.kind == BATCH_TILE_128) GemmTile<CfgL, T, T, SR, true>::run(a, it.m0, it.n0, smem_raw);
    else GemmTile<CfgM, T, T, SR, true>::run(a, it.m0, it.n0, smem_raw);
}

static_assert(CfgL::NT == 256 && CfgM::NT == 256, "grouped kernel mixes both tile shapes");

// The same squaring step for the wave kinds: one 64-thread workgroup per tile.
template <typename T, int SR>
__global__ __launch_bounds__(64) void grouped_wave_step_kernel(const BatchGraph* __restrict__ graphs,
                                                                const BatchItem* __restrict__ items,
                                                                const int* __restrict__ maxabs,
                                                                int* __restrict__ changed,
                                                                int float_storage, int early_stride) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const BatchItem it = items[blockIdx.x];
    if (it.kind == BATCH_TILE_NONE) return;
    const BatchGraph g = graphs[it.graph];
    const bool odd = ((g.parity + it.step) & 1) != 0;  // squaring it.step writes buf[odd]
    const T* src = (const T*)(odd ? g.buf[0] : g.buf[1]);
    T* dst = (T*)(odd ? g.buf[1] : g.buf[0]);
    int* chg;
    if (!step_flag(changed, it, early_stride, chg)) return;
    TileArgs<T> a{g.n, g.n, g.n, src, g.ld, src, g.ld, src, g.ld, dst, g.ld, chg, nullptr};
    const bool narrow = graph_is_narrow<T>(g, maxabs, it.graph);
    if constexpr (std::is_same_v<T, int32_t>) {
        if (narrow && float_storage) {
            TileArgs<float> f{g.n, g.n, g.n, (const float*)src, g.ld, (const float*)src, g.ld,
                              (const float*)src, g.ld, (float*)dst, g.ld, chg, nullptr};
            if (it.kind == BATCH_TILE_W64) GemmTile<CfgW, float, float, SR, true>::run(f, it.m0, it.n0, smem_raw);
            else GemmTile<CfgS, float, float, SR, true>::run(f, it.m0, it.n0, smem_raw);
            return;
        }
        if (narrow) {
            if (it.kind == BATCH_TILE_W64) GemmTile<CfgW, T, float, SR, true>::run(a, it.m0, it.n0, smem_raw);
            else GemmTile<CfgS, T, float, SR, true>::run(a, it.m0, it.n0, smem_raw);
            return;
        }
    }
    if (it.kind == BATCH_TILE_W64) GemmTile<CfgW, T, T, SR, true>::run(a, it.m0, it.n0, smem_raw);
    else GemmTile<CfgS, T, T, SR, true>::run(a, it.m0, it.n0, smem_raw);
}

static_assert(CfgW::NT == 64 && CfgS::NT == 64, "wave kernel mixes both wave tile shapes");

// Direct-load step for graphs stored padded (np x np, absent beyond n): every
// 64x64 tile of the padded matrix is full, so the operands go from global
// memory straight into LDS (no staging registers, four waves per SIMD); the
// padding stays absent (a padded row or column only meets absent values).
// int32 graphs outside the binary32-exact range (rare) take the staged
// integer tile on the same padded matrix.
template <typename T, int SR>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(4))) void
grouped_direct_step_kernel(const BatchGraph* __restrict__ graphs, const BatchItem* __restrict__ items,
                           const int* __restrict__ maxabs, int* __restrict__ changed,
                           int float_storage, int early_stride) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const BatchItem it = items[blockIdx.x];
    if (it.kind == BATCH_TILE_NONE) return;
    const BatchGraph g = graphs[it.graph];
    const bool odd = ((g.parity + it.step) & 1) != 0;
    const T* src = (const T*)(odd ? g.buf[0] : g.buf[1]);
    T* dst = (T*)(odd ? g.buf[1] : g.buf[0]);
    int* chg;
    if (!step_flag(changed, it, early_stride, chg)) return;
    const int np = g.np;
    // The k loop stops at n rounded up to the k-block: the terms beyond it
    // pair an absent entry of the padding with anything and never win, and
    // skipping them removes most of the padding's work (the 4096-graph
    // workload: padded over useful terms 1.31 -> 1.20).
    const int kk = (g.n + CfgWD::BK - 1) / CfgWD::BK * CfgWD::BK;
    if (std::is_same_v<T, float> || (float_storage && graph_is_narrow<T>(g, maxabs, it.graph))) {
        TileArgs<float> f{np, np, kk, (const float*)src, np, (const float*)src, np,
                          (const float*)src, np, (float*)dst, np, chg, nullptr};
        switch (it.kind) {
            case BATCH_TILE_W64x32D: GemmTileDirect<CfgWD64x32, SR>::run(f, it.m0, it.n0, smem_raw); break;
            case BATCH_TILE_W32x64D: GemmTileDirect<CfgWD32x64, SR>::run(f, it.m0, it.n0, smem_raw); break;
            case BATCH_TILE_W32D: GemmTileDirect<CfgWD32, SR>::run(f, it.m0, it.n0, smem_raw); break;
            default: GemmTileDirect<CfgWD, SR>::run(f, it.m0, it.n0, smem_raw); break;
        }
        return;
    }
    if constexpr (std::is_same_v<T, int32_t>) {
        TileArgs<T> a{np, np, kk, src, np, src, np, src, np, dst, np, chg, nullptr};
        GemmTile<CfgW, T, T, SR, true>::run(a, it.m0, it.n0, smem_raw);
    }
}

hipError_t launch_grouped_step(int dt, const BatchGraph* graphs, const BatchItem* items,
                               int nitems, const int* maxabs, int* changed, hipStream_t s,
                               int family, bool float_storage, int early_stride) {
    if (nitems <= 0) return hipSuccess;
    const int fs = float_storage ? 1 : 0;
    if (family == 2) {
        const size_t lds = GemmTileDirect<CfgWD, BTAS_MIN_PLUS>::lds_bytes > CfgW::lds_bytes
                               ? GemmTileDirect<CfgWD, BTAS_MIN_PLUS>::lds_bytes : CfgW::lds_bytes;
        if (dt == BTAS_FLOAT32)
            hipLaunchKernelGGL((grouped_direct_step_kernel<float, BTAS_MIN_PLUS>), dim3(nitems),
                               dim3(64), lds, s, graphs, items, nullptr, changed, 0, early_stride);
        else
            hipLaunchKernelGGL((grouped_direct_step_kernel<int32_t, BTAS_MIN_PLUS>), dim3(nitems),
                               dim3(64), lds, s, graphs, items, maxabs, changed, fs, early_stride);
        return hipGetLastError();
    }
    if (family == 1) {
        const size_t lds = CfgW::lds_bytes > CfgS::lds_bytes ? CfgW::lds_bytes : CfgS::lds_bytes;
        if (dt == BTAS_FLOAT32)
            hipLaunchKernelGGL((grouped_wave_step_kernel<float, BTAS_MIN_PLUS>), dim3(nitems),
                               dim3(64), lds, s, graphs, items, nullptr, changed, 0, early_stride);
        else
            hipLaunchKernelGGL((grouped_wave_step_kernel<int32_t, BTAS_MIN_PLUS>), dim3(nitems),
                               dim3(64), lds, s, graphs, items, maxabs, changed, fs, early_stride);
        return hipGetLastError();
    }
    const size_t lds = CfgL::lds_bytes > CfgM::lds_bytes ? CfgL::lds_bytes : CfgM::lds_bytes;
    if (dt == BTAS_FLOAT32)
        hipLaunchKernelGGL((grouped_step_kernel<float, BTAS_MIN_PLUS>), dim3(nitems), dim3(256), lds,
                           s, graphs, items, nullptr, changed, 0, early_stride);
    else
        hipLaunchKernelGGL((grouped_step_kernel<int32_t, BTAS_MIN_PLUS>), dim3(nitems), dim3(256),
                           lds, s, graphs, items, maxabs, changed, fs, early_stride);
    return hipGetLastError();
}

// Job owning workgroup `b` (jobs sorted by first_block).
__device__ __forceinline__ int find_job(const BatchCopy* jobs, int njobs, int b) {
    int lo = 0, hi = njobs - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (jobs[mid].first_block <= b) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// ---- init: buf[parity] <- I (+) W, and max |finite w| per graph (int32) ----
// |x| of a finite int32 element (the absent value excluded), saturating.
__device__ __forceinline__ int abs_finite(int32_t w) {
    if (w == BTAS_I32_INF) return 0;
    return w < 0 ? (w == INT32_MIN ? INT32_MAX : -w) : w;
}

__device__ __forceinline__ void block_max_to(int* dst, int mx) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
        const int o = __shfl_xor(mx, off, 64);
        mx = o > mx ? o : mx;
    }
    if ((threadIdx.x & 63) == 0 && mx > 0) atomicMax(dst, mx);
}

// The three passes below work on quads: four consecutive columns of one row
// (one index division per quad; 16-byte loads and stores on the padded
// internal buffers, whose rows are multiples of 4), QB quads per thread per
// round with every load issued before any is used, so that each thread keeps
// several HBM reads in flight.
constexpr int QB = 4;

// int32, first pass of the float-storage mode: maxabs[graph] <- max |finite
// element of I (+) W|.
__global__ __launch_bounds__(256) void grouped_maxabs_kernel(const BatchGraph* __restrict__ graphs,
                                                              const BatchCopy* __restrict__ jobs,
                                                              int njobs, const int* __restrict__ block_job,
                                                              int* __restrict__ maxabs) {
    const BatchCopy jb = jobs[block_job != nullptr ? block_job[blockIdx.x] : find_job(jobs, njobs, blockIdx.x)];
    const int n = graphs[jb.graph].n;
    const int32_t* W = (const int32_t*)jb.ext;
    const int nq = (n + 3) / 4;
    const long total = (long)n * nq;
    const long stride = (long)jb.nblocks * blockDim.x;
    const bool vec = jb.ld_ext % 4 == 0 && (uintptr_t)W % 16 == 0;  // 16-byte row quads
    int mx = 0;
    // QB quads per thread per round, all loads issued before any is used
    for (long e0 = (long)(blockIdx.x - jb.first_block) * blockDim.x + threadIdx.x; e0 < total;
         e0 += QB * stride) {
        int32_t w[QB][4];
        long ii[QB], qq[QB];
#pragma unroll
        for (int b = 0; b < QB; ++b) {
            const long e = e0 + b * stride;
            ii[b] = -1;
            if (e < total) flat_to_rc(e, nq, total, ii[b], qq[b]);
            if (vec && ii[b] >= 0 && qq[b] * 4 + 3 < n) {
                const v4<int32_t> x = *reinterpret_cast<const v4<int32_t>*>(W + ii[b] * jb.ld_ext + qq[b] * 4);
#pragma unroll
                for (int u = 0; u < 4; ++u) w[b][u] = x[u];
                continue;
            }
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const long j = qq[b] * 4 + u;
                w[b][u] = (ii[b] >= 0 && j < n) ? W[ii[b] * jb.ld_ext + j] : BTAS_I32_INF;
            }
        }
#pragma unroll
        for (int b = 0; b < QB; ++b)
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                int32_t x = w[b][u];
                if (ii[b] == qq[b] * 4 + u && x > 0) x = 0;
                const int aw = abs_finite(x);
                mx = aw > mx ? aw : mx;
            }
    }
    block_max_to(maxabs + jb.graph, mx);
}

// float_storage (int32 only; maxabs already complete): graphs whose squarings
// stay in the binary32-exact range are written as binary32 values (absent ->
// +inf), so the squaring kernels read and write them without conversions.
// Otherwise (int32) maxabs[graph] is accumulated here.  Padded graphs (np > 0)
// get the absent value in rows and columns n..np-1, in both buffers.
template <typename T>
__global__ __launch_bounds__(256) void grouped_init_kernel(const BatchGraph* __restrict__ graphs,
                                                            const BatchCopy* __restrict__ jobs,
                                                            int njobs, const int* __restrict__ block_job,
                                                            int* __restrict__ maxabs, int float_storage) {
    const BatchCopy jb = jobs[block_job != nullptr ? block_job[blockIdx.x] : find_job(jobs, njobs, blockIdx.x)];
    const BatchGraph g = graphs[jb.graph];
    const int n = g.n;
    const T* W = (const T*)jb.ext;
    uint32_t* D = (uint32_t*)g.buf[g.parity & 1];
    uint32_t* D1 = (uint32_t*)g.buf[(g.parity + 1) & 1];
    bool as_float = false;
    if constexpr (std::is_same_v<T, int32_t>) as_float = float_storage && graph_is_narrow<T>(g, maxabs, jb.graph);
    const uint32_t absent = as_float || std::is_same_v<T, float>
                                ? __float_as_uint(Ring<BTAS_MIN_PLUS, float>::absent())
                                : (uint32_t)BTAS_I32_INF;
    // quads over the stored rows x columns: np x np when padded, else n x n
    // (the last quad of a row may reach into columns n..ld-1, which nothing reads)
    const int rows = g.np > 0 ? g.np : n;
    const int nq = ((g.np > 0 ? g.np : n) + 3) / 4;
    const long total = (long)rows * nq;
    const long stride = (long)jb.nblocks * blockDim.x;
    const bool vec = jb.ld_ext % 4 == 0 && (uintptr_t)W % 16 == 0;
    int mx = 0;
    for (long e0 = (long)(blockIdx.x - jb.first_block) * blockDim.x + threadIdx.x; e0 < total;
         e0 += QB * stride) {
        T w[QB][4];
        long ii[QB], qq[QB];
#pragma unroll
        for (int b = 0; b < QB; ++b) {
            const long e = e0 + b * stride;
            ii[b] = -1;
            if (e < total) flat_to_rc(e, nq, total, ii[b], qq[b]);
            if (vec && ii[b] >= 0 && ii[b] < n && qq[b] * 4 + 3 < n) {
                const v4<T> x = *reinterpret_cast<const v4<T>*>(W + ii[b] * jb.ld_ext + qq[b] * 4);
#pragma unroll
                for (int u = 0; u < 4; ++u) w[b][u] = x[u];
                continue;
            }
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const long j = qq[b] * 4 + u;
                w[b][u] = (ii[b] >= 0 && ii[b] < n && j < n) ? W[ii[b] * jb.ld_ext + j] : (T)0;
            }
        }
#pragma unroll
        for (int b = 0; b < QB; ++b) {
            if (ii[b] < 0) continue;
            const long i = ii[b];
            v4<uint32_t> out;
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const long j = qq[b] * 4 + u;
                uint32_t bits = absent;
                if (i < n && j < n) {
                    T x = w[b][u];
                    if (i == j && x > (T)0) x = (T)0;
                    if constexpr (std::is_same_v<T, int32_t>) {
                        if (as_float) {
                            bits = __float_as_uint(Conv<int32_t, float, BTAS_MIN_PLUS>::in(x));
                        } else {
                            bits = (uint32_t)x;
                            const int aw = abs_finite(x);
                            mx = aw > mx ? aw : mx;
                        }
                    } else {
                        bits = __float_as_uint(x);
                    }
                }
                out[u] = bits;
            }
            *reinterpret_cast<v4<uint32_t>*>(D + i * g.ld + qq[b] * 4) = out;
            // The padding of the other buffer too: a plan whose edge tiles stop
            // at n rounded up to 32 never writes rows or columns beyond that
            // there, and a staged 64-wide tile may read them.  (Its entries
            // below n are overwritten by the first squaring before any read.)
            if (g.np > 0 && (i >= n || qq[b] * 4 + 3 >= n))
                *reinterpret_cast<v4<uint32_t>*>(D1 + i * g.ld + qq[b] * 4) = out;
        }
    }
    if constexpr (std::is_same_v<T, int32_t>) {
        if (maxabs != nullptr && !float_storage) block_max_to(maxabs + jb.graph, mx);
    }
}

// ---- final copy: D_ext <- buf[(parity + T) & 1] ----
// float_maxabs (int32 float-storage mode, else null): graphs stored as
// binary32 are converted back to int32 (exact integers, +inf -> INF).
__global__ __launch_bounds__(256) void grouped_copy_out_kernel(const BatchGraph* __restrict__ graphs,
                                                                const BatchCopy* __restrict__ jobs,
                                                                int njobs, const int* __restrict__ block_job,
                                                                const int* __restrict__ float_maxabs) {
    const BatchCopy jb = jobs[block_job != nullptr ? block_job[blockIdx.x] : find_job(jobs, njobs, blockIdx.x)];
    const BatchGraph g = graphs[jb.graph];
    const int n = g.n;
    const uint32_t* S = (const uint32_t*)g.buf[(g.parity + g.T) & 1];
    uint32_t* D = (uint32_t*)const_cast<void*>(jb.ext);
    const int nq = (n + 3) / 4;
    const long total = (long)n * nq;
    const long stride = (long)jb.nblocks * blockDim.x;
    const bool from_float =
        float_maxabs != nullptr && graph_is_narrow<int32_t>(g, float_maxabs, jb.graph);
    const bool vec = jb.ld_ext % 4 == 0 && (uintptr_t)D % 16 == 0;
    for (long e0 = (long)(blockIdx.x - jb.first_block) * blockDim.x + threadIdx.x; e0 < total;
         e0 += QB * stride) {
        v4<uint32_t> x[QB];
        long ii[QB], qq[QB];
#pragma unroll
        for (int b = 0; b < QB; ++b) {
            const long e = e0 + b * stride;
            ii[b] = -1;
            if (e < total) {
                flat_to_rc(e, nq, total, ii[b], qq[b]);
                x[b] = *reinterpret_cast<const v4<uint32_t>*>(S + ii[b] * g.ld + qq[b] * 4);
            }
        }
#pragma unroll
        for (int b = 0; b < QB; ++b) {
            if (ii[b] < 0) continue;
            uint32_t* row = D + ii[b] * jb.ld_ext;
            v4<uint32_t> y;
#pragma unroll
            for (int u = 0; u < 4; ++u)
                y[u] = from_float ? (uint32_t)Conv<int32_t, float, BTAS_MIN_PLUS>::out(__uint_as_float(x[b][u]))
                                  : x[b][u];
            if (vec && qq[b] * 4 + 3 < n) {
                *reinterpret_cast<v4<uint32_t>*>(row + qq[b] * 4) = y;
                continue;
            }
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const long j = qq[b] * 4 + u;
                if (j < n) row[j] = y[u];
            }
        }
    }
}

// ---- served requests: densify a COO edge list into I (+) W ----
template <typename T>
__global__ __launch_bounds__(256) void fill_identity_kernel(T* D, int n, int ld) {
    const long total = (long)n * n;
    for (long e = (long)blockIdx.x * blockDim.x + threadIdx.x; e < total;
         e += (long)gridDim.x * blockDim.x) {
        long i, j;
        flat_to_rc(e, n, total, i, j);
        D[i * ld + j] = i == j ? (T)0 : Ring<BTAS_MIN_PLUS, T>::absent();
    }
}

__device__ __forceinline__ void atomic_min_elem(int32_t* p, int32_t v) { atomicMin(p, v); }

__device__ __forceinline__ void atomic_min_elem(float* p, float v) {
    unsigned* ip = reinterpret_cast<unsigned*>(p);
    unsigned old = *ip;
    while (v < __uint_as_float(old)) {
        const unsigned seen = atomicCAS(ip, old, __float_as_uint(v));
        if (seen == old) break;
        old = seen;
    }
}

// D[r][c] <- min(D[r][c], w) for every edge (duplicates keep the lightest).
// Indices were range-checked on the host.
template <typename T>
__global__ __launch_bounds__(256) void scatter_min_kernel(T* D, int ld, int nnz,
                                                           const int32_t* __restrict__ rows,
                                                           const int32_t* __restrict__ cols,
                                                           const T* __restrict__ w) {
    for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < nnz; e += gridDim.x * blockDim.x)
        atomic_min_elem(D + (long)rows[e] * ld + cols[e], w[e]);
}

hipError_t launch_densify(int dt, void* D, int n, int ld, int nnz, const int32_t* rows,
                          const int32_t* cols, const void* w, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    long blocks = ((long)n * n + 1023) / 1024;
    if (blocks > 16384) blocks = 16384;
    int eb = (nnz + 255) / 256;
    if (eb > 4096) eb = 4096;
    if (dt == BTAS_FLOAT32) {
        hipLaunchKernelGGL(fill_identity_kernel<float>, dim3((unsigned)blocks), dim3(256), 0, s,
                           (float*)D, n, ld);
        if (nnz > 0)
            hipLaunchKernelGGL(scatter_min_kernel<float>, dim3(eb), dim3(256), 0, s, (float*)D, ld,
                               nnz, rows, cols, (const float*)w);
    } else {
        hipLaunchKernelGGL(fill_identity_kernel<int32_t>, dim3((unsigned)blocks), dim3(256), 0, s,
                           (int32_t*)D, n, ld);
        if (nnz > 0)
            hipLaunchKernelGGL(scatter_min_kernel<int32_t>, dim3(eb), dim3(256), 0, s,
                               (int32_t*)D, ld, nnz, rows, cols, (const int32_t*)w);
    }
    return hipGetLastError();
}

template <typename T>
__global__ __launch_bounds__(LDS_SOLVE_NT) void batched_lds_solve_kernel(const BatchSmall* __restrict__ jobs,
                                                                         int early) {
    __shared__ __align__(16) LdsSolveBuffers<T> sm;
    const BatchSmall j = jobs[blockIdx.x];
    (void)lds_solve_graph<T>(j.n, (const T*)j.W, j.ldw, (T*)j.D, j.ldd, j.T, early, sm);
}

hipError_t launch_batched_lds_solve(int dt, const BatchSmall* jobs, int njobs, bool early,
                                    hipStream_t s) {
    if (njobs <= 0) return hipSuccess;
    if (dt == BTAS_FLOAT32)
        hipLaunchKernelGGL(batched_lds_solve_kernel<float>, dim3((unsigned)njobs), dim3(LDS_SOLVE_NT), 0,
                           s, jobs, early ? 1 : 0);
    else
        hipLaunchKernelGGL(batched_lds_solve_kernel<int32_t>, dim3((unsigned)njobs), dim3(LDS_SOLVE_NT),
                           0, s, jobs, early ? 1 : 0);
    return hipGetLastError();
}

__global__ void clear_ints_kernel(int* p, int count) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < count; i += gridDim.x * blockDim.x)
        p[i] = 0;
}

hipError_t launch_clear_ints(int* p, int count, hipStream_t s) {
    if (count <= 0) return hipSuccess;
    int blocks = (count + 255) / 256;
    if (blocks > 1024) blocks = 1024;
    hipLaunchKernelGGL(clear_ints_kernel, dim3(blocks), dim3(256), 0, s, p, count);
    return hipGetLastError();
}

hipError_t launch_grouped_maxabs(const BatchGraph* graphs, const BatchCopy* jobs, int njobs,
                                 int total_blocks, int* maxabs, hipStream_t s, const int* block_job) {
    if (njobs <= 0 || total_blocks <= 0) return hipSuccess;
    hipLaunchKernelGGL(grouped_maxabs_kernel, dim3(total_blocks), dim3(256), 0, s, graphs, jobs,
                       njobs, block_job, maxabs);
    return hipGetLastError();
}

hipError_t launch_grouped_init(int dt, const BatchGraph* graphs, const BatchCopy* jobs, int njobs,
                               int total_blocks, int* maxabs, hipStream_t s, bool float_storage,
                               const int* block_job) {
    if (njobs <= 0 || total_blocks <= 0) return hipSuccess;
    if (dt == BTAS_FLOAT32)
        hipLaunchKernelGGL(grouped_init_kernel<float>, dim3(total_blocks), dim3(256), 0, s, graphs,
                           jobs, njobs, block_job, nullptr, 0);
    else
        hipLaunchKernelGGL(grouped_init_kernel<int32_t>, dim3(total_blocks), dim3(256), 0, s,
                           graphs, jobs, njobs, block_job, maxabs, float_storage ? 1 : 0);
    return hipGetLastError();
}

hipError_t launch_grouped_copy_out(const BatchGraph* graphs, const BatchCopy* jobs, int njobs,
                                   int total_blocks, hipStream_t s, const int* float_maxabs,
                                   const int* block_job) {
    if (njobs <= 0 || total_blocks <= 0) return hipSuccess;
    hipLaunchKernelGGL(grouped_copy_out_kernel, dim3(total_blocks), dim3(256), 0, s, graphs, jobs,
                       njobs, block_job, float_maxabs);
    return hipGetLastError();
}

}  // namespace btas
