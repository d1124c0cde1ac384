// Sparse-aware squarings of APSP (min-plus).
//
// A squaring E = D (+) D (.) D (Sec. III) of a sparse graph's distance matrix
// has few finite terms: while D_t has r_i finite entries in row i, the
// product's terms are sum_i sum_{k finite in row i} r_k, far below n^3 for
// the first squarings of a graph with small out-degree (the first input of a
// degree-16 graph with n = 16384 is 99.9% absent).  Such a step runs here
// as a row-by-row sparse product into a dense row accumulator in LDS:
//   1. count the finite entries of every row (and their total);
//   2. compress D into CSR (column order kept) and sum the step's term count;
//   3. per row i: acc = D_i,:, then acc_j <- min(acc_j, D_ik + D_kj) for
//      every finite D_ik and finite D_kj, then store the row and the flags.
// The host decides between this and the dense product from the counts.  The
// result is the same min of the same rounded terms as the dense step
// (absent terms never win a min), so it is bit-identical.
#include <hip/hip_runtime.h>

#include <type_traits>

#include "gemm_tile.h"
#include "kernels.h"
#include "semiring.h"

namespace btas {

namespace {

constexpr int SP_NT = 256;

template <typename T>
__device__ __forceinline__ bool present(T x) {
    return x != Ring<BTAS_MIN_PLUS, T>::absent();
}

// Sum over the workgroup; every thread gets the total.
__device__ __forceinline__ long long block_sum(long long v, long long* red) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
    const int w = threadIdx.x / 64;
    __syncthreads();
    if ((threadIdx.x & 63) == 0) red[w] = v;
    __syncthreads();
    long long t = 0;
    for (int q = 0; q < SP_NT / 64; ++q) t += red[q];
    return t;
}

// rownnz[i] = finite entries of row i (off the diagonal if skip_diag);
// counters[0] += their total.
template <typename T>
__global__ __launch_bounds__(SP_NT) void sp_count_kernel(int n, const T* D, long ld, int* rownnz,
                                                        unsigned long long* counters, int skip_diag) {
    __shared__ long long red[SP_NT / 64];
    const int i = blockIdx.x;
    const T* row = D + (long)i * ld;
    long long c = 0;
    for (int j = threadIdx.x; j < n; j += SP_NT) c += present(row[j]) && !(skip_diag && j == i) ? 1 : 0;
    c = block_sum(c, red);
    if (threadIdx.x == 0) {
        rownnz[i] = (int)c;
        atomicAdd(counters, (unsigned long long)c);
    }
}

// rowptr = exclusive prefix sum of rownnz (n + 1 entries), one workgroup.
__global__ __launch_bounds__(1024) void sp_scan_kernel(int n, const int* rownnz, int* rowptr) {
    __shared__ int part[1024];
    const int per = (n + 1023) / 1024;
    const int b = threadIdx.x * per, e = min(n, b + per);
    int s = 0;
    for (int i = b; i < e; ++i) s += rownnz[i];
    part[threadIdx.x] = s;
    __syncthreads();
    for (int o = 1; o < 1024; o <<= 1) {  // inclusive scan of the partial sums
        const int v = threadIdx.x >= o ? part[threadIdx.x - o] : 0;
        __syncthreads();
        part[threadIdx.x] += v;
        __syncthreads();
    }
    int run = part[threadIdx.x] - s;
    for (int i = b; i < e; ++i) {
        rowptr[i] = run;
        run += rownnz[i];
    }
    if (threadIdx.x == 1023) rowptr[n] = part[1023];
}

// Row i's finite entries, in column order, to cols/vals at rowptr[i];
// counters[1] += sum over them of rownnz[column] (the step's term count).
template <typename T>
__global__ __launch_bounds__(SP_NT) void sp_compact_kernel(int n, const T* D, long ld, const int* rownnz,
                                                          const int* rowptr, int* cols, T* vals,
                                                          unsigned long long* counters, int skip_diag) {
    __shared__ int wave_count[SP_NT / 64];
    __shared__ long long red[SP_NT / 64];
    const int i = blockIdx.x;
    const T* row = D + (long)i * ld;
    const int lane = threadIdx.x & 63, w = threadIdx.x / 64;
    int base = rowptr[i];
    long long terms = 0;
    for (int j0 = 0; j0 < n; j0 += SP_NT) {
        const int j = j0 + threadIdx.x;
        const T x = j < n ? row[j] : Ring<BTAS_MIN_PLUS, T>::absent();
        const bool f = j < n && present(x) && !(skip_diag && j == i);
        const unsigned long long mask = __ballot(f);
        const int before = __popcll(mask & ((1ull << lane) - 1));
        __syncthreads();  // wave_count of the previous chunk is consumed
        if (lane == 0) wave_count[w] = __popcll(mask);
        __syncthreads();
        int off = base;
        for (int q = 0; q < w; ++q) off += wave_count[q];
        if (f) {
            cols[off + before] = j;
            vals[off + before] = x;
            terms += rownnz[j];
        }
        for (int q = 0; q < SP_NT / 64; ++q) base += wave_count[q];
    }
    terms = block_sum(terms, red);
    if (threadIdx.x == 0) atomicAdd(counters + 1, (unsigned long long)terms);
}

template <typename T>
__device__ __forceinline__ void lds_min(T* p, T v) {
    __hip_atomic_fetch_min(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

// E_i,: = D_i,: (+) (+)_k D_ik (.) D_k,:  over the finite entries only; one
// workgroup per row, the row accumulated in LDS (n entries).
template <typename T>
__global__ __launch_bounds__(SP_NT) void sp_square_kernel(int n, const T* D, long ld, T* E, long lde,
                                                         const int* rowptr, const int* cols,
                                                         const T* vals, int* changed, int* wide_out) {
    using R = Ring<BTAS_MIN_PLUS, T>;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    T* acc = reinterpret_cast<T*>(smem_raw);
    const int i = blockIdx.x;
    const T* drow = D + (long)i * ld;
    for (int j = threadIdx.x; j < n; j += SP_NT) acc[j] = drow[j];
    __syncthreads();
    const int lane = threadIdx.x & 63, w = threadIdx.x / 64;
    const int e1 = rowptr[i + 1];
    for (int e = rowptr[i] + w; e < e1; e += SP_NT / 64) {
        const int k = cols[e];
        const T a = vals[e];
        const int f1 = rowptr[k + 1];
        for (int f = rowptr[k] + lane; f < f1; f += 64) lds_min(&acc[cols[f]], R::mul(a, vals[f]));
    }
    __syncthreads();
    bool diff = false, wide = false;
    T* erow = E + (long)i * lde;
    for (int j = threadIdx.x; j < n; j += SP_NT) {
        const T v = acc[j];
        erow[j] = v;
        diff |= bits_of(v) != bits_of(drow[j]);
        if constexpr (std::is_same_v<T, int32_t>)
            wide |= v != R::absent() && (v > FP32_EXACT_MAX || v < -FP32_EXACT_MAX);
    }
    if (changed != nullptr && __any(diff) && lane == 0) *changed = 1;
    if (wide_out != nullptr && __any(wide) && lane == 0) *wide_out = 1;
}

// Successors from the CSR of W without its diagonal: S_ij = the first u (in
// column order, so the smallest) of row i's edges minimising W_iu (.) D_uj,
// -1 if every such term is absent; S_ii = i.  One workgroup per row, each
// thread four consecutive columns per round.
template <typename T>
__global__ __launch_bounds__(SP_NT) void sp_successor_kernel(int n, const int* rowptr, const int* cols,
                                                            const T* vals, const T* D, long ldd,
                                                            int32_t* S, long lds) {
    using R = Ring<BTAS_MIN_PLUS, T>;
    const int i = blockIdx.x;
    const int e0 = rowptr[i], e1 = rowptr[i + 1];
    int32_t* srow = S + (long)i * lds;
    for (int j0 = threadIdx.x * 4; j0 < n; j0 += SP_NT * 4) {
        T best[4];
        int arg[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            best[q] = R::absent();
            arg[q] = -1;
        }
        for (int e = e0; e < e1; ++e) {
            const int u = cols[e];
            const T w = vals[e];
            const T* drow = D + (long)u * ldd;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                if (j0 + q >= n) break;
                const T d = drow[j0 + q];
                if (!present(d)) continue;  // an absent D_uj never wins
                const T t = R::mul(w, d);
                if (t < best[q]) {
                    best[q] = t;
                    arg[q] = u;
                }
            }
        }
#pragma unroll
        for (int q = 0; q < 4; ++q)
            if (j0 + q < n) srow[j0 + q] = j0 + q == i ? i : arg[q];
    }
}

}  // namespace

size_t sparse_step_lds_bytes(int n) { return (size_t)n * 4; }

hipError_t launch_sparse_count(int dt, int n, const void* D, long ld, int* rownnz,
                               unsigned long long* counters, hipStream_t s, bool skip_diag) {
    const int sd = skip_diag ? 1 : 0;
    if (dt == BTAS_FLOAT32)
        hipLaunchKernelGGL(sp_count_kernel<float>, dim3(n), dim3(SP_NT), 0, s, n, (const float*)D, ld,
                           rownnz, counters, sd);
    else
        hipLaunchKernelGGL(sp_count_kernel<int32_t>, dim3(n), dim3(SP_NT), 0, s, n, (const int32_t*)D,
                           ld, rownnz, counters, sd);
    return hipGetLastError();
}

hipError_t launch_sparse_build(int dt, int n, const void* D, long ld, const int* rownnz, int* rowptr,
                               int* cols, void* vals, unsigned long long* counters, hipStream_t s,
                               bool skip_diag) {
    const int sd = skip_diag ? 1 : 0;
    hipLaunchKernelGGL(sp_scan_kernel, dim3(1), dim3(1024), 0, s, n, rownnz, rowptr);
    if (dt == BTAS_FLOAT32)
        hipLaunchKernelGGL(sp_compact_kernel<float>, dim3(n), dim3(SP_NT), 0, s, n, (const float*)D, ld,
                           rownnz, rowptr, cols, (float*)vals, counters, sd);
    else
        hipLaunchKernelGGL(sp_compact_kernel<int32_t>, dim3(n), dim3(SP_NT), 0, s, n, (const int32_t*)D,
                           ld, rownnz, rowptr, cols, (int32_t*)vals, counters, sd);
    return hipGetLastError();
}

hipError_t launch_sparse_successors(int dt, int n, const int* rowptr, const int* cols,
                                    const void* vals, const void* D, long ldd, int32_t* S, long lds,
                                    hipStream_t s) {
    if (dt == BTAS_FLOAT32)
        hipLaunchKernelGGL(sp_successor_kernel<float>, dim3(n), dim3(SP_NT), 0, s, n, rowptr, cols,
                           (const float*)vals, (const float*)D, ldd, S, lds);
    else
        hipLaunchKernelGGL(sp_successor_kernel<int32_t>, dim3(n), dim3(SP_NT), 0, s, n, rowptr, cols,
                           (const int32_t*)vals, (const int32_t*)D, ldd, S, lds);
    return hipGetLastError();
}

hipError_t launch_sparse_square(int dt, int n, const void* D, long ld, void* E, long lde,
                                const int* rowptr, const int* cols, const void* vals, int* changed,
                                int* wide_out, hipStream_t s) {
    const size_t lds = sparse_step_lds_bytes(n);
    if (dt == BTAS_FLOAT32)
        hipLaunchKernelGGL(sp_square_kernel<float>, dim3(n), dim3(SP_NT), lds, s, n, (const float*)D, ld,
                           (float*)E, lde, rowptr, cols, (const float*)vals, changed, wide_out);
    else
        hipLaunchKernelGGL(sp_square_kernel<int32_t>, dim3(n), dim3(SP_NT), lds, s, n,
                           (const int32_t*)D, ld, (int32_t*)E, lde, rowptr, cols, (const int32_t*)vals,
                           changed, wide_out);
    return hipGetLastError();
}

}  // namespace btas
