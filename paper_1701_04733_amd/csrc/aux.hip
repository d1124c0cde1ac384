// Small elementwise kernels around the squaring loop: D_0 = I (+) W, flag
// resets, the negative-cycle check, strided matrix copies and the optional
// domain scan.  All are O(n^2) and HBM-bound.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <type_traits>

#include "gemm_tile.h"
#include "kernels.h"
#include "semiring.h"
#include "flat_index.h"

namespace btas {

// D_0 = I (+) W (Sec. III starts the squaring from the adjacency matrix; the
// tropical identity puts 0 on the diagonal, so D_ii = min(W_ii, 0) for
// min-plus and max(W_ii, 0) for max-plus).
template <typename T, int SR>
__global__ __launch_bounds__(256) void apsp_init_kernel(int n, const T* W, long ldw, T* D,
                                                         long ldd, int* wide) {
    using R = Ring<SR, T>;
    const long total = (long)n * n;
    bool w_wide = false;
    for (long e = (long)blockIdx.x * blockDim.x + threadIdx.x; e < total;
         e += (long)gridDim.x * blockDim.x) {
        long i, j;
        flat_to_rc(e, n, total, i, j);
        T w = W[i * ldw + j];
        if (i == j && (SR == BTAS_MIN_PLUS ? w > (T)0 : w < (T)0)) w = (T)0;
        D[i * ldd + j] = w;
        if constexpr (std::is_same_v<T, int32_t>)
            w_wide |= w != R::absent() && (w > FP32_EXACT_MAX || w < -FP32_EXACT_MAX);
    }
    if (wide != nullptr && w_wide) *wide = 1;
}

static unsigned blocks_for(long total) {
    long b = (total + 1023) / 1024;
    if (b < 1) b = 1;
    if (b > 16384) b = 16384;
    return (unsigned)b;
}

template <int SR>
static hipError_t closure_init(int dt, int n, const void* W, long ldw, void* dst, long ldd,
                               int* wide, hipStream_t s) {
    if (n == 0) return hipSuccess;
    const unsigned g = blocks_for((long)n * n);
    if (dt == BTAS_FLOAT32)
        hipLaunchKernelGGL((apsp_init_kernel<float, SR>), dim3(g), dim3(256), 0, s, n,
                           (const float*)W, ldw, (float*)dst, ldd, nullptr);
    else
        hipLaunchKernelGGL((apsp_init_kernel<int32_t, SR>), dim3(g), dim3(256), 0, s, n,
                           (const int32_t*)W, ldw, (int32_t*)dst, ldd, wide);
    return hipGetLastError();
}

hipError_t launch_apsp_init(int dt, int n, const void* W, long ldw, void* dst, long ldd,
                            int* wide, hipStream_t s) {
    return closure_init<BTAS_MIN_PLUS>(dt, n, W, ldw, dst, ldd, wide, s);
}

hipError_t launch_closure_init(int sr, int dt, int n, const void* W, long ldw, void* dst, long ldd,
                               int* wide, hipStream_t s) {
    return sr == BTAS_MIN_PLUS ? closure_init<BTAS_MIN_PLUS>(dt, n, W, ldw, dst, ldd, wide, s)
                               : closure_init<BTAS_MAX_PLUS>(dt, n, W, ldw, dst, ldd, wide, s);
}

template <int SR>
__global__ __launch_bounds__(256) void range_scan_kernel(int m, int n, const int32_t* X, long ld,
                                                          int* flag) {
    const long total = (long)m * n;
    bool wide = false;
    for (long e = (long)blockIdx.x * blockDim.x + threadIdx.x; e < total;
         e += (long)gridDim.x * blockDim.x) {
        long i, j;
        flat_to_rc(e, n, total, i, j);
        const int32_t x = X[i * ld + j];
        wide |= x != Ring<SR, int32_t>::absent() && (x > FP32_EXACT_MAX || x < -FP32_EXACT_MAX);
    }
    if (wide) *flag = 1;
}

hipError_t launch_range_scan(int sr, int m, int n, const void* X, long ld, int* flag,
                             hipStream_t s) {
    if (m == 0 || n == 0) return hipSuccess;
    const dim3 g(blocks_for((long)m * n)), b(256);
    if (sr == BTAS_MIN_PLUS)
        hipLaunchKernelGGL(range_scan_kernel<BTAS_MIN_PLUS>, g, b, 0, s, m, n, (const int32_t*)X,
                           ld, flag);
    else
        hipLaunchKernelGGL(range_scan_kernel<BTAS_MAX_PLUS>, g, b, 0, s, m, n, (const int32_t*)X,
                           ld, flag);
    return hipGetLastError();
}

__global__ __launch_bounds__(256) void zero_words_kernel(uint64_t* p, size_t words) {
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < words;
         i += (size_t)gridDim.x * blockDim.x)
        p[i] = 0;
}

hipError_t launch_zero_words(void* p, size_t words, hipStream_t s) {
    if (words == 0) return hipSuccess;
    const size_t blocks = std::min<size_t>((words + 255) / 256, 4096);
    hipLaunchKernelGGL(zero_words_kernel, dim3((unsigned)blocks), dim3(256), 0, s,
                       static_cast<uint64_t*>(p), words);
    return hipGetLastError();
}

__global__ void clear_flags_kernel(int* flag, int count) {
    for (int i = threadIdx.x; i < count; i += blockDim.x) flag[i] = 0;
}

hipError_t launch_clear_flags(int* flag, int count, hipStream_t s) {
    hipLaunchKernelGGL(clear_flags_kernel, dim3(1), dim3(256), 0, s, flag, count);
    return hipGetLastError();
}

// flag <- 1 if some D_ii is past 0 on the semiring's improving side (min-plus
// < 0: a negative cycle; max-plus > 0: a positive cycle).
template <typename T, int SR>
__global__ __launch_bounds__(256) void diag_check_kernel(int n, const T* D, long ldd, int* flag) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        const T d = D[(long)i * ldd + i];
        if (SR == BTAS_MIN_PLUS ? d < (T)0 : d > (T)0) *flag = 1;
    }
}

template <int SR>
static hipError_t diag_check(int dt, int n, const void* D, long ldd, int* flag, hipStream_t s) {
    if (n == 0) return hipSuccess;
    const unsigned g = (unsigned)((n + 255) / 256);
    if (dt == BTAS_FLOAT32)
        hipLaunchKernelGGL((diag_check_kernel<float, SR>), dim3(g), dim3(256), 0, s, n,
                           (const float*)D, ldd, flag);
    else
        hipLaunchKernelGGL((diag_check_kernel<int32_t, SR>), dim3(g), dim3(256), 0, s, n,
                           (const int32_t*)D, ldd, flag);
    return hipGetLastError();
}

hipError_t launch_neg_diag_check(int dt, int n, const void* D, long ldd, int* flag,
                                 hipStream_t s) {
    return diag_check<BTAS_MIN_PLUS>(dt, n, D, ldd, flag, s);
}

hipError_t launch_diag_check(int sr, int dt, int n, const void* D, long ldd, int* flag,
                             hipStream_t s) {
    return sr == BTAS_MIN_PLUS ? diag_check<BTAS_MIN_PLUS>(dt, n, D, ldd, flag, s)
                               : diag_check<BTAS_MAX_PLUS>(dt, n, D, ldd, flag, s);
}

__global__ __launch_bounds__(256) void copy_matrix_kernel(int m, int n, const uint32_t* src,
                                                           long lds, uint32_t* dst, long ldd) {
    const long total = (long)m * n;
    for (long e = (long)blockIdx.x * blockDim.x + threadIdx.x; e < total;
         e += (long)gridDim.x * blockDim.x) {
        long i, j;
        flat_to_rc(e, n, total, i, j);
        dst[i * ldd + j] = src[i * lds + j];
    }
}

hipError_t launch_copy_matrix(int m, int n, const void* src, long lds, void* dst, long ldd,
                              hipStream_t s) {
    if (m == 0 || n == 0) return hipSuccess;
    hipLaunchKernelGGL(copy_matrix_kernel, dim3(blocks_for((long)m * n)), dim3(256), 0, s, m, n,
                       (const uint32_t*)src, lds, (uint32_t*)dst, ldd);
    return hipGetLastError();
}

// Legal (.) operands: the semiring's absent value or a finite value within
// +-BTAS_I32_FINITE_MAX (int32); anything but NaN and the other infinity
// (float32).
template <typename T, int SR>
__device__ __forceinline__ bool operand_ok(T x);

template <>
__device__ __forceinline__ bool operand_ok<int32_t, BTAS_MIN_PLUS>(int32_t x) {
    return x == BTAS_I32_INF || (x >= -BTAS_I32_FINITE_MAX && x <= BTAS_I32_FINITE_MAX);
}
template <>
__device__ __forceinline__ bool operand_ok<int32_t, BTAS_MAX_PLUS>(int32_t x) {
    return x == BTAS_I32_NEG_INF || (x >= -BTAS_I32_FINITE_MAX && x <= BTAS_I32_FINITE_MAX);
}
template <>
__device__ __forceinline__ bool operand_ok<float, BTAS_MIN_PLUS>(float x) {
    return !(x != x) && x != -__builtin_inff();
}
template <>
__device__ __forceinline__ bool operand_ok<float, BTAS_MAX_PLUS>(float x) {
    return !(x != x) && x != __builtin_inff();
}

template <typename T, int SR>
__global__ __launch_bounds__(256) void domain_scan_kernel(int m, int n, const T* X, long ld,
                                                           int* flag) {
    const long total = (long)m * n;
    bool bad = false;
    for (long e = (long)blockIdx.x * blockDim.x + threadIdx.x; e < total;
         e += (long)gridDim.x * blockDim.x) {
        long i, j;
        flat_to_rc(e, n, total, i, j);
        bad |= !operand_ok<T, SR>(X[i * ld + j]);
    }
    if (bad) *flag = 1;
}

hipError_t launch_domain_scan(int sr, int dt, int m, int n, const void* X, long ld, int* flag,
                              hipStream_t s) {
    if (m == 0 || n == 0) return hipSuccess;
    const dim3 g(blocks_for((long)m * n)), b(256);
    if (dt == BTAS_FLOAT32) {
        if (sr == BTAS_MIN_PLUS)
            hipLaunchKernelGGL((domain_scan_kernel<float, 0>), g, b, 0, s, m, n, (const float*)X,
                               ld, flag);
        else
            hipLaunchKernelGGL((domain_scan_kernel<float, 1>), g, b, 0, s, m, n, (const float*)X,
                               ld, flag);
    } else {
        if (sr == BTAS_MIN_PLUS)
            hipLaunchKernelGGL((domain_scan_kernel<int32_t, 0>), g, b, 0, s, m, n,
                               (const int32_t*)X, ld, flag);
        else
            hipLaunchKernelGGL((domain_scan_kernel<int32_t, 1>), g, b, 0, s, m, n,
                               (const int32_t*)X, ld, flag);
    }
    return hipGetLastError();
}

}  // namespace btas
