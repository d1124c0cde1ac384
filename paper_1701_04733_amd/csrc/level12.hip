// Tropical level-2 (gemv) and level-1 (vadd, vmul, axpy, dot) kernels.
//
// "Standard vector and matrix operations" of the library (Abstract; Sec. III)
// over the semirings of Sec. I, eqs. (1)-(4).  All of these are HBM-bound
// (at most one (.) and one (+) per element loaded), so the design goal is
// coalesced 128-bit streaming: one wave per output row for gemv with the
// vector x re-read from cache, grid-stride elementwise loops for level 1 and
// a deterministic two-pass reduction for dot (min/max are exact, so the
// reduction order never changes the bits).
#include <hip/hip_runtime.h>

#include <algorithm>

#include "kernels.h"
#include "semiring.h"

namespace btas {

template <typename T>
using v4 = T __attribute__((ext_vector_type(4)));

template <typename T, int SR>
__device__ __forceinline__ T wave_reduce(T v) {
    using R = Ring<SR, T>;
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v = R::add(v, __shfl_xor(v, off, 64));
    return v;
}

// ---------------------------------------------------------------- gemv ---
// One wave per row of A: y_i <- y_i (+) (+)_j a_ij (.) x_j.
template <typename T, int SR, bool VEC>
__global__ __launch_bounds__(256) void tropical_gemv_kernel(int m, int n,
                                                             const T* __restrict__ A, long lda,
                                                             const T* __restrict__ x, long incx,
                                                             T* __restrict__ y, long incy) {
    using R = Ring<SR, T>;
    const int lane = threadIdx.x & 63;
    const long row = (long)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (row >= m) return;
    const T* a = A + row * lda;
    T acc = R::absent();
    int j0 = 0;
    if (VEC) {
        const int nv = n / 4;
        const v4<T>* a4 = reinterpret_cast<const v4<T>*>(a);
        const v4<T>* x4 = reinterpret_cast<const v4<T>*>(x);
        for (int v = lane; v < nv; v += 64) {
            const v4<T> av = __builtin_nontemporal_load(a4 + v);
            const v4<T> xv = x4[v];
            acc = R::add3(acc, R::mul(av[0], xv[0]), R::mul(av[1], xv[1]));
            acc = R::add3(acc, R::mul(av[2], xv[2]), R::mul(av[3], xv[3]));
        }
        j0 = nv * 4;
    }
    for (int j = j0 + lane; j < n; j += 64) acc = R::add(acc, R::mul(a[j], x[(long)j * incx]));
    acc = wave_reduce<T, SR>(acc);
    if (lane == 0) y[row * incy] = R::add(y[row * incy], R::finish(acc));
}

template <typename T, int SR>
static hipError_t gemv_typed(int m, int n, const void* A, long lda, const void* x, long incx,
                             void* y, long incy, hipStream_t s) {
    if (m == 0) return hipSuccess;
    const bool vec = incx == 1 && lda % 4 == 0 && (((uintptr_t)A | (uintptr_t)x) % 16 == 0);
    dim3 grid((unsigned)((m + 3) / 4)), block(256);
    if (vec)
        hipLaunchKernelGGL((tropical_gemv_kernel<T, SR, true>), grid, block, 0, s, m, n,
                           (const T*)A, lda, (const T*)x, incx, (T*)y, incy);
    else
        hipLaunchKernelGGL((tropical_gemv_kernel<T, SR, false>), grid, block, 0, s, m, n,
                           (const T*)A, lda, (const T*)x, incx, (T*)y, incy);
    return hipGetLastError();
}

hipError_t launch_gemv(int sr, int dt, int m, int n, const void* A, long lda, const void* x,
                       long incx, void* y, long incy, hipStream_t s) {
    if (dt == BTAS_FLOAT32)
        return sr == BTAS_MIN_PLUS
                   ? gemv_typed<float, BTAS_MIN_PLUS>(m, n, A, lda, x, incx, y, incy, s)
                   : gemv_typed<float, BTAS_MAX_PLUS>(m, n, A, lda, x, incx, y, incy, s);
    return sr == BTAS_MIN_PLUS
               ? gemv_typed<int32_t, BTAS_MIN_PLUS>(m, n, A, lda, x, incx, y, incy, s)
               : gemv_typed<int32_t, BTAS_MAX_PLUS>(m, n, A, lda, x, incx, y, incy, s);
}

// ------------------------------------------------------------- level 1 ---
static inline unsigned grid_for(long n, int per_thread) {
    long blocks = (n + 256L * per_thread - 1) / (256L * per_thread);
    if (blocks < 1) blocks = 1;
    if (blocks > 8192) blocks = 8192;
    return (unsigned)blocks;
}

// Streaming kernels over 16-byte vectors: one vector per thread (the loops
// still stride for longer vectors).  Measured on 2^26-element fp32 vectors:
// a grid capped at 8192 workgroups, eight vectors per thread, moved
// 6.6 TB/s for two loads and a store; one vector per thread 7.6 TB/s, while
// more loads in flight per thread (two or four vectors an iteration) were
// slower (5.1-5.9 TB/s).
static inline unsigned grid_one(long nv) {
    long blocks = (nv + 255) / 256;
    if (blocks < 1) blocks = 1;
    if (blocks > (1L << 20)) blocks = 1L << 20;
    return (unsigned)blocks;
}

template <typename T, int SR, int OP>
__global__ __launch_bounds__(256) void tropical_vec_binary_kernel(long n, const T* x, long incx,
                                                                   const T* y, long incy, T* z,
                                                                   long incz) {
    using R = Ring<SR, T>;
    for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (long)gridDim.x * blockDim.x) {
        const T a = x[i * incx], b = y[i * incy];
        z[i * incz] = OP == 0 ? R::add(a, b) : R::finish(R::mul(a, b));
    }
}

template <typename T, int SR, int OP>
__global__ __launch_bounds__(256) void tropical_vec_binary_v4_kernel(long nv, const v4<T>* x,
                                                                      const v4<T>* y,
                                                                      v4<T>* z) {
    using R = Ring<SR, T>;
    for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < nv;
         i += (long)gridDim.x * blockDim.x) {
        const v4<T> a = __builtin_nontemporal_load(x + i), b = __builtin_nontemporal_load(y + i);
        v4<T> r;
#pragma unroll
        for (int e = 0; e < 4; ++e) r[e] = OP == 0 ? R::add(a[e], b[e]) : R::finish(R::mul(a[e], b[e]));
        __builtin_nontemporal_store(r, z + i);
    }
}

template <typename T, int SR, int OP>
static hipError_t vec_binary_typed(long n, const void* x, long incx, const void* y, long incy,
                                   void* z, long incz, hipStream_t s) {
    if (n == 0) return hipSuccess;
    const bool vec = incx == 1 && incy == 1 && incz == 1 &&
                     (((uintptr_t)x | (uintptr_t)y | (uintptr_t)z) % 16 == 0);
    long head = 0;
    if (vec) {
        const long nv = n / 4;
        if (nv > 0)
            hipLaunchKernelGGL((tropical_vec_binary_v4_kernel<T, SR, OP>), dim3(grid_one(nv)),
                               dim3(256), 0, s, nv, (const v4<T>*)x, (const v4<T>*)y,
                               (v4<T>*)z);
        head = nv * 4;
    }
    if (head < n)
        hipLaunchKernelGGL((tropical_vec_binary_kernel<T, SR, OP>), dim3(grid_for(n - head, 4)),
                           dim3(256), 0, s, n - head, (const T*)x + head * incx, incx,
                           (const T*)y + head * incy, incy, (T*)z + head * incz, incz);
    return hipGetLastError();
}

hipError_t launch_vec_binary(int op, int sr, int dt, int n, const void* x, long incx,
                             const void* y, long incy, void* z, long incz, hipStream_t s) {
#define BTAS_VB(T, SRV, OPV) vec_binary_typed<T, SRV, OPV>(n, x, incx, y, incy, z, incz, s)
    if (dt == BTAS_FLOAT32) {
        if (sr == BTAS_MIN_PLUS) return op == 0 ? BTAS_VB(float, 0, 0) : BTAS_VB(float, 0, 1);
        return op == 0 ? BTAS_VB(float, 1, 0) : BTAS_VB(float, 1, 1);
    }
    if (sr == BTAS_MIN_PLUS) return op == 0 ? BTAS_VB(int32_t, 0, 0) : BTAS_VB(int32_t, 0, 1);
    return op == 0 ? BTAS_VB(int32_t, 1, 0) : BTAS_VB(int32_t, 1, 1);
#undef BTAS_VB
}

template <typename T, int SR>
__global__ __launch_bounds__(256) void tropical_axpy_kernel(long n, T alpha, const T* x,
                                                             long incx, T* y, long incy) {
    using R = Ring<SR, T>;
    for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (long)gridDim.x * blockDim.x)
        y[i * incy] = R::add(y[i * incy], R::finish(R::mul(alpha, x[i * incx])));
}

// Unit strides, 16-byte aligned: 128-bit non-temporal accesses, one vector
// per thread (grid_one); the n % 4 tail elements go to workgroup 0.
template <typename T, int SR>
__global__ __launch_bounds__(256) void tropical_axpy_v4_kernel(long n, T alpha, const T* x, T* y) {
    using R = Ring<SR, T>;
    const long nv = n / 4, stride = (long)gridDim.x * blockDim.x;
    const v4<T>* x4 = reinterpret_cast<const v4<T>*>(x);
    v4<T>* y4 = reinterpret_cast<v4<T>*>(y);
    for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < nv; i += stride) {
        const v4<T> a = __builtin_nontemporal_load(x4 + i), b = __builtin_nontemporal_load(y4 + i);
        v4<T> r;
#pragma unroll
        for (int e = 0; e < 4; ++e) r[e] = R::add(b[e], R::finish(R::mul(alpha, a[e])));
        __builtin_nontemporal_store(r, y4 + i);
    }
    if (blockIdx.x == 0 && threadIdx.x < n - nv * 4) {
        const long i = nv * 4 + threadIdx.x;
        y[i] = R::add(y[i], R::finish(R::mul(alpha, x[i])));
    }
}

template <typename T, int SR>
static void axpy_typed(long n, T alpha, const void* x, long incx, void* y, long incy,
                       hipStream_t s) {
    const bool vec = incx == 1 && incy == 1 && (((uintptr_t)x | (uintptr_t)y) % 16 == 0);
    if (vec)
        hipLaunchKernelGGL((tropical_axpy_v4_kernel<T, SR>), dim3(grid_one(n / 4)),
                           dim3(256), 0, s, n, alpha, (const T*)x, (T*)y);
    else
        hipLaunchKernelGGL((tropical_axpy_kernel<T, SR>), dim3(grid_for(n, 4)), dim3(256), 0, s, n,
                           alpha, (const T*)x, incx, (T*)y, incy);
}

hipError_t launch_axpy(int sr, int dt, int n, uint32_t alpha_bits, const void* x, long incx,
                       void* y, long incy, hipStream_t s) {
    if (n == 0) return hipSuccess;
    if (dt == BTAS_FLOAT32) {
        const float a = __builtin_bit_cast(float, alpha_bits);
        if (sr == BTAS_MIN_PLUS) axpy_typed<float, 0>(n, a, x, incx, y, incy, s);
        else axpy_typed<float, 1>(n, a, x, incx, y, incy, s);
    } else {
        const int32_t a = (int32_t)alpha_bits;
        if (sr == BTAS_MIN_PLUS) axpy_typed<int32_t, 0>(n, a, x, incx, y, incy, s);
        else axpy_typed<int32_t, 1>(n, a, x, incx, y, incy, s);
    }
    return hipGetLastError();
}

// ---------------------------------------------------------------- dot ---
static constexpr int DOT_MAX_BLOCKS = 8192;

int dot_partials_needed(int /*n*/) { return DOT_MAX_BLOCKS; }

template <typename T, int SR>
__global__ __launch_bounds__(256) void tropical_dot_partial_kernel(long n, const T* x, long incx,
                                                                    const T* y, long incy,
                                                                    T* partials) {
    using R = Ring<SR, T>;
    __shared__ T red[4];
    T acc = R::absent();
    for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (long)gridDim.x * blockDim.x)
        acc = R::add(acc, R::mul(x[i * incx], y[i * incy]));
    acc = wave_reduce<T, SR>(acc);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0)
        partials[blockIdx.x] = R::add(R::add(red[0], red[1]), R::add(red[2], red[3]));
}

// Unit strides, 16-byte aligned: 128-bit non-temporal loads, one vector of
// each operand per thread and iteration (up to 8192 workgroups: 2^26
// elements measured 6.7 TB/s against 6.2 with 2048 workgroups and two vectors
// an iteration); the n % 4 tail elements go to workgroup 0.
template <typename T, int SR>
__global__ __launch_bounds__(256) void tropical_dot_partial_v4_kernel(long n, const T* x,
                                                                       const T* y, T* partials) {
    using R = Ring<SR, T>;
    __shared__ T red[4];
    const long nv = n / 4;
    const v4<T>* x4 = reinterpret_cast<const v4<T>*>(x);
    const v4<T>* y4 = reinterpret_cast<const v4<T>*>(y);
    const long stride = (long)gridDim.x * blockDim.x;
    T acc0 = R::absent(), acc1 = R::absent();
    for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < nv; i += stride) {
        const v4<T> a = __builtin_nontemporal_load(x4 + i), b = __builtin_nontemporal_load(y4 + i);
        acc0 = R::add3(acc0, R::mul(a[0], b[0]), R::mul(a[1], b[1]));
        acc1 = R::add3(acc1, R::mul(a[2], b[2]), R::mul(a[3], b[3]));
    }
    if (blockIdx.x == 0 && threadIdx.x < n - nv * 4)
        acc0 = R::add(acc0, R::mul(x[nv * 4 + threadIdx.x], y[nv * 4 + threadIdx.x]));
    T acc = wave_reduce<T, SR>(R::add(acc0, acc1));
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0)
        partials[blockIdx.x] = R::add(R::add(red[0], red[1]), R::add(red[2], red[3]));
}

// One workgroup of 1024 threads: eight partials per thread, loaded before
// they are combined.
template <typename T, int SR>
__global__ __launch_bounds__(1024) void tropical_dot_final_kernel(int np, const T* partials,
                                                                   T* result) {
    using R = Ring<SR, T>;
    __shared__ T red[16];
    T acc = R::absent();
    for (int i0 = 0; i0 < np; i0 += 8 * 1024) {
        T v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int i = i0 + u * 1024 + (int)threadIdx.x;
            v[u] = i < np ? partials[i] : R::absent();
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) acc = R::add(acc, v[u]);
    }
    acc = wave_reduce<T, SR>(acc);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        T r = red[0];
        for (int w = 1; w < 16; ++w) r = R::add(r, red[w]);
        *result = R::finish(r);
    }
}

template <typename T, int SR>
static hipError_t dot_typed(int n, const void* x, long incx, const void* y, long incy,
                            void* partials, void* result, hipStream_t s) {
    int blocks = 0;
    if (n > 0) {
        const bool vec = incx == 1 && incy == 1 && (((uintptr_t)x | (uintptr_t)y) % 16 == 0);
        blocks = vec ? (int)std::min<long>(grid_one((long)n / 4), DOT_MAX_BLOCKS) : (int)grid_for(n, 8);
        if (blocks > DOT_MAX_BLOCKS) blocks = DOT_MAX_BLOCKS;
        if (vec)
            hipLaunchKernelGGL((tropical_dot_partial_v4_kernel<T, SR>), dim3(blocks), dim3(256), 0, s,
                               (long)n, (const T*)x, (const T*)y, (T*)partials);
        else
            hipLaunchKernelGGL((tropical_dot_partial_kernel<T, SR>), dim3(blocks), dim3(256), 0, s,
                               (long)n, (const T*)x, incx, (const T*)y, incy, (T*)partials);
    }
    hipLaunchKernelGGL((tropical_dot_final_kernel<T, SR>), dim3(1), dim3(1024), 0, s, blocks,
                       (const T*)partials, (T*)result);
    return hipGetLastError();
}

hipError_t launch_dot(int sr, int dt, int n, const void* x, long incx, const void* y, long incy,
                      void* partials, void* result, hipStream_t s) {
    if (dt == BTAS_FLOAT32)
        return sr == BTAS_MIN_PLUS
                   ? dot_typed<float, 0>(n, x, incx, y, incy, partials, result, s)
                   : dot_typed<float, 1>(n, x, incx, y, incy, partials, result, s);
    return sr == BTAS_MIN_PLUS ? dot_typed<int32_t, 0>(n, x, incx, y, incy, partials, result, s)
                               : dot_typed<int32_t, 1>(n, x, incx, y, incy, partials, result, s);
}

}  // namespace btas
