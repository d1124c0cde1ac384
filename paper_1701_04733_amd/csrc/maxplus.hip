// Maximum cycle mean of a max-plus matrix (its max-plus eigenvalue: the
// cycle time of the system x(k+1) = A (x) x(k), an application of the
// max-plus semiring of Sec. I), by Karp's theorem.
//
// With x_0 = 0 and x_{k+1} = A (x) x_k, x_k(v) is the heaviest walk of exactly
// k edges from v, and the largest cycle mean is
//     max over v with x_n(v) present of
//     min over k < n with x_k(v) present of (x_n(v) - x_k(v)) / (n - k);
// no v has x_n(v) present iff the graph has no cycle.  The n products are the
// library's max-plus gemv; the kernels here prepare the walk table X (row k
// holds x_k) and reduce it.  int32: the fraction is exact (64-bit cross
// multiplication) and returned in lowest terms; float32: the ratios are
// evaluated in binary64, as (double)x_n - (double)x_k divided by n - k.
#include <hip/hip_runtime.h>

#include <cstdlib>
#include <type_traits>

#include "kernels.h"
#include "semiring.h"

namespace btas {

namespace {

constexpr int CM_NT = 256;

// max |A_ij| over present (finite) entries, int32.
__global__ __launch_bounds__(CM_NT) void cm_maxabs_kernel(int n, const int32_t* A, long lda,
                                                         int* out) {
    int m = 0;
    const long total = (long)n * n;
    for (long e = (long)blockIdx.x * CM_NT + threadIdx.x; e < total; e += (long)gridDim.x * CM_NT) {
        const int32_t x = A[(e / n) * lda + e % n];
        if (x != BTAS_I32_NEG_INF) m = max(m, x < 0 ? -x : x);
    }
    for (int o = 32; o > 0; o >>= 1) m = max(m, __shfl_down(m, o, 64));
    if ((threadIdx.x & 63) == 0 && m > 0) atomicMax(out, m);
}

// X row 0 = 0 (every vertex a start), rows 1..n = absent (each row is the
// accumulator of one product).
template <typename T>
__global__ __launch_bounds__(CM_NT) void cm_fill_kernel(int n, T* X) {
    const long total = (long)(n + 1) * n;
    for (long e = (long)blockIdx.x * CM_NT + threadIdx.x; e < total; e += (long)gridDim.x * CM_NT)
        X[e] = e < n ? (T)0 : Ring<BTAS_MAX_PLUS, T>::absent();
}

// Per vertex v: the min over k of the ratio (p / q), or q = 0 if x_n(v) is
// absent.  int32: p, q exact; float32: the binary64 ratio in p (q = 1).
struct Ratio {
    long long p, q;
    double r;
};

template <typename T>
__global__ __launch_bounds__(CM_NT) void cm_vertex_kernel(int n, const T* X, Ratio* out) {
    using R = Ring<BTAS_MAX_PLUS, T>;
    const int v = blockIdx.x * CM_NT + threadIdx.x;
    if (v >= n) return;
    const T xn = X[(long)n * n + v];
    Ratio best{0, 0, 0.0};
    if (xn != R::absent()) {
        if constexpr (std::is_same_v<T, int32_t>) {
            long long mp = 0, mq = 0;
            for (int k = 0; k < n; ++k) {
                const T xk = X[(long)k * n + v];
                if (xk == R::absent()) continue;
                const long long p = (long long)xn - xk, q = n - k;
                if (mq == 0 || p * mq < mp * q) {
                    mp = p;
                    mq = q;
                }
            }
            best = Ratio{mp, mq, 0.0};
        } else {
            double mr = __builtin_inf();
            for (int k = 0; k < n; ++k) {
                const T xk = X[(long)k * n + v];
                if (xk == R::absent()) continue;
                const double r = ((double)xn - (double)xk) / (double)(n - k);
                if (r < mr) mr = r;
            }
            best = Ratio{0, 1, mr};
        }
    }
    out[v] = best;
}

__device__ __forceinline__ bool ratio_greater(const Ratio& a, const Ratio& b, bool exact) {
    if (a.q == 0) return false;
    if (b.q == 0) return true;
    return exact ? a.p * b.q > b.p * a.q : a.r > b.r;
}

// One workgroup: the max over vertices; result[0] = num, [1] = den (lowest
// terms; den = 0: no cycle), bits of lambda in [2].
__global__ __launch_bounds__(1024) void cm_final_kernel(int n, const Ratio* per, bool exact,
                                                        long long* result) {
    __shared__ Ratio red[1024];
    Ratio best{0, 0, 0.0};
    for (int v = threadIdx.x; v < n; v += 1024)
        if (ratio_greater(per[v], best, exact)) best = per[v];
    red[threadIdx.x] = best;
    __syncthreads();
    for (int o = 512; o > 0; o >>= 1) {
        if (threadIdx.x < o && ratio_greater(red[threadIdx.x + o], red[threadIdx.x], exact))
            red[threadIdx.x] = red[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        Ratio b = red[0];
        double lambda = -__builtin_inf();
        long long num = 0, den = 0;
        if (b.q != 0) {
            if (exact) {
                long long a = b.p < 0 ? -b.p : b.p, c = b.q;
                while (c != 0) {
                    const long long t = a % c;
                    a = c;
                    c = t;
                }
                num = a > 1 ? b.p / a : b.p;
                den = a > 1 ? b.q / a : b.q;
                lambda = (double)num / (double)den;
            } else {
                lambda = b.r;
            }
        }
        result[0] = num;
        result[1] = den;
        result[2] = __builtin_bit_cast(long long, lambda);
    }
}

// ---- all n products in one cooperative launch (n <= 4096) ----
// Wave w of workgroup b owns row v = 16b + w of A, lane l its columns l,
// l+64, ..., l+4032, in registers for the whole launch; step k stages x_k
// (row k of X) in LDS, each wave folds its row's 64 terms per lane and
// reduces over the lanes, and x_{k+1}(v) goes to row k+1 of X.  The same
// terms as the gemv (one rounded sum each, max exact), so the same values.
// Between steps a device-wide barrier: each workgroup stores its arrival
// word (2b for barrier b, two sets by parity) and polls all of them; X and
// the words are accessed with device-scope loads and stores, so no cache
// maintenance is needed across the XCDs.  Every wait is bounded; on a
// timeout *err is set and the kernel runs to its end.
constexpr int CP_NT = 1024;                 // threads per workgroup: 16 rows
constexpr int CP_ROWS = CP_NT / 64;
constexpr int CP_COLS = 64;                 // columns per lane
constexpr int CP_MAX_N = 64 * CP_COLS;      // 4096
constexpr int CP_MAX_GRID = CP_MAX_N / CP_ROWS;

template <typename T>
__device__ __forceinline__ T cp_ld(const T* p) {
    return __hip_atomic_load(const_cast<T*>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <typename T>
__device__ __forceinline__ void cp_st(T* p, T v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ void cp_barrier(unsigned* arrive, unsigned b, int* err, int spin_limit) {
    asm volatile("s_waitcnt vmcnt(0)" ::: "memory");  // this wave's stores are performed
    __syncthreads();
    unsigned* words = arrive + (b & 1) * CP_MAX_GRID;
    if (threadIdx.x == 0) cp_st(words + blockIdx.x, 2 * b);
    for (int polls = 0;; ++polls) {
        int ok = 1;
        for (unsigned i = threadIdx.x; i < gridDim.x; i += CP_NT) ok &= cp_ld(words + i) >= 2 * b;
        if (__syncthreads_and(ok)) break;
        if (polls >= spin_limit) {
            if (threadIdx.x == 0) cp_st(err, 1);
            break;
        }
        __builtin_amdgcn_s_sleep(1);
    }
}

template <typename T>
__global__ __launch_bounds__(CP_NT) void cm_persistent_kernel(int n, const T* __restrict__ A, long lda,
                                                              T* X, unsigned* arrive, int* err,
                                                              int spin_limit) {
    using R = Ring<BTAS_MAX_PLUS, T>;
    __shared__ T xs[CP_MAX_N];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int v = blockIdx.x * CP_ROWS + w;
    T a[CP_COLS];
#pragma unroll
    for (int i = 0; i < CP_COLS; ++i) {
        const int u = lane + 64 * i;
        a[i] = (v < n && u < n) ? A[(long)v * lda + u] : R::absent();
    }
    for (int k = 0; k < n; ++k) {
        const T* xk = X + (long)k * n;
        for (int u = threadIdx.x; u < CP_MAX_N; u += CP_NT) xs[u] = u < n ? cp_ld(xk + u) : R::absent();
        __syncthreads();
        T p0 = R::absent(), p1 = R::absent();
#pragma unroll
        for (int i = 0; i < CP_COLS; i += 4) {
            p0 = R::add3(p0, R::mul(a[i], xs[lane + 64 * i]), R::mul(a[i + 1], xs[lane + 64 * (i + 1)]));
            p1 = R::add3(p1, R::mul(a[i + 2], xs[lane + 64 * (i + 2)]), R::mul(a[i + 3], xs[lane + 64 * (i + 3)]));
        }
        T y = R::add(p0, p1);
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1) y = R::add(y, __shfl_xor(y, off, 64));
        if (lane == 0 && v < n) cp_st(X + (long)(k + 1) * n + v, R::finish(y));
        cp_barrier(arrive, (unsigned)k + 1, err, spin_limit);
    }
}

unsigned grid_for(long total) {
    long b = (total + CM_NT * 4 - 1) / (CM_NT * 4);
    return (unsigned)(b < 1 ? 1 : (b > 8192 ? 8192 : b));
}

}  // namespace

// Workspace: the walk table X, the per-vertex ratios, then the persistent
// launch's error word and arrival words.
size_t cycle_mean_ws_bytes(int n) {
    return ((size_t)(n + 1) * n * 4 + 255) / 256 * 256 + ((size_t)n * sizeof(Ratio) + 255) / 256 * 256 +
           (size_t)(1 + 2 * CP_MAX_GRID) * 4 + 64;
}

hipError_t launch_cycle_mean_maxabs(int n, const void* A, long lda, int* out, hipStream_t s) {
    hipLaunchKernelGGL(cm_maxabs_kernel, dim3(grid_for((long)n * n)), dim3(CM_NT), 0, s, n,
                       (const int32_t*)A, lda, out);
    return hipGetLastError();
}

hipError_t launch_cycle_mean(int dt, int n, const void* A, long lda, void* ws, long long* result,
                             int num_cus, int* err_out, hipStream_t s) {
    char* base = static_cast<char*>(ws);
    const size_t xbytes = ((size_t)(n + 1) * n * 4 + 255) / 256 * 256;
    Ratio* per = reinterpret_cast<Ratio*>(base + xbytes);
    int* words = reinterpret_cast<int*>(base + xbytes + ((size_t)n * sizeof(Ratio) + 255) / 256 * 256);
    const unsigned g = grid_for((long)(n + 1) * n);
    hipError_t e = hipSuccess;
    if (dt == BTAS_FLOAT32)
        hipLaunchKernelGGL(cm_fill_kernel<float>, dim3(g), dim3(CM_NT), 0, s, n, (float*)ws);
    else
        hipLaunchKernelGGL(cm_fill_kernel<int32_t>, dim3(g), dim3(CM_NT), 0, s, n, (int32_t*)ws);
    e = hipGetLastError();
    // One cooperative launch when the rows fit the resident workgroups (one
    // per 16 rows, at most one per CU), else one gemv launch per step.
    // (BTAS_CM_PERSISTENT=0 keeps the per-step launches at every size.)
    const int grid = (n + CP_ROWS - 1) / CP_ROWS;
    const char* pe = getenv("BTAS_CM_PERSISTENT");
    bool persistent = n <= CP_MAX_N && grid <= num_cus && e == hipSuccess && !(pe && pe[0] == '0');
    if (persistent) {
        e = launch_clear_flags(words, 1 + 2 * CP_MAX_GRID, s);
        int* err = words;
        unsigned* arrive = reinterpret_cast<unsigned*>(words + 1);
        int spin = 1 << 20;
        long ldl = lda;
        void* Xp = ws;
        void* args[] = {&n, const_cast<void**>(&A), &ldl, &Xp, &arrive, &err, &spin};
        if (e == hipSuccess) {
            const void* fnp = dt == BTAS_FLOAT32 ? reinterpret_cast<const void*>(cm_persistent_kernel<float>)
                                                 : reinterpret_cast<const void*>(cm_persistent_kernel<int32_t>);
            // A refused cooperative launch (the workgroups cannot all be
            // resident) falls back to one product launch per step.
            if (hipLaunchCooperativeKernel(fnp, dim3((unsigned)grid), dim3(CP_NT), args, 0, s) != hipSuccess) {
                (void)hipGetLastError();
                persistent = false;
            }
        }
        if (err_out) *err_out = persistent ? 1 : 0;  // the caller reads words[0] after synchronising
    }
    if (!persistent && e == hipSuccess) {
        if (err_out) *err_out = 0;
        for (int k = 0; k < n && e == hipSuccess; ++k)
            e = launch_gemv(BTAS_MAX_PLUS, dt, n, n, A, lda, base + (size_t)k * n * 4, 1,
                            base + (size_t)(k + 1) * n * 4, 1, s);
    }
    if (e != hipSuccess) return e;
    const unsigned gv = (unsigned)((n + CM_NT - 1) / CM_NT);
    if (dt == BTAS_FLOAT32)
        hipLaunchKernelGGL(cm_vertex_kernel<float>, dim3(gv), dim3(CM_NT), 0, s, n, (const float*)ws,
                           per);
    else
        hipLaunchKernelGGL(cm_vertex_kernel<int32_t>, dim3(gv), dim3(CM_NT), 0, s, n,
                           (const int32_t*)ws, per);
    hipLaunchKernelGGL(cm_final_kernel, dim3(1), dim3(1024), 0, s, n, per, dt == BTAS_INT32, result);
    return hipGetLastError();
}

const int* cycle_mean_error_word(int n, const void* ws) {
    const size_t xbytes = ((size_t)(n + 1) * n * 4 + 255) / 256 * 256;
    return reinterpret_cast<const int*>(static_cast<const char*>(ws) + xbytes +
                                        ((size_t)n * sizeof(Ratio) + 255) / 256 * 256);
}

}  // namespace btas
