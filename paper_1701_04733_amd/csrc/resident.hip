// Whole-solve APSP in one cooperative launch, for small graphs.
//
// Repeated squaring (Sec. III) needs every entry of D_{t-1} before any entry
// of D_t can be finished, so the ordinary path issues one product launch (and
// for small n a split-K reduction) per squaring; for n of a few hundred the
// launches, not the O(n^3) work, set the latency.  Here one launch of at most
// one resident workgroup set does the whole solve:
//
//   D_0 = I (+) W;  for t = 1..T:  D_t = D_{t-1} (+) D_{t-1} (.) D_{t-1}
//
// with a device-wide barrier between squarings.  Each workgroup owns 16x16
// output tiles (one output per thread, full k): it stages the tile's 16 rows
// of D_{t-1} and its 16 columns (transposed) in LDS, folds four k per pair of
// three-input min/max, and writes D_t to the other buffer of the ping-pong
// pair.
//
// Coherence across the XCDs (each has its own L2) is obtained without cache
// maintenance: every access to the matrices that another workgroup may touch
// in the same launch is a device-scope (relaxed atomic) load or store, which
// the hardware performs at the device's coherence point, and every wave waits
// for its stores to complete before its workgroup arrives at the barrier.
// (Writing back and invalidating the L2 around plain loads measured slower.)
//
// The barrier: every workgroup stores one arrival word of its own, 2b | c for
// barrier b, with c = 1 if its tiles changed D in the squaring just ended,
// and then polls the words of all workgroups until each reads at least 2b.
// The OR of the c bits is the early-exit decision, so every workgroup takes
// the same one without a shared flag (256 workgroups storing to one word
// serialise there: that cost several microseconds a squaring).  The words
// come in two sets, used by barriers of odd and even b: a workgroup can only
// arrive at barrier b + 2, and overwrite its word of barrier b, after every
// workgroup has arrived at b + 1, that is after every poll of barrier b has
// ended, so the bit read there is always the one of barrier b.  The caller
// zeroes the words before each launch.  The launch is cooperative, so every
// workgroup is resident and the barrier cannot wait on one that has not
// started; each wait is still bounded and, when the bound is hit, the kernel
// records an error and runs to its end so that no wave is left spinning.
#include <hip/hip_runtime.h>

#include <atomic>
#include <type_traits>

#include "gemm_tile.h"
#include "kernels.h"
#include "semiring.h"
#include "flat_index.h"

namespace btas {

namespace {

constexpr int RT = 16;        // output tile edge
constexpr int RNT = RT * RT;  // threads per workgroup, one output each
constexpr int PB = 16;        // panel loads in flight per thread (one batch up to n = 256)

template <typename T>
struct ResidentArgs {
    int n;
    int nsq;          // squarings to run (the fixed count T)
    int early;        // stop after the first squaring that changes nothing
    int cur0;         // buffer index that receives D_0
    int ls;           // LDS row stride in elements (>= n rounded to 8, plus padding)
    int spin_limit;   // bound on each barrier wait, in polls
    const T* W;
    long ldw;
    T* buf0;          // the caller's D
    long ld0;
    T* buf1;          // the handle's workspace, leading dimension n
    long ld1;
    int* flags;       // [0] error, [1] steps executed
    unsigned* arrive; // two sets of RESIDENT_MAX_GRID arrival words
    int* latch;       // pinned host word, set with flags[0] on a timeout
};

// Device-scope loads and stores (coherent across XCDs without cache flushes).
template <typename T>
__device__ __forceinline__ T ld_dev(const T* p) {
    return __hip_atomic_load(const_cast<T*>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <typename T>
__device__ __forceinline__ void st_dev(T* p, T v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// A barrier wait hit its bound: the device flag for a caller that reads the
// step count, and the handle's pinned host word for one that does not.
__device__ __forceinline__ void report_timeout(int* err, int* latch) {
    st_dev(err, 1);
    __hip_atomic_store(latch, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
}

// Device-wide barrier number b (1, 2, ... within a launch), carrying one bit
// per workgroup; returns the OR of every workgroup's `changed`.  Every thread
// of every workgroup calls it with the same b.  On a wait that hits the bound
// (at once when spin_limit < 0) the timeout is reported and the result is
// incomplete.
__device__ int grid_barrier(unsigned* arrive, unsigned b, int changed, int* err, int* latch,
                            int spin_limit) {
    asm volatile("s_waitcnt vmcnt(0)" ::: "memory");  // this wave's stores are performed
    const int mine = __syncthreads_or(changed);
    unsigned* words = arrive + (b & 1) * RESIDENT_MAX_GRID;
    if (threadIdx.x == 0) st_dev(words + blockIdx.x, 2 * b | (mine ? 1u : 0u));
    if (spin_limit < 0) {
        if (threadIdx.x == 0) report_timeout(err, latch);
        return mine;
    }
    int any = 0;
    for (int polls = 0;; ++polls) {
        int ok = 1;
        any = 0;
        for (unsigned i = threadIdx.x; i < gridDim.x; i += RNT) {
            const unsigned w = ld_dev(words + i);
            ok &= w >= 2 * b;
            any |= w & 1;
        }
        if (__syncthreads_and(ok)) break;
        if (polls >= spin_limit) {
            if (threadIdx.x == 0) report_timeout(err, latch);
            break;
        }
        __builtin_amdgcn_s_sleep(1);
    }
    return __syncthreads_or(any);
}

template <typename T>
__global__ __launch_bounds__(RNT) void apsp_resident_kernel(ResidentArgs<T> a) {
    using R = Ring<BTAS_MIN_PLUS, T>;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    T* As = reinterpret_cast<T*>(smem_raw);  // [RT][ls]: rows m0.. of D_{t-1}
    T* Bt = As + RT * a.ls;                  // [RT][ls]: columns n0.. of D_{t-1}, transposed
    const int n = a.n, tid = threadIdx.x;
    const long total = (long)n * n;
    const long gthreads = (long)gridDim.x * RNT;
    int cur = a.cur0;

    // D_0 = I (+) W (the diagonal gets min(W_ii, 0)); in place when W is D.
    {
        T* D0 = cur ? a.buf1 : a.buf0;
        const long ld0 = cur ? a.ld1 : a.ld0;
        for (long e = (long)blockIdx.x * RNT + tid; e < total; e += gthreads) {
            long i, j;
            flat_to_rc(e, n, total, i, j);
            T w = a.W[i * a.ldw + j];
            if (i == j && w > (T)0) w = (T)0;
            st_dev(D0 + i * ld0 + j, w);
        }
    }
    unsigned bno = 1;
    grid_barrier(a.arrive, bno++, 0, a.flags, a.latch, a.spin_limit);

    const int nt = (n + RT - 1) / RT;
    const int kpad = (n + 7) & ~7;
    const int r = tid / RT, c = tid % RT;
    int steps = 0;
    for (int t = 1; t <= a.nsq; ++t) {
        const T* src = cur ? a.buf1 : a.buf0;
        const long lds = cur ? a.ld1 : a.ld0;
        T* dst = cur ? a.buf0 : a.buf1;
        const long ldd = cur ? a.ld0 : a.ld1;
        bool changed = false;
        for (int tile = blockIdx.x; tile < nt * nt; tile += gridDim.x) {
            const int m0 = (tile / nt) * RT, n0 = (tile % nt) * RT;
            // Rows m0..m0+15 of src (k along the row) and columns n0..n0+15
            // (stored transposed, Bt[col][k]), in batches of PB loads per
            // thread so that the device-scope loads overlap their latency.
            for (int e0 = 0; e0 < RT * kpad; e0 += RNT * PB) {
                T va[PB], vb[PB];
#pragma unroll
                for (int u = 0; u < PB; ++u) {
                    const int e = e0 + u * RNT + tid;
                    const int rr = e / kpad, ka = e - rr * kpad;
                    const int kb = e / RT, cc = e - kb * RT;
                    va[u] = (e < RT * kpad && m0 + rr < n && ka < n)
                                ? ld_dev(src + (long)(m0 + rr) * lds + ka) : R::absent();
                    vb[u] = (e < RT * kpad && n0 + cc < n && kb < n)
                                ? ld_dev(src + (long)kb * lds + n0 + cc) : R::absent();
                }
#pragma unroll
                for (int u = 0; u < PB; ++u) {
                    const int e = e0 + u * RNT + tid;
                    if (e < RT * kpad) {
                        const int rr = e / kpad, ka = e - rr * kpad;
                        const int kb = e / RT, cc = e - kb * RT;
                        As[rr * a.ls + ka] = va[u];
                        Bt[cc * a.ls + kb] = vb[u];
                    }
                }
            }
            __syncthreads();
            // Two accumulators and an unrolled loop keep several LDS reads in
            // flight and break the serial min chain; the order of the (+)
            // does not matter (associative, commutative, one rounding per term).
            T acc0 = R::absent(), acc1 = R::absent();
            const T* ar = As + r * a.ls;
            const T* bc = Bt + c * a.ls;
#pragma unroll 4
            for (int k = 0; k < kpad; k += 8) {
                const v4<T> x0 = *reinterpret_cast<const v4<T>*>(ar + k);
                const v4<T> y0 = *reinterpret_cast<const v4<T>*>(bc + k);
                const v4<T> x1 = *reinterpret_cast<const v4<T>*>(ar + k + 4);
                const v4<T> y1 = *reinterpret_cast<const v4<T>*>(bc + k + 4);
                acc0 = R::add3(acc0, R::mul(x0[0], y0[0]), R::mul(x0[1], y0[1]));
                acc1 = R::add3(acc1, R::mul(x1[0], y1[0]), R::mul(x1[1], y1[1]));
                acc0 = R::add3(acc0, R::mul(x0[2], y0[2]), R::mul(x0[3], y0[3]));
                acc1 = R::add3(acc1, R::mul(x1[2], y1[2]), R::mul(x1[3], y1[3]));
            }
            const T acc = R::add(acc0, acc1);
            const int row = m0 + r, col = n0 + c;
            if (row < n && col < n) {
                // D_{t-1}[row][col] is in the staged row panel (k = col).
                const T old = As[r * a.ls + col];
                const T nv = R::add(old, R::finish(acc));
                changed |= bits_of(nv) != bits_of(old);
                st_dev(dst + (long)row * ldd + col, nv);
            }
            __syncthreads();  // LDS is reloaded for the next tile
        }
        const int any = grid_barrier(a.arrive, bno++, changed, a.flags, a.latch, a.spin_limit);
        cur ^= 1;
        steps = t;
        if (a.early && !any) break;
    }

    // After an early exit the result may sit in the workspace: copy it to D.
    if (cur != 0) {
        for (long e = (long)blockIdx.x * RNT + tid; e < total; e += gthreads) {
            long i, j;
            flat_to_rc(e, n, total, i, j);
            a.buf0[i * a.ld0 + j] = ld_dev(a.buf1 + i * a.ld1 + j);
        }
    }
    if (blockIdx.x == 0 && tid == 0) a.flags[1] = steps;
}

template <typename T>
hipError_t launch_typed(int n, const void* W, long ldw, void* D, long ldd, void* ws, int T_,
                        bool early, int* flags, int* latch, int num_cus, int spin_limit,
                        hipStream_t s) {
    ResidentArgs<T> a;
    a.n = n;
    a.nsq = T_;
    a.early = early ? 1 : 0;
    // The fixed-T solve ends in buf[0] when D_0 goes to buf[T & 1].
    a.cur0 = T_ & 1;
    a.ls = ((n + 7) & ~7) + 4;  // k padded to 8; rows start in distinct LDS banks
    a.spin_limit = spin_limit;
    a.W = (const T*)W;
    a.ldw = ldw;
    a.buf0 = (T*)D;
    a.ld0 = ldd;
    a.buf1 = (T*)ws;
    a.ld1 = n;
    a.flags = flags;
    a.arrive = reinterpret_cast<unsigned*>(flags + 2);
    a.latch = latch;
    const size_t lds = resident_lds_bytes(n);
    // Workgroups per CU depend only on the LDS size (k padded to 8): the
    // occupancy query runs once per size, not on every call.
    static std::atomic<int> per_cu_cache[RESIDENT_MAX_N / 8 + 2];
    const int slot = ((n + 7) & ~7) / 8;
    int per_cu = per_cu_cache[slot].load(std::memory_order_relaxed);
    if (per_cu == 0) {
        const hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(
            &per_cu, reinterpret_cast<const void*>(apsp_resident_kernel<T>), RNT, lds);
        if (e != hipSuccess) return e;
        if (per_cu < 1) return hipErrorInvalidConfiguration;
        per_cu_cache[slot].store(per_cu, std::memory_order_relaxed);
    }
    const int nt = (n + RT - 1) / RT;
    long grid = (long)per_cu * num_cus;
    if (grid > (long)nt * nt) grid = (long)nt * nt;
    if (grid > RESIDENT_MAX_GRID) grid = RESIDENT_MAX_GRID;
    void* args[] = {&a};
    return hipLaunchCooperativeKernel(reinterpret_cast<const void*>(apsp_resident_kernel<T>),
                                      dim3((unsigned)grid), dim3(RNT), args, (unsigned)lds, s);
}

// Graphs of at most 64 vertices: the whole solve in one workgroup, both
// ping-pong matrices in LDS, a workgroup barrier between squarings (no
// device-wide one).  Lane j of wave w computes column j of rows w, w+16,
// w+32, w+48: per four k it reads the column's four entries once and each
// row's four entries as one 16-byte broadcast read.  The early-exit decision
// is the OR of the workgroup's change bits.  The same terms and the same
// per-output mapping of int32 sums as the other squaring kernels, so the
// same bits.
constexpr int LDS_SOLVE_MAX_N = 64;
constexpr int LDS_SOLVE_NT = 1024;
constexpr int LDS_SOLVE_LS = LDS_SOLVE_MAX_N + 4;  // row stride: 16-byte aligned rows

template <typename T>
__global__ __launch_bounds__(LDS_SOLVE_NT) void apsp_lds_kernel(int n, const T* __restrict__ W, long ldw,
                                                                T* D, long ldd, int nsq, int early,
                                                                int* flags) {
    using R = Ring<BTAS_MIN_PLUS, T>;
    __shared__ __align__(16) T buf[2][LDS_SOLVE_MAX_N * LDS_SOLVE_LS];
    const int tid = threadIdx.x;
    // both buffers absent outside n x n, so that k runs to n rounded up to 4
    for (int e = tid; e < 2 * LDS_SOLVE_MAX_N * LDS_SOLVE_LS; e += LDS_SOLVE_NT) (&buf[0][0])[e] = R::absent();
    __syncthreads();
    for (int o = tid; o < n * n; o += LDS_SOLVE_NT) {
        const int i = o / n, j = o - i * n;
        T w = W[(long)i * ldw + j];
        if (i == j && w > (T)0) w = (T)0;
        buf[0][i * LDS_SOLVE_LS + j] = w;
    }
    __syncthreads();
    const int j = tid & 63, ib = tid >> 6;
    const int n4 = (n + 3) & ~3;
    int cur = 0, steps = 0;
    for (int t = 1; t <= nsq; ++t) {
        const T* S = buf[cur];
        T* Dn = buf[cur ^ 1];
        T acc[4][2];
#pragma unroll
        for (int r = 0; r < 4; ++r) acc[r][0] = acc[r][1] = R::absent();
        for (int k = 0; k < n4; k += 4) {
            const T b0 = S[k * LDS_SOLVE_LS + j], b1 = S[(k + 1) * LDS_SOLVE_LS + j];
            const T b2 = S[(k + 2) * LDS_SOLVE_LS + j], b3 = S[(k + 3) * LDS_SOLVE_LS + j];
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const v4<T> a = *reinterpret_cast<const v4<T>*>(S + (ib + 16 * r) * LDS_SOLVE_LS + k);
                acc[r][0] = R::add3(acc[r][0], R::mul(a[0], b0), R::mul(a[1], b1));
                acc[r][1] = R::add3(acc[r][1], R::mul(a[2], b2), R::mul(a[3], b3));
            }
        }
        bool changed = false;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int i = ib + 16 * r;
            if (i < n && j < n) {
                const T old = S[i * LDS_SOLVE_LS + j];
                const T nv = R::add(old, R::finish(R::add(acc[r][0], acc[r][1])));
                changed |= bits_of(nv) != bits_of(old);
                Dn[i * LDS_SOLVE_LS + j] = nv;
            }
        }
        const int any = __syncthreads_or(changed);  // also: Dn complete before it is read
        cur ^= 1;
        steps = t;
        if (early && !any) break;
    }
    for (int o = tid; o < n * n; o += LDS_SOLVE_NT) {
        const int i = o / n, jj = o - i * n;
        D[(long)i * ldd + jj] = buf[cur][i * LDS_SOLVE_LS + jj];
    }
    if (tid == 0) flags[1] = steps;
}

}  // namespace

size_t resident_lds_bytes(int n) { return (size_t)2 * RT * (((n + 7) & ~7) + 4) * 4; }

hipError_t launch_apsp_resident(int dt, int n, const void* W, long ldw, void* D, long ldd,
                                void* ws, int T, bool early, int* flags, int* latch,
                                int num_cus, int spin_limit, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    if (n <= LDS_SOLVE_MAX_N) {
        if (dt == BTAS_FLOAT32)
            hipLaunchKernelGGL(apsp_lds_kernel<float>, dim3(1), dim3(LDS_SOLVE_NT), 0, s, n,
                               (const float*)W, ldw, (float*)D, ldd, T, early ? 1 : 0, flags);
        else
            hipLaunchKernelGGL(apsp_lds_kernel<int32_t>, dim3(1), dim3(LDS_SOLVE_NT), 0, s, n,
                               (const int32_t*)W, ldw, (int32_t*)D, ldd, T, early ? 1 : 0, flags);
        return hipGetLastError();
    }
    if (dt == BTAS_FLOAT32)
        return launch_typed<float>(n, W, ldw, D, ldd, ws, T, early, flags, latch, num_cus,
                                   spin_limit, s);
    return launch_typed<int32_t>(n, W, ldw, D, ldd, ws, T, early, flags, latch, num_cus,
                                 spin_limit, s);
}

}  // namespace btas
