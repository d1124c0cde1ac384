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
// with, in the general case, a device-wide barrier between squarings (two
// faster orderings for a grid of one workgroup per tile follow below: the
// tagged mode and, without its buffer, the panel wait).  Each workgroup owns 16x16
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
// ended, so the bit read there is always the one of barrier b.  Each launch
// carries an epoch (a per-handle launch count, below 2^24) in the high bits
// of its words, so the words a previous launch left behind read as "not
// arrived" and nothing has to be cleared between launches; the host clears
// them only when the count wraps.  The launch is cooperative, so every
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
#include "lds_solve.h"

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
    int* flags;       // [0] epoch of a launch that timed out, [1] steps executed
    unsigned* arrive; // two sets of RESIDENT_MAX_GRID arrival words
    unsigned epoch;   // this launch's tag in the arrival words, 1 .. 2^24 - 1
    int* latch;       // pinned host word, set with flags[0] on a timeout
    // Packed 16-bit mode (int32 only): gate_max >= 0 enables it for graphs
    // whose finite off-diagonal weights lie in [0, gate_max] with no negative
    // diagonal entry; u16[0..1] are two n x ld16 matrices of 16-bit distances.
    int gate_max;
    int ld16;
    uint16_t* u16[2];
    // Tagged mode (one tile per workgroup, a tag buffer of the handle's own):
    // D_s as 64-bit words in tag[s % 2] (n x n), and per-squaring change
    // words cw[s * RESIDENT_MAX_GRID + workgroup] for early exit.
    uint64_t* tag[2];
    uint64_t* cw;
};

// ---- packed 16-bit mode ------------------------------------------------
// An int32 graph whose weights are non-negative and at most gate_max =
// floor(65534 / (2 (n - 1))) is squared on 16-bit distances, two per 32-bit
// register: v_pk_add_u16 with clamp forms two terms, v_pk_min_u16 folds
// them (Sec. I semirings on 16-bit lanes).  Exact: every finite entry of
// every D_t is the length of a simple path (non-negative weights: dropping
// a cycle never lengthens a walk), so it is at most (n - 1) * gate_max and
// every sum of two finite entries is at most 65534; any sum that involves
// the absent value 0xFFFF clamps to 0xFFFF, which is again absent.  The
// output is mapped back to int32 (0xFFFF -> BTAS_I32_INF): the same bits as
// the int32 squarings, with half the bytes per panel load and one VALU
// instruction per term.
using u16x2 = uint16_t __attribute__((ext_vector_type(2)));
constexpr uint16_t U16_ABSENT = 0xFFFF;

__device__ __forceinline__ uint32_t pk_add_sat(uint32_t x, uint32_t y) {
    return __builtin_bit_cast(uint32_t, __builtin_elementwise_add_sat(__builtin_bit_cast(u16x2, x),
                                                                      __builtin_bit_cast(u16x2, y)));
}
__device__ __forceinline__ uint32_t pk_min(uint32_t x, uint32_t y) {
    return __builtin_bit_cast(uint32_t, __builtin_elementwise_min(__builtin_bit_cast(u16x2, x),
                                                                  __builtin_bit_cast(u16x2, y)));
}
// Absent in the halves whose column index (2 kp, 2 kp + 1) is >= n.
__device__ __forceinline__ uint32_t mask_pair(uint32_t v, int k_lo, int n) {
    if (k_lo + 1 >= n) v |= 0xFFFF0000u;
    if (k_lo >= n) v |= 0x0000FFFFu;
    return v;
}

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
__device__ __forceinline__ void report_timeout(int* err, int* latch, unsigned epoch) {
    st_dev(err, (int)epoch);
    __hip_atomic_store(latch, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
}

// Device-wide barrier number b (1, 2, ... within a launch), carrying one bit
// per workgroup; returns the OR of every workgroup's `changed`.  Every thread
// of every workgroup calls it with the same b.  On a wait that hits the bound
// (at once when spin_limit < 0) the timeout is reported and the result is
// incomplete.
__device__ int grid_barrier(unsigned* arrive, unsigned b, int changed, int* err, int* latch,
                            int spin_limit, unsigned epoch) {
    asm volatile("s_waitcnt vmcnt(0)" ::: "memory");  // this wave's stores are performed
    const int mine = __syncthreads_or(changed);
    unsigned* words = arrive + (b & 1) * RESIDENT_MAX_GRID;
    const unsigned tag = epoch << 8 | b << 1;  // b < 128: at most T + 2 barriers
    if (threadIdx.x == 0) st_dev(words + blockIdx.x, tag | (mine ? 1u : 0u));
    if (spin_limit < 0) {
        if (threadIdx.x == 0) report_timeout(err, latch, epoch);
        return mine;
    }
    int any = 0;
    for (int polls = 0;; ++polls) {
        int ok = 1;
        any = 0;
        for (unsigned i = threadIdx.x; i < gridDim.x; i += RNT) {
            const unsigned w = ld_dev(words + i);
            ok &= w >= tag;
            any |= w & 1;
        }
        if (__syncthreads_and(ok)) break;
        if (polls >= spin_limit) {
            if (threadIdx.x == 0) report_timeout(err, latch, epoch);
            break;
        }
        __builtin_amdgcn_s_sleep(1);
    }
    return __syncthreads_or(any);
}

// The squarings of the 16-bit mode, then D <- the result as int32.  D_0 is
// in u16[0]; every workgroup has passed barrier bno - 1.
__device__ void solve_u16(const ResidentArgs<int32_t>& a, unsigned char* smem, unsigned bno) {
    const int n = a.n, tid = threadIdx.x;
    const int kpad = (n + 7) & ~7;           // k padded to 8 (one 16-byte LDS read)
    const int kh = kpad / 2;                 // 32-bit pairs per staged row
    const int ls16 = kpad + 8;               // LDS row stride (16-byte aligned rows)
    uint16_t* As = reinterpret_cast<uint16_t*>(smem);  // [RT][ls16]: rows m0.. of D_{t-1}
    uint16_t* Bt = As + RT * ls16;                       // [RT][ls16]: columns n0.., transposed
    const int nt = (n + RT - 1) / RT;
    const int r = tid / RT, c = tid % RT;
    const long ld16 = a.ld16;
    int cur = 0, steps = 0;
    for (int t = 1; t <= a.nsq; ++t) {
        const uint16_t* src = a.u16[cur];
        uint16_t* dst = a.u16[cur ^ 1];
        bool changed = false;
        for (int tile = blockIdx.x; tile < nt * nt; tile += gridDim.x) {
            const int m0 = (tile / nt) * RT, n0 = (tile % nt) * RT;
            // Rows m0..m0+15 as pairs along k, and columns n0..n0+15 as pairs
            // of adjacent columns at one k (split into the transposed panel).
            constexpr int PB16 = 8;
            for (int e0 = 0; e0 < RT * kh; e0 += RNT * PB16) {
                uint32_t va[PB16], vb[PB16];
#pragma unroll
                for (int u = 0; u < PB16; ++u) {
                    const int e = e0 + u * RNT + tid;
                    const int rr = e / kh, kp = e - rr * kh;
                    const int kb = e / (RT / 2), cp = e - kb * (RT / 2);
                    const int col = n0 + 2 * cp;
                    va[u] = (e < RT * kh && m0 + rr < n)
                                ? mask_pair(ld_dev(reinterpret_cast<const uint32_t*>(
                                                src + (long)(m0 + rr) * ld16) + kp), 2 * kp, n)
                                : 0xFFFFFFFFu;
                    vb[u] = (e < RT * kh && kb < n && col < n)
                                ? mask_pair(ld_dev(reinterpret_cast<const uint32_t*>(
                                                src + (long)kb * ld16 + col)), col, n)
                                : 0xFFFFFFFFu;
                }
#pragma unroll
                for (int u = 0; u < PB16; ++u) {
                    const int e = e0 + u * RNT + tid;
                    if (e < RT * kh) {
                        const int rr = e / kh, kp = e - rr * kh;
                        const int kb = e / (RT / 2), cp = e - kb * (RT / 2);
                        reinterpret_cast<uint32_t*>(As + rr * ls16)[kp] = va[u];
                        Bt[(2 * cp) * ls16 + kb] = (uint16_t)(vb[u] & 0xFFFFu);
                        Bt[(2 * cp + 1) * ls16 + kb] = (uint16_t)(vb[u] >> 16);
                    }
                }
            }
            __syncthreads();
            // Eight k per pair of 16-byte LDS reads: four packed adds (two
            // terms each) and four packed mins into two accumulators.
            uint32_t acc0 = 0xFFFFFFFFu, acc1 = 0xFFFFFFFFu;
            const uint32_t* ar = reinterpret_cast<const uint32_t*>(As + r * ls16);
            const uint32_t* bc = reinterpret_cast<const uint32_t*>(Bt + c * ls16);
#pragma unroll 4
            for (int k2 = 0; k2 < kh; k2 += 4) {
                const v4<uint32_t> x = *reinterpret_cast<const v4<uint32_t>*>(ar + k2);
                const v4<uint32_t> y = *reinterpret_cast<const v4<uint32_t>*>(bc + k2);
                acc0 = pk_min(acc0, pk_add_sat(x[0], y[0]));
                acc1 = pk_min(acc1, pk_add_sat(x[1], y[1]));
                acc0 = pk_min(acc0, pk_add_sat(x[2], y[2]));
                acc1 = pk_min(acc1, pk_add_sat(x[3], y[3]));
            }
            const uint32_t m2 = pk_min(acc0, acc1);
            const uint32_t lo = m2 & 0xFFFFu, hi = m2 >> 16;
            const int row = m0 + r, col = n0 + c;
            const uint32_t old = col < n ? As[r * ls16 + col] : U16_ABSENT;
            const uint32_t acc = lo < hi ? lo : hi;
            const uint32_t nv = acc < old ? acc : old;
            changed |= row < n && col < n && nv != old;
            // lanes c and c + 1 (adjacent) store one 32-bit pair; a pair whose
            // second column is n writes into the row padding, never read as
            // data (masked when staged)
            const uint32_t nb = (uint32_t)__shfl_down((int)nv, 1);
            if ((c & 1) == 0 && row < n && col < n)
                st_dev(reinterpret_cast<uint32_t*>(dst + (long)row * ld16 + col), nv | (nb << 16));
            __syncthreads();  // LDS is reloaded for the next tile
        }
        const int any = grid_barrier(a.arrive, bno++, changed, a.flags, a.latch, a.spin_limit, a.epoch);
        cur ^= 1;
        steps = t;
        if (a.early && !any) break;
    }
    // D <- the 16-bit result as int32
    const long total = (long)n * n;
    const long gthreads = (long)gridDim.x * RNT;
    for (long e = (long)blockIdx.x * RNT + tid; e < total; e += gthreads) {
        long i, j;
        flat_to_rc(e, n, total, i, j);
        const uint16_t v = ld_dev(a.u16[cur] + i * ld16 + j);
        a.buf0[i * a.ld0 + j] = v == U16_ABSENT ? BTAS_I32_INF : (int32_t)v;
    }
    if (blockIdx.x == 0 && tid == 0) a.flags[1] = steps | RESIDENT_PACKED16_BIT;
}

// ---- tagged mode --------------------------------------------------------
// One 16x16 tile per workgroup.  Every entry of D_s (s < T) is stored as one
// 64-bit word, (epoch << 8 | s) << 32 | value bits, in buffer s mod 2 of a
// tag buffer that only these launches write.  Squaring t loads its row and
// column panels of D_{t-1} and loads again every word whose tag is not yet
// that of D_{t-1}: the data says by itself that it has arrived, so nothing
// (no flag, no wait for store completion, no barrier) separates squarings.
// Two buffers suffice: squaring t overwrites this tile of D_{t-2}, which
// only the workgroups of the tile's row and column panels read (a workgroup
// reads tile (I, J) exactly when the owner of (I, J) reads the
// workgroup's tile: same row or same column), in their squaring t - 1; the
// D_{t-1} entries squaring t has just loaded were written by those same
// workgroups at the end of their squaring t - 1, after its loads had
// returned.  The entry a thread owns stays in a register from squaring to
// squaring, and the last one goes to D.
//
// Early exit without a barrier: each workgroup publishes one change word per
// squaring (tagged the same way); after squaring t every workgroup reads the
// words of squaring t - 1 of all workgroups, and if none changed, D_{t-1} is
// the fixpoint (D_t equals it bit for bit) and all stop with the same step
// count, t - 1, as the barrier path.  The extra squaring t is the price of
// not waiting for the OR.
__device__ __forceinline__ uint64_t tag_word(uint32_t tag, uint32_t bits) {
    return (uint64_t)tag << 32 | bits;
}

template <typename T>
__device__ __forceinline__ T word_value(uint64_t w) {
    return __builtin_bit_cast(T, (uint32_t)w);
}

template <typename T>
__global__ __launch_bounds__(RNT) void apsp_tagged_kernel(ResidentArgs<T> a) {
    using R = Ring<BTAS_MIN_PLUS, T>;
    extern __shared__ __align__(16) unsigned char smem[];
    T* As = reinterpret_cast<T*>(smem);  // [RT][ls]: rows m0.. of D_{t-1}
    T* Bt = As + RT * a.ls;              // [RT][ls]: columns n0.. of D_{t-1}, transposed
    const int n = a.n, tid = threadIdx.x;
    const int nt = (n + RT - 1) / RT;
    const int kpad = (n + 7) & ~7;
    const int r = tid / RT, c = tid % RT;
    const int m0 = (blockIdx.x / nt) * RT, n0 = (blockIdx.x % nt) * RT;
    const int row = m0 + r, col = n0 + c;
    const bool mine = row < n && col < n;
    const uint32_t base = a.epoch << 8;
    const uint32_t absent_bits = __builtin_bit_cast(uint32_t, R::absent());
    int spin = a.spin_limit;
    if (spin < 0) {
        if (tid == 0) report_timeout(a.flags, a.latch, a.epoch);
        spin = 0;
    }

    // D_0 = I (+) W, this tile only (W may be D: each entry is read and
    // written by its own thread only).
    T d = R::absent();
    if (mine) {
        T w = a.W[(long)row * a.ldw + col];
        if (row == col && w > (T)0) w = (T)0;
        d = w;
        if (a.nsq > 0) st_dev(a.tag[0] + (long)row * n + col, tag_word(base, __builtin_bit_cast(uint32_t, w)));
    }
    int steps = 0;
    for (int t = 1; t <= a.nsq; ++t) {
        const uint64_t* src = a.tag[(t - 1) & 1];
        const uint32_t want = base | (uint32_t)(t - 1);
        const uint64_t pad = tag_word(want, absent_bits);
        for (int e0 = 0; e0 < RT * kpad; e0 += RNT * PB) {
            uint64_t va[PB], vb[PB];
            auto load = [&](int u, bool a_side) -> uint64_t {
                const int e = e0 + u * RNT + tid;
                if (a_side) {
                    const int rr = e / kpad, ka = e - rr * kpad;
                    return (e < RT * kpad && m0 + rr < n && ka < n)
                               ? ld_dev(src + (long)(m0 + rr) * n + ka) : pad;
                }
                const int kb = e / RT, cc = e - kb * RT;
                return (e < RT * kpad && n0 + cc < n && kb < n) ? ld_dev(src + (long)kb * n + n0 + cc)
                                                                : pad;
            };
#pragma unroll
            for (int u = 0; u < PB; ++u) {
                va[u] = load(u, true);
                vb[u] = load(u, false);
            }
            for (int polls = 0;; ++polls) {
                bool late = false;
#pragma unroll
                for (int u = 0; u < PB; ++u)
                    late |= (uint32_t)(va[u] >> 32) != want || (uint32_t)(vb[u] >> 32) != want;
                if (!late) break;
                if (polls >= spin) {
                    report_timeout(a.flags, a.latch, a.epoch);
                    spin = 0;
                    break;
                }
                __builtin_amdgcn_s_sleep(1);
#pragma unroll
                for (int u = 0; u < PB; ++u) {
                    if ((uint32_t)(va[u] >> 32) != want) va[u] = load(u, true);
                    if ((uint32_t)(vb[u] >> 32) != want) vb[u] = load(u, false);
                }
            }
#pragma unroll
            for (int u = 0; u < PB; ++u) {
                const int e = e0 + u * RNT + tid;
                if (e < RT * kpad) {
                    const int rr = e / kpad, ka = e - rr * kpad;
                    const int kb = e / RT, cc = e - kb * RT;
                    As[rr * a.ls + ka] = word_value<T>(va[u]);
                    Bt[cc * a.ls + kb] = word_value<T>(vb[u]);
                }
            }
        }
        __syncthreads();
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
        const T nv = R::add(d, R::finish(R::add(acc0, acc1)));
        const bool changed = mine && bits_of(nv) != bits_of(d);
        d = nv;
        steps = t;
        if (t < a.nsq && mine)
            st_dev(a.tag[t & 1] + (long)row * n + col, tag_word(base | (uint32_t)t, __builtin_bit_cast(uint32_t, nv)));
        if (a.early) {
            const int here = __syncthreads_or(changed);  // also: LDS is free for the next squaring
            if (tid == 0)
                st_dev(a.cw + (long)t * RESIDENT_MAX_GRID + blockIdx.x, tag_word(base | (uint32_t)t, here));
            if (t >= 2) {
                const uint32_t prev = base | (uint32_t)(t - 1);
                int any = 0;
                for (int i = tid; i < (int)gridDim.x; i += RNT) {
                    const uint64_t* p = a.cw + (long)(t - 1) * RESIDENT_MAX_GRID + i;
                    uint64_t w = ld_dev(p);
                    for (int polls = 0; (uint32_t)(w >> 32) != prev; ++polls) {
                        if (polls >= spin) {
                            report_timeout(a.flags, a.latch, a.epoch);
                            spin = 0;
                            break;
                        }
                        __builtin_amdgcn_s_sleep(1);
                        w = ld_dev(p);
                    }
                    any |= (int)(w & 1);
                }
                if (!__syncthreads_or(any)) {
                    steps = t - 1;  // D_t == D_{t-1}: the fixpoint
                    break;
                }
            }
        } else {
            __syncthreads();  // LDS is reloaded for the next squaring
        }
    }
    if (mine) a.buf0[(long)row * a.ld0 + col] = d;
    if (blockIdx.x == 0 && tid == 0) a.flags[1] = steps;
}

// Dataflow wait (fixed T, one tile per workgroup): before squaring t, wait
// only for the workgroups that own the tiles of this tile's row panel and
// column panel to have finished squaring t - 1 (their words, monotone within
// a launch, reach `want`).  Those are also the only readers of this tile's
// entries of D_{t-1}, so the overwrite of D_{t-1}'s buffer at t + 1 is safe.
__device__ void panel_wait(const unsigned* words, unsigned want, int nt, int* err, int* latch,
                           int spin_limit, unsigned epoch) {
    const int I = blockIdx.x / nt, J = blockIdx.x % nt;
    for (int polls = 0;; ++polls) {
        int ok = 1;
        if ((int)threadIdx.x < 2 * nt) {
            const int src = (int)threadIdx.x < nt ? I * nt + (int)threadIdx.x
                                                  : ((int)threadIdx.x - nt) * nt + J;
            ok = ld_dev(words + src) >= want;
        }
        if (__syncthreads_and(ok)) break;
        if (spin_limit < 0 || polls >= spin_limit) {
            if (threadIdx.x == 0) report_timeout(err, latch, epoch);
            break;
        }
        __builtin_amdgcn_s_sleep(1);
    }
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
    // With the 16-bit mode enabled, also a 16-bit copy of D_0 and the gate:
    // the first barrier's OR tells every workgroup whether some entry falls
    // outside it.
    bool bad = false;
    {
        T* D0 = cur ? a.buf1 : a.buf0;
        const long ld0 = cur ? a.ld1 : a.ld0;
        for (long e = (long)blockIdx.x * RNT + tid; e < total; e += gthreads) {
            long i, j;
            flat_to_rc(e, n, total, i, j);
            T w = a.W[i * a.ldw + j];
            if (i == j && w > (T)0) w = (T)0;
            st_dev(D0 + i * ld0 + j, w);
            if constexpr (std::is_same_v<T, int32_t>) {
                if (a.gate_max >= 0) {
                    const bool absent = w == BTAS_I32_INF;
                    bad |= !absent && (w < 0 || w > a.gate_max);
                    st_dev(a.u16[0] + i * a.ld16 + j, absent ? U16_ABSENT : (uint16_t)w);
                }
            }
        }
    }
    unsigned bno = 1;
    const bool u16mode =
        grid_barrier(a.arrive, bno++, bad, a.flags, a.latch, a.spin_limit, a.epoch) == 0 &&
        a.gate_max >= 0;
    if constexpr (std::is_same_v<T, int32_t>) {
        if (u16mode) {
            solve_u16(a, smem_raw, bno);
            return;
        }
    }

    const int nt = (n + RT - 1) / RT;
    const int kpad = (n + 7) & ~7;
    const int r = tid / RT, c = tid % RT;
    int steps = 0;
    const bool dataflow = !a.early && (int)gridDim.x == nt * nt && 2 * nt <= RNT;
    unsigned* dwords = a.arrive;  // one word per workgroup, tags rising within the launch
    for (int t = 1; t <= a.nsq; ++t) {
        if (dataflow && t > 1)
            panel_wait(dwords, a.epoch << 8 | (unsigned)t << 1, nt, a.flags, a.latch, a.spin_limit,
                       a.epoch);
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
        int any = 1;
        if (dataflow) {
            asm volatile("s_waitcnt vmcnt(0)" ::: "memory");  // this wave's stores are performed
            __syncthreads();
            if (tid == 0) st_dev(dwords + blockIdx.x, a.epoch << 8 | (unsigned)(t + 1) << 1);
        } else {
            any = grid_barrier(a.arrive, bno++, changed, a.flags, a.latch, a.spin_limit, a.epoch);
        }
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
hipError_t launch_typed(int n, const void* W, long ldw, void* D, long ldd, void* ws, void* tagws,
                        int T_, bool early, int* flags, int* latch, int num_cus, int spin_limit,
                        bool allow_u16, unsigned epoch, hipStream_t s) {
    ResidentArgs<T> a;
    a.tag[0] = a.tag[1] = nullptr;
    a.cw = nullptr;
    a.gate_max = -1;
    a.ld16 = (n + 7) & ~7;
    a.u16[0] = a.u16[1] = nullptr;
    if (std::is_same_v<T, int32_t> && allow_u16 && n >= 2) {
        a.gate_max = 65534 / (2 * (n - 1));
        const size_t part = ((size_t)n * n * 4 + 255) / 256 * 256;
        const size_t half = ((size_t)n * a.ld16 * 2 + 255) / 256 * 256;
        a.u16[0] = reinterpret_cast<uint16_t*>((char*)ws + part);
        a.u16[1] = reinterpret_cast<uint16_t*>((char*)ws + part + half);
    }
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
    a.epoch = epoch;
    const size_t lds = resident_lds_bytes(n);
    // Workgroups per CU depend only on the LDS size (k padded to 8): the
    // occupancy query runs once per size, not on every call.
    const void* kernel = reinterpret_cast<const void*>(apsp_resident_kernel<T>);
    static std::atomic<int> per_cu_cache[RESIDENT_MAX_N / 8 + 2];
    const int slot = ((n + 7) & ~7) / 8;
    int per_cu = per_cu_cache[slot].load(std::memory_order_relaxed);
    if (per_cu == 0) {
        const hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, RNT, lds);
        if (e != hipSuccess) return e;
        if (per_cu < 1) return hipErrorInvalidConfiguration;
        per_cu_cache[slot].store(per_cu, std::memory_order_relaxed);
    }
    const int nt = (n + RT - 1) / RT;
    long grid = (long)per_cu * num_cus;
    if (grid > (long)nt * nt) grid = (long)nt * nt;
    if (grid > RESIDENT_MAX_GRID) grid = RESIDENT_MAX_GRID;
    void* args[] = {&a};
    if (tagws != nullptr && a.gate_max < 0 && T_ < RESIDENT_TAG_STEPS) {
        // One workgroup per tile, if that many can be resident.
        static std::atomic<int> tag_cu_cache[RESIDENT_MAX_N / 8 + 2];
        int tag_cu = tag_cu_cache[slot].load(std::memory_order_relaxed);
        if (tag_cu == 0) {
            const hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(
                &tag_cu, reinterpret_cast<const void*>(apsp_tagged_kernel<T>), RNT, lds);
            if (e != hipSuccess) return e;
            tag_cu = tag_cu < 1 ? -1 : tag_cu;
            tag_cu_cache[slot].store(tag_cu, std::memory_order_relaxed);
        }
        if ((long)tag_cu * num_cus >= (long)nt * nt && (long)nt * nt <= RESIDENT_MAX_GRID) {
            uint64_t* tw = static_cast<uint64_t*>(tagws);
            constexpr long region = (long)RESIDENT_MAX_N * RESIDENT_MAX_N;
            for (int i = 0; i < 2; ++i) a.tag[i] = tw + i * region;
            a.cw = tw + 2 * region;
            return hipLaunchCooperativeKernel(reinterpret_cast<const void*>(apsp_tagged_kernel<T>),
                                              dim3((unsigned)(nt * nt)), dim3(RNT), args,
                                              (unsigned)lds, s);
        }
    }
    return hipLaunchCooperativeKernel(kernel,
                                      dim3((unsigned)grid), dim3(RNT), args, (unsigned)lds, s);
}

// Graphs of at most 64 vertices: the whole solve in one workgroup, both
// ping-pong matrices in LDS, a workgroup barrier between squarings (no
// device-wide one).
template <typename T>
__global__ __launch_bounds__(LDS_SOLVE_NT) void apsp_lds_kernel(int n, const T* __restrict__ W, long ldw,
                                                                T* D, long ldd, int nsq, int early,
                                                                int* flags) {
    __shared__ __align__(16) LdsSolveBuffers<T> sm;
    const int steps = lds_solve_graph<T>(n, W, ldw, D, ldd, nsq, early, sm);
    if (threadIdx.x == 0) flags[1] = steps;
}

}  // namespace

size_t resident_lds_bytes(int n) { return (size_t)2 * RT * (((n + 7) & ~7) + 4) * 4; }

size_t resident_ws_bytes(int dt, int n) {
    const size_t part = ((size_t)n * n * 4 + 255) / 256 * 256;
    if (dt != BTAS_INT32 || n <= 64 || n > RESIDENT_MAX_N) return part;
    const size_t half = ((size_t)n * ((n + 7) & ~7) * 2 + 255) / 256 * 256;
    return part + 2 * half;
}

size_t resident_tag_bytes() {
    return ((size_t)2 * RESIDENT_MAX_N * RESIDENT_MAX_N + (size_t)RESIDENT_TAG_STEPS * RESIDENT_MAX_GRID) * 8;
}

hipError_t launch_apsp_resident(int dt, int n, const void* W, long ldw, void* D, long ldd,
                                void* ws, void* tagws, int T, bool early, int* flags, int* latch,
                                int num_cus, int spin_limit, bool allow_u16, unsigned epoch,
                                hipStream_t s) {
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
        return launch_typed<float>(n, W, ldw, D, ldd, ws, tagws, T, early, flags, latch, num_cus,
                                   spin_limit, false, epoch, s);
    return launch_typed<int32_t>(n, W, ldw, D, ldd, ws, tagws, T, early, flags, latch, num_cus,
                                 spin_limit, allow_u16, epoch, s);
}

}  // namespace btas
