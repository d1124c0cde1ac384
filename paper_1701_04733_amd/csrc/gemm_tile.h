// One output macro-tile of the tropical product, shared by the single-GEMM
// kernel and the grouped (batched / served APSP) kernel.
//
//   Cout[m0.., n0..] <- Cin (+) A (.) B     over a BM x BN tile, k fully reduced.
//
// The paper's matrix product (Sec. IV, min-plus form of the matrix-product
// listing) assigns sub-matrices of the output to threads; here a workgroup
// owns a BM x BN tile and each thread a TM x TN register tile, with A and B
// panels staged through LDS.
//
// Storage type T (the caller's element type) and compute type CT may differ:
// int32 data whose finite values all satisfy |x| <= 2^23-1 is computed on the
// binary32 pipeline (CT = float), which is exact because every such value and
// every sum of two of them (|s| <= 2^24-2) is an exactly representable
// binary32 integer, and the absent values map to +-inf.  That path issues the
// (.) as a 2-operand float add, which gfx950 dual-issues, instead of a
// saturating integer add with a clamp modifier, which it does not.
#pragma once

#include <hip/hip_runtime.h>

#include <type_traits>

#include "semiring.h"

namespace btas {

template <typename T>
using v4 = T __attribute__((ext_vector_type(4)));

// Largest magnitude of a finite int32 element that the binary32 path accepts.
constexpr int32_t FP32_EXACT_MAX = (1 << 23) - 1;

template <int BM_, int BN_, int BK_, int TM_, int TN_, int NBUF_ = 2>
struct GemmCfg {
    static constexpr int BM = BM_, BN = BN_, BK = BK_, TM = TM_, TN = TN_;
    static constexpr int NBUF = NBUF_;           // LDS buffers: 2 = double-buffered, 1 = single
    static constexpr int TXN = BN / TN;          // threads along n
    static constexpr int TYN = BM / TM;          // threads along m
    static constexpr int NT = TXN * TYN;         // threads per workgroup
    static constexpr int CG = TN / 4;            // 4-col groups per thread
    static constexpr int APAD = 4, BPAD = 4;
    static constexpr int LDA_S = BK + APAD;      // LDS row stride of the A tile
    static constexpr int LDB_S = BN + BPAD;      // LDS row stride of the B tile
    static constexpr int A_VECS = BM * BK / 4;   // 4-vectors in an A tile
    static constexpr int B_VECS = BK * BN / 4;
    static constexpr int LA = A_VECS / NT;       // per-thread vector loads
    static constexpr int LB = B_VECS / NT;
    static_assert(TM % 4 == 0 && TN % 4 == 0, "register tile is built from 4-wide groups");
    static_assert(BK % 4 == 0, "k-block is consumed in quads");
    static_assert(A_VECS % NT == 0 && B_VECS % NT == 0, "tile loads must split evenly");
    static_assert(NBUF == 1 || NBUF == 2, "one or two LDS buffers");
    static constexpr size_t lds_bytes = NBUF * (BM * LDA_S + BK * LDB_S) * 4;
    // Tile row of a thread's r-th register row: rows are strided by TYN, so
    // the lanes of a wave read consecutive A rows, whose padded LDS rows
    // start in distinct banks (no conflicts for up to 8 distinct rows).
    __device__ __forceinline__ static int row_of(int r, int ty) { return r * TYN + ty; }
};

using CfgL = GemmCfg<128, 128, 16, 8, 8>;  // large problems: 256 threads, 8x8 per thread
// Large products whose full 256x256 tiles fill rounds of one per CU:
// 1024 threads, 8x8 per thread, direct loads only.  One workgroup per CU
// whose 16 waves share each k-block through one barrier: the A and B panels
// a CU reads per output halve, and the workgroups that share panels stay in
// step (8192^3: 4.5-4.8 instead of 8.0-8.2 GB fetched from beyond the L2).
using CfgXL = GemmCfg<256, 256, 16, 8, 8>;
using CfgM = GemmCfg<64, 64, 16, 4, 4>;    // mid-size: 256 threads, 4x4 per thread
using CfgS = GemmCfg<32, 32, 16, 4, 4>;    // small / latency-bound: 64 threads
// One wave computes a 64x64 tile with the 8x8 register tile of CfgL.  The
// 8-deep k-block keeps the prefetch registers at CfgL's count (about 160 VGPRs,
// three waves per SIMD); its double-buffered LDS (10.5 KB) lets LDS hold as
// many of these workgroups as the register file does.
using CfgW = GemmCfg<64, 64, 8, 8, 8>;

// Element conversion between storage and compute types.
template <typename T, typename CT, int SR>
struct Conv {
    __device__ __forceinline__ static CT in(T x) { return x; }
    __device__ __forceinline__ static T out(CT acc) { return Ring<SR, T>::finish(acc); }
};

template <int SR>
struct Conv<int32_t, float, SR> {
    __device__ __forceinline__ static float in(int32_t x) {
        return x == Ring<SR, int32_t>::absent() ? Ring<SR, float>::absent() : (float)x;
    }
    // acc is an exact integer of magnitude < 2^24, or the absent infinity.
    __device__ __forceinline__ static int32_t out(float acc) {
        return __builtin_isinf(acc) ? Ring<SR, int32_t>::absent() : (int32_t)acc;
    }
};

template <typename T>
struct TileArgs {
    int m, n, k;
    const T* A;
    long lda;
    const T* B;
    long ldb;
    const T* Cin;   // null: the accumulator starts from the absent value (split-K partials)
    long ldci;
    T* Cout;
    long ldco;
    int* changed;   // set to 1 if an output differs bitwise from Cin (may be null)
    int* wide_out;  // int32: set to 1 if a finite output exceeds FP32_EXACT_MAX (may be null)
};

template <typename Cfg, typename T, typename CT, int SR, bool VEC>
struct GemmTile {
    using R = Ring<SR, CT>;
    using Cv = Conv<T, CT, SR>;

    // HBM -> registers (converted to the compute type) for one k-block.
    __device__ __forceinline__ static void load_global(v4<CT> (&ra)[Cfg::LA], v4<CT> (&rb)[Cfg::LB],
                                                       const TileArgs<T>& a, int m0, int n0,
                                                       int k0, bool interior, int tid) {
        const CT z = R::absent();
#pragma unroll
        for (int i = 0; i < Cfg::LA; ++i) {
            const int l = tid + i * Cfg::NT;
            const int row = l / (Cfg::BK / 4);
            const int kq = l % (Cfg::BK / 4);
            const int gr = m0 + row, gc = k0 + kq * 4;
            if (VEC && interior) {
                const v4<T> x = *reinterpret_cast<const v4<T>*>(a.A + (long)gr * a.lda + gc);
#pragma unroll
                for (int e = 0; e < 4; ++e) ra[i][e] = Cv::in(x[e]);
            } else {
#pragma unroll
                for (int e = 0; e < 4; ++e)
                    ra[i][e] = (gr < a.m && gc + e < a.k) ? Cv::in(a.A[(long)gr * a.lda + gc + e]) : z;
            }
        }
#pragma unroll
        for (int i = 0; i < Cfg::LB; ++i) {
            const int l = tid + i * Cfg::NT;
            const int row = l / (Cfg::BN / 4);
            const int nq = l % (Cfg::BN / 4);
            const int gr = k0 + row, gc = n0 + nq * 4;
            if (VEC && interior) {
                const v4<T> x = *reinterpret_cast<const v4<T>*>(a.B + (long)gr * a.ldb + gc);
#pragma unroll
                for (int e = 0; e < 4; ++e) rb[i][e] = Cv::in(x[e]);
            } else {
#pragma unroll
                for (int e = 0; e < 4; ++e)
                    rb[i][e] = (gr < a.k && gc + e < a.n) ? Cv::in(a.B[(long)gr * a.ldb + gc + e]) : z;
            }
        }
    }

    // registers -> LDS buffer.
    __device__ __forceinline__ static void store_lds(const v4<CT> (&ra)[Cfg::LA],
                                                     const v4<CT> (&rb)[Cfg::LB], CT* As, CT* Bs,
                                                     int tid) {
#pragma unroll
        for (int i = 0; i < Cfg::LA; ++i) {
            const int l = tid + i * Cfg::NT;
            const int row = l / (Cfg::BK / 4);
            const int kq = l % (Cfg::BK / 4);
            *reinterpret_cast<v4<CT>*>(As + row * Cfg::LDA_S + kq * 4) = ra[i];
        }
#pragma unroll
        for (int i = 0; i < Cfg::LB; ++i) {
            const int l = tid + i * Cfg::NT;
            const int row = l / (Cfg::BN / 4);
            const int nq = l % (Cfg::BN / 4);
            *reinterpret_cast<v4<CT>*>(Bs + row * Cfg::LDB_S + nq * 4) = rb[i];
        }
    }

    // Consume one LDS k-block into the register tile.  The quad loop is kept
    // rolled so that only one quad's operands are live (about 150 VGPRs for
    // the 8x8 tile, three waves per SIMD); each quad folds two k-steps per
    // three-input min/max.
    template <int LDA = Cfg::LDA_S, int LDB = Cfg::LDB_S>
    __device__ __forceinline__ static void compute(CT (&acc)[Cfg::TM][Cfg::TN], const CT* As,
                                                   const CT* Bs, int tx, int ty) {
#pragma unroll 1
        for (int q = 0; q < Cfg::BK / 4; ++q) {
            v4<CT> av[Cfg::TM];
#pragma unroll
            for (int r = 0; r < Cfg::TM; ++r) {
                const int row = Cfg::row_of(r, ty);
                av[r] = *reinterpret_cast<const v4<CT>*>(As + row * LDA + q * 4);
            }
#pragma unroll
            for (int kk = 0; kk < 4; kk += 2) {
                CT b0[Cfg::TN], b1[Cfg::TN];
#pragma unroll
                for (int g = 0; g < Cfg::CG; ++g) {
                    const int col = g * (Cfg::BN / Cfg::CG) + tx * 4;
                    const v4<CT> x0 = *reinterpret_cast<const v4<CT>*>(
                        Bs + (q * 4 + kk) * LDB + col);
                    const v4<CT> x1 = *reinterpret_cast<const v4<CT>*>(
                        Bs + (q * 4 + kk + 1) * LDB + col);
#pragma unroll
                    for (int e = 0; e < 4; ++e) {
                        b0[g * 4 + e] = x0[e];
                        b1[g * 4 + e] = x1[e];
                    }
                }
#pragma unroll
                for (int r = 0; r < Cfg::TM; ++r)
#pragma unroll
                    for (int c = 0; c < Cfg::TN; ++c)
                        acc[r][c] = R::add3(acc[r][c], R::mul(av[r][kk], b0[c]),
                                            R::mul(av[r][kk + 1], b1[c]));
            }
        }
    }

    // The whole tile: k loop with double-buffered LDS, then the epilogue.
    __device__ __forceinline__ static void run(const TileArgs<T>& a, int m0, int n0,
                                               unsigned char* smem) {
        using RT = Ring<SR, T>;
        CT* As0 = reinterpret_cast<CT*>(smem);
        CT* Bs0 = As0 + Cfg::BM * Cfg::LDA_S;
        CT* As1 = Cfg::NBUF == 2 ? Bs0 + Cfg::BK * Cfg::LDB_S : As0;
        CT* Bs1 = Cfg::NBUF == 2 ? As1 + Cfg::BM * Cfg::LDA_S : Bs0;
        const int tid = threadIdx.x;
        const int tx = tid % Cfg::TXN, ty = tid / Cfg::TXN;
        const bool mn_interior = (m0 + Cfg::BM <= a.m) && (n0 + Cfg::BN <= a.n);

        CT acc[Cfg::TM][Cfg::TN];
#pragma unroll
        for (int r = 0; r < Cfg::TM; ++r)
#pragma unroll
            for (int c = 0; c < Cfg::TN; ++c) acc[r][c] = R::absent();

        const int nkb = (a.k + Cfg::BK - 1) / Cfg::BK;
        v4<CT> ra[Cfg::LA], rb[Cfg::LB];
        if (nkb > 0) {
            load_global(ra, rb, a, m0, n0, 0, mn_interior && Cfg::BK <= a.k, tid);
            store_lds(ra, rb, As0, Bs0, tid);
        }
        __syncthreads();
        for (int kb = 0; kb < nkb; ++kb) {
            const bool even = Cfg::NBUF == 1 || (kb & 1) == 0;
            const bool more = kb + 1 < nkb;
            if (more) {
                const int k0 = (kb + 1) * Cfg::BK;
                load_global(ra, rb, a, m0, n0, k0, mn_interior && k0 + Cfg::BK <= a.k, tid);
            }
            compute(acc, even ? As0 : As1, even ? Bs0 : Bs1, tx, ty);
            if constexpr (Cfg::NBUF == 1) {
                // every thread has read the block before it is overwritten
                if (more) {
                    __syncthreads();
                    store_lds(ra, rb, As0, Bs0, tid);
                }
            } else {
                if (more) store_lds(ra, rb, even ? As1 : As0, even ? Bs1 : Bs0, tid);
            }
            __syncthreads();
        }

        // Epilogue: finish the accumulator, (+)-combine with Cin, store Cout.
        bool diff = false, wide = false;
#pragma unroll
        for (int r = 0; r < Cfg::TM; ++r) {
            const int row = m0 + Cfg::row_of(r, ty);
            if (row >= a.m) continue;
#pragma unroll
            for (int g = 0; g < Cfg::CG; ++g) {
                const int col = n0 + g * (Cfg::BN / Cfg::CG) + tx * 4;
                if (VEC && mn_interior) {
                    v4<T> old;
                    if (a.Cin != nullptr) {
                        old = *reinterpret_cast<const v4<T>*>(a.Cin + (long)row * a.ldci + col);
                    } else {
#pragma unroll
                        for (int e = 0; e < 4; ++e) old[e] = RT::absent();
                    }
                    v4<T> nv;
#pragma unroll
                    for (int e = 0; e < 4; ++e) {
                        nv[e] = RT::add(old[e], Cv::out(acc[r][g * 4 + e]));
                        diff |= bits_of(nv[e]) != bits_of(old[e]);
                        wide |= is_wide(nv[e]);
                    }
                    *reinterpret_cast<v4<T>*>(a.Cout + (long)row * a.ldco + col) = nv;
                } else {
#pragma unroll
                    for (int e = 0; e < 4; ++e) {
                        if (col + e >= a.n) break;
                        const T old = a.Cin != nullptr ? a.Cin[(long)row * a.ldci + col + e] : RT::absent();
                        const T nv = RT::add(old, Cv::out(acc[r][g * 4 + e]));
                        diff |= bits_of(nv) != bits_of(old);
                        wide |= is_wide(nv);
                        a.Cout[(long)row * a.ldco + col + e] = nv;
                    }
                }
            }
        }
        if (a.changed != nullptr && __any(diff) && (threadIdx.x & 63) == 0) *a.changed = 1;
        if (a.wide_out != nullptr && __any(wide) && (threadIdx.x & 63) == 0) *a.wide_out = 1;
    }

    __device__ __forceinline__ static bool is_wide(T x) {
        if constexpr (std::is_same_v<T, int32_t>) {
            return x != Ring<SR, T>::absent() && (x > FP32_EXACT_MAX || x < -FP32_EXACT_MAX);
        } else {
            return false;
        }
    }
};

// fp32 operands, every tile full (m % BM == n % BN == k % BK == 0, rows
// 16-byte aligned): A and B k-blocks go from global memory straight into LDS
// (gfx950 global_load_lds_dwordx4: each wave instruction fills 1 KB of LDS in
// lane order), so no registers hold the next block while the current one is
// consumed.  The LDS rows are therefore unpadded; with the register-row
// mapping of GemmCfg::row_of the lanes of a wave still read A rows that start
// in distinct banks, and B rows are read as contiguous 16-byte chunks.
//
// int32 storage on the binary32-exact path (every finite operand within
// +-(2^23-1)) uses the same kernel: the int32 bits land in LDS and each lane
// turns the four elements its own load wrote into binary32 before the
// k-block's barrier.  That conversion is a plain int-to-float of every
// element, absent values included: an absent operand becomes -+2^31 (the
// nearest binary32), so every term it enters has magnitude above 2^30 and
// loses to every finite sum (|s| <= 2^24 - 2), and the epilogue maps any
// accumulator of magnitude above 2^24 back to the absent value.
template <typename Cfg, int SR, typename T = float>
struct GemmTileDirect {
    static_assert(std::is_same_v<T, float> || std::is_same_v<T, int32_t>, "fp32 or int32 storage");
    using R = Ring<SR, float>;
    static constexpr int LDA = Cfg::BK, LDB = Cfg::BN;  // unpadded LDS rows
    static constexpr int NW = Cfg::NT / 64;              // waves per workgroup
    static constexpr int A_ROWS = 1024 / (Cfg::BK * 4);  // A rows per wave instruction
    static constexpr int B_ROWS = 1024 / (Cfg::BN * 4);  // B rows per wave instruction
    static constexpr int AI = Cfg::BM / A_ROWS / NW;     // instructions per wave per k-block
    static constexpr int BI = Cfg::BK / B_ROWS / NW;
    static_assert(AI >= 1 && BI >= 1 && Cfg::BM % (A_ROWS * NW) == 0 && Cfg::BK % (B_ROWS * NW) == 0,
                  "each wave moves whole 1 KB pieces of both k-block tiles");
    static constexpr size_t lds_bytes = 2 * (Cfg::BM * LDA + Cfg::BK * LDB) * 4;

    using lds_ptr = __attribute__((address_space(3))) void*;
    using gbl_ptr = __attribute__((address_space(1))) void*;

    __device__ __forceinline__ static void issue(const TileArgs<T>& a, int m0, int n0, int k0,
                                                 float* As, float* Bs) {
        const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
        for (int i = 0; i < AI; ++i) {
            const int rb = (w * AI + i) * A_ROWS;
            const int row = rb + lane / (Cfg::BK / 4), kq = lane % (Cfg::BK / 4);
            const T* src = a.A + (long)(m0 + row) * a.lda + k0 + kq * 4;
            __builtin_amdgcn_global_load_lds((gbl_ptr)src, (lds_ptr)(As + rb * LDA), 16, 0, 0);
        }
#pragma unroll
        for (int i = 0; i < BI; ++i) {
            const int rb = (w * BI + i) * B_ROWS;
            const int row = rb + lane / (Cfg::BN / 4), cq = lane % (Cfg::BN / 4);
            const T* src = a.B + (long)(k0 + row) * a.ldb + n0 + cq * 4;
            __builtin_amdgcn_global_load_lds((gbl_ptr)src, (lds_ptr)(Bs + rb * LDB), 16, 0, 0);
        }
    }

    // int32 storage: the lanes of this wave convert, in place, the pieces their
    // own loads wrote (lane L of an instruction wrote the 16 bytes at
    // base + 16 L), once the wave's loads have completed.
    __device__ __forceinline__ static void to_binary32(float* As, float* Bs) {
        if constexpr (std::is_same_v<T, int32_t>) {
            const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
            auto cvt = [](float* p) {
                const v4<int32_t> x = __builtin_bit_cast(v4<int32_t>, *reinterpret_cast<v4<float>*>(p));
                v4<float> f;
#pragma unroll
                for (int e = 0; e < 4; ++e) f[e] = (float)x[e];
                *reinterpret_cast<v4<float>*>(p) = f;
            };
#pragma unroll
            for (int i = 0; i < AI; ++i) cvt(As + (w * AI + i) * A_ROWS * LDA + lane * 4);
#pragma unroll
            for (int i = 0; i < BI; ++i) cvt(Bs + (w * BI + i) * B_ROWS * LDB + lane * 4);
        }
    }

    // Output element from Cin and the binary32 accumulator.
    __device__ __forceinline__ static T finish(T old, float acc, bool& wide) {
        if constexpr (std::is_same_v<T, int32_t>) {
            using RI = Ring<SR, int32_t>;
            const int32_t v = __builtin_fabsf(acc) > 16777216.0f ? RI::absent() : (int32_t)acc;
            const int32_t nv = RI::add(old, v);
            wide |= nv != RI::absent() && (nv > FP32_EXACT_MAX || nv < -FP32_EXACT_MAX);
            return nv;
        } else {
            return R::add(old, acc);
        }
    }

    // One LDS k-block into the register tile, two k-steps per iteration: the
    // A operands are read as k-pairs (8-byte LDS reads), which keeps the live
    // registers under the 128 that four waves per SIMD allow.
    __device__ __forceinline__ static void compute(float (&acc)[Cfg::TM][Cfg::TN], const float* As,
                                                   const float* Bs, int tx, int ty) {
        using v2 = float __attribute__((ext_vector_type(2)));
#pragma unroll 1
        for (int kp = 0; kp < Cfg::BK / 2; ++kp) {
            v2 av[Cfg::TM];
#pragma unroll
            for (int r = 0; r < Cfg::TM; ++r)
                av[r] = *reinterpret_cast<const v2*>(As + Cfg::row_of(r, ty) * LDA + kp * 2);
            float b0[Cfg::TN], b1[Cfg::TN];
#pragma unroll
            for (int g = 0; g < Cfg::CG; ++g) {
                const int col = g * (Cfg::BN / Cfg::CG) + tx * 4;
                const v4<float> x0 = *reinterpret_cast<const v4<float>*>(Bs + (kp * 2) * LDB + col);
                const v4<float> x1 = *reinterpret_cast<const v4<float>*>(Bs + (kp * 2 + 1) * LDB + col);
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    b0[g * 4 + e] = x0[e];
                    b1[g * 4 + e] = x1[e];
                }
            }
#pragma unroll
            for (int r = 0; r < Cfg::TM; ++r)
#pragma unroll
                for (int c = 0; c < Cfg::TN; ++c)
                    acc[r][c] = R::add3(acc[r][c], R::mul(av[r][0], b0[c]), R::mul(av[r][1], b1[c]));
        }
    }

    __device__ __forceinline__ static void run(const TileArgs<T>& a, int m0, int n0,
                                               unsigned char* smem) {
        float* As0 = reinterpret_cast<float*>(smem);
        float* Bs0 = As0 + Cfg::BM * LDA;
        float* As1 = Bs0 + Cfg::BK * LDB;
        float* Bs1 = As1 + Cfg::BM * LDA;
        const int tid = threadIdx.x;
        const int tx = tid % Cfg::TXN, ty = tid / Cfg::TXN;
        float acc[Cfg::TM][Cfg::TN];
#pragma unroll
        for (int r = 0; r < Cfg::TM; ++r)
#pragma unroll
            for (int c = 0; c < Cfg::TN; ++c) acc[r][c] = R::absent();
        const int nkb = a.k / Cfg::BK;
        if (nkb > 0) issue(a, m0, n0, 0, As0, Bs0);
        asm volatile("s_waitcnt vmcnt(0)" ::: "memory");  // this wave's pieces are in LDS
        if (nkb > 0) to_binary32(As0, Bs0);
        __syncthreads();                                   // and everyone else's
        for (int kb = 0; kb < nkb; ++kb) {
            const bool even = (kb & 1) == 0;
            const bool more = kb + 1 < nkb;
            if (more) issue(a, m0, n0, (kb + 1) * Cfg::BK, even ? As1 : As0, even ? Bs1 : Bs0);
            compute(acc, even ? As0 : As1, even ? Bs0 : Bs1, tx, ty);
            asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
            if (more) to_binary32(even ? As1 : As0, even ? Bs1 : Bs0);
            __syncthreads();
        }
        // Epilogue (every tile is interior): Cout = Cin (+) acc (Cin null: the
        // absent value, a split-K partial), changed flag.
        bool diff = false, wide = false;
#pragma unroll
        for (int r = 0; r < Cfg::TM; ++r) {
            const int row = m0 + Cfg::row_of(r, ty);
#pragma unroll
            for (int g = 0; g < Cfg::CG; ++g) {
                const int col = n0 + g * (Cfg::BN / Cfg::CG) + tx * 4;
                v4<T> old;
                if (a.Cin != nullptr) {
                    old = *reinterpret_cast<const v4<T>*>(a.Cin + (long)row * a.ldci + col);
                } else {
#pragma unroll
                    for (int e = 0; e < 4; ++e) old[e] = Ring<SR, T>::absent();
                }
                v4<T> nv;
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    nv[e] = finish(old[e], acc[r][g * 4 + e], wide);
                    diff |= bits_of(nv[e]) != bits_of(old[e]);
                }
                *reinterpret_cast<v4<T>*>(a.Cout + (long)row * a.ldco + col) = nv;
            }
        }
        if (a.changed != nullptr && __any(diff) && (threadIdx.x & 63) == 0) *a.changed = 1;
        if (a.wide_out != nullptr && __any(wide) && (threadIdx.x & 63) == 0) *a.wide_out = 1;
    }
};

}  // namespace btas
