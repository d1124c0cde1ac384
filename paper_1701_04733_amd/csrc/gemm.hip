// Tropical GEMM for gfx950:  Cout <- Cin (+) A (.) B   (min-plus / max-plus).
//
// The product is the min-plus form of the matrix-product listing of Sec. IV
// (z_ij <- min(z_ij, min_k x_ik + y_kj)), generalised to max-plus and to an
// out-of-place accumulator so that one kernel serves both the BLAS-style call
// (Cin == Cout == C) and a squaring step of APSP (A == B == Cin == D_{t-1},
// Cout == D_t, plus a "did anything change" flag for early exit).
//
// Design (gfx950, wave64, 4 SIMD16 per CU, 160 KB LDS):
//  * (min,+) is not a multiply-accumulate, so there is no matrix-core path;
//    the roofline is VALU issue.  Each term costs one add; two terms are
//    folded into the accumulator with one three-input min/max
//    (v_min3_* / v_max3_*), i.e. 1.5 VALU instructions per term.
//  * A workgroup owns a BM x BN macro-tile of C; each thread owns a TM x TN
//    register tile split into 4-wide groups (rows ty*4.. and BM/2+ty*4.. for
//    TM = 8) so that LDS reads are 128-bit and conflict-free.
//  * A is staged row-major (BM x BK, padded) and B row-major (BK x BN,
//    padded) in LDS, double-buffered: the next k-block is fetched from HBM
//    into registers while the current one is consumed, one barrier per block.
//  * Ragged m/n/k edges are filled with the absent value, which never wins
//    the (+)-reduction, so tile boundaries need no special compute path.
//  * Workgroup ids are remapped so that each XCD (own L2) receives a
//    contiguous band of tiles, then swizzled in groups of tile rows so that
//    co-resident workgroups share A and B panels.
#include <hip/hip_runtime.h>

#include "kernels.h"
#include "semiring.h"

namespace btas {

template <typename T>
using v4 = T __attribute__((ext_vector_type(4)));

template <int BM_, int BN_, int BK_, int TM_, int TN_>
struct GemmCfg {
    static constexpr int BM = BM_, BN = BN_, BK = BK_, TM = TM_, TN = TN_;
    static constexpr int TXN = BN / TN;          // threads along n
    static constexpr int TYN = BM / TM;          // threads along m
    static constexpr int NT = TXN * TYN;         // threads per workgroup
    static constexpr int RG = TM / 4;            // 4-row groups per thread
    static constexpr int CG = TN / 4;            // 4-col groups per thread
    static constexpr int APAD = 4, BPAD = 4;
    static constexpr int LDA_S = BK + APAD;      // LDS row stride of A tile
    static constexpr int LDB_S = BN + BPAD;      // LDS row stride of B tile
    static constexpr int A_VECS = BM * BK / 4;   // float4s in an A tile
    static constexpr int B_VECS = BK * BN / 4;
    static constexpr int LA = A_VECS / NT;       // per-thread vector loads
    static constexpr int LB = B_VECS / NT;
    static_assert(TM % 4 == 0 && TN % 4 == 0, "register tile is built from 4-wide groups");
    static_assert(BK % 4 == 0, "k-block is consumed in quads");
    static_assert(A_VECS % NT == 0 && B_VECS % NT == 0, "tile loads must split evenly");
    static constexpr size_t lds_bytes = 2 * (BM * LDA_S + BK * LDB_S) * 4;
};

// Tile index of workgroup `bid`: XCD-contiguous bands, then grouped rows.
__device__ __forceinline__ void tile_of(int bid, int nb, int nbm, int nbn, int& tm, int& tn) {
    constexpr int NXCD = 8;
    const int per = nb / NXCD;
    if (bid < per * NXCD) bid = (bid % NXCD) * per + bid / NXCD;
    constexpr int GROUP_M = 8;
    const int group = GROUP_M * nbn;
    const int gid = bid / group;
    const int first_m = gid * GROUP_M;
    const int gsz = min(nbm - first_m, GROUP_M);
    const int in_g = bid - gid * group;
    tm = first_m + in_g % gsz;
    tn = in_g / gsz;
}

template <typename Cfg, typename T, int SR, bool VEC>
struct GemmTile {
    using R = Ring<SR, T>;

    // HBM -> registers for one k-block.
    __device__ __forceinline__ static void load_global(v4<T> (&ra)[Cfg::LA], v4<T> (&rb)[Cfg::LB],
                                                       const T* __restrict__ A, long lda,
                                                       const T* __restrict__ B, long ldb, int m,
                                                       int n, int k, int m0, int n0, int k0,
                                                       bool interior, int tid) {
        const T z = R::absent();
#pragma unroll
        for (int i = 0; i < Cfg::LA; ++i) {
            const int l = tid + i * Cfg::NT;
            const int row = l / (Cfg::BK / 4);
            const int kq = l % (Cfg::BK / 4);
            const int gr = m0 + row, gc = k0 + kq * 4;
            if (VEC && interior) {
                ra[i] = *reinterpret_cast<const v4<T>*>(A + (long)gr * lda + gc);
            } else {
#pragma unroll
                for (int e = 0; e < 4; ++e)
                    ra[i][e] = (gr < m && gc + e < k) ? A[(long)gr * lda + gc + e] : z;
            }
        }
#pragma unroll
        for (int i = 0; i < Cfg::LB; ++i) {
            const int l = tid + i * Cfg::NT;
            const int row = l / (Cfg::BN / 4);
            const int nq = l % (Cfg::BN / 4);
            const int gr = k0 + row, gc = n0 + nq * 4;
            if (VEC && interior) {
                rb[i] = *reinterpret_cast<const v4<T>*>(B + (long)gr * ldb + gc);
            } else {
#pragma unroll
                for (int e = 0; e < 4; ++e)
                    rb[i][e] = (gr < k && gc + e < n) ? B[(long)gr * ldb + gc + e] : z;
            }
        }
    }

    // registers -> LDS buffer.
    __device__ __forceinline__ static void store_lds(const v4<T> (&ra)[Cfg::LA],
                                                     const v4<T> (&rb)[Cfg::LB], T* As, T* Bs,
                                                     int tid) {
#pragma unroll
        for (int i = 0; i < Cfg::LA; ++i) {
            const int l = tid + i * Cfg::NT;
            const int row = l / (Cfg::BK / 4);
            const int kq = l % (Cfg::BK / 4);
            *reinterpret_cast<v4<T>*>(As + row * Cfg::LDA_S + kq * 4) = ra[i];
        }
#pragma unroll
        for (int i = 0; i < Cfg::LB; ++i) {
            const int l = tid + i * Cfg::NT;
            const int row = l / (Cfg::BN / 4);
            const int nq = l % (Cfg::BN / 4);
            *reinterpret_cast<v4<T>*>(Bs + row * Cfg::LDB_S + nq * 4) = rb[i];
        }
    }

    // Consume one LDS k-block into the register tile.
    __device__ __forceinline__ static void compute(T (&acc)[Cfg::TM][Cfg::TN], const T* As,
                                                   const T* Bs, int tx, int ty) {
#pragma unroll 1
        for (int q = 0; q < Cfg::BK / 4; ++q) {
            v4<T> a[Cfg::TM];
#pragma unroll
            for (int r = 0; r < Cfg::TM; ++r) {
                const int row = (r / 4) * (Cfg::BM / Cfg::RG) + ty * 4 + (r % 4);
                a[r] = *reinterpret_cast<const v4<T>*>(As + row * Cfg::LDA_S + q * 4);
            }
#pragma unroll
            for (int kk = 0; kk < 4; kk += 2) {
                T b0[Cfg::TN], b1[Cfg::TN];
#pragma unroll
                for (int g = 0; g < Cfg::CG; ++g) {
                    const int col = g * (Cfg::BN / Cfg::CG) + tx * 4;
                    const v4<T> x0 = *reinterpret_cast<const v4<T>*>(
                        Bs + (q * 4 + kk) * Cfg::LDB_S + col);
                    const v4<T> x1 = *reinterpret_cast<const v4<T>*>(
                        Bs + (q * 4 + kk + 1) * Cfg::LDB_S + col);
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
                        acc[r][c] = R::add3(acc[r][c], R::mul(a[r][kk], b0[c]),
                                            R::mul(a[r][kk + 1], b1[c]));
            }
        }
    }
};

template <typename Cfg, typename T, int SR, bool VEC>
__global__ __launch_bounds__(Cfg::NT) void tropical_gemm_kernel(
    int m, int n, int k, const T* __restrict__ A, long lda, const T* __restrict__ B, long ldb,
    const T* Cin, long ldci, T* Cout, long ldco, int* __restrict__ changed) {
    using Tile = GemmTile<Cfg, T, SR, VEC>;
    using R = Ring<SR, T>;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    T* As0 = reinterpret_cast<T*>(smem_raw);
    T* Bs0 = As0 + Cfg::BM * Cfg::LDA_S;
    T* As1 = Bs0 + Cfg::BK * Cfg::LDB_S;
    T* Bs1 = As1 + Cfg::BM * Cfg::LDA_S;

    const int nbm = (m + Cfg::BM - 1) / Cfg::BM;
    const int nbn = (n + Cfg::BN - 1) / Cfg::BN;
    int tm, tn;
    tile_of(blockIdx.x, nbm * nbn, nbm, nbn, tm, tn);
    const int m0 = tm * Cfg::BM, n0 = tn * Cfg::BN;
    const int tid = threadIdx.x;
    const int tx = tid % Cfg::TXN, ty = tid / Cfg::TXN;
    const bool mn_interior = (m0 + Cfg::BM <= m) && (n0 + Cfg::BN <= n);

    T acc[Cfg::TM][Cfg::TN];
#pragma unroll
    for (int r = 0; r < Cfg::TM; ++r)
#pragma unroll
        for (int c = 0; c < Cfg::TN; ++c) acc[r][c] = R::absent();

    const int nkb = (k + Cfg::BK - 1) / Cfg::BK;
    v4<T> ra[Cfg::LA], rb[Cfg::LB];
    if (nkb > 0) {
        Tile::load_global(ra, rb, A, lda, B, ldb, m, n, k, m0, n0, 0,
                          mn_interior && Cfg::BK <= k, tid);
        Tile::store_lds(ra, rb, As0, Bs0, tid);
    }
    __syncthreads();
    for (int kb = 0; kb < nkb; ++kb) {
        const bool even = (kb & 1) == 0;
        const T* Acur = even ? As0 : As1;
        const T* Bcur = even ? Bs0 : Bs1;
        const bool more = kb + 1 < nkb;
        if (more) {
            const int k0 = (kb + 1) * Cfg::BK;
            Tile::load_global(ra, rb, A, lda, B, ldb, m, n, k, m0, n0, k0,
                              mn_interior && k0 + Cfg::BK <= k, tid);
        }
        Tile::compute(acc, Acur, Bcur, tx, ty);
        if (more) Tile::store_lds(ra, rb, even ? As1 : As0, even ? Bs1 : Bs0, tid);
        __syncthreads();
    }

    // Epilogue: finish the accumulator, (+)-combine with Cin, store to Cout.
    bool diff = false;
#pragma unroll
    for (int r = 0; r < Cfg::TM; ++r) {
        const int row = m0 + (r / 4) * (Cfg::BM / Cfg::RG) + ty * 4 + (r % 4);
        if (row >= m) continue;
#pragma unroll
        for (int g = 0; g < Cfg::CG; ++g) {
            const int col = n0 + g * (Cfg::BN / Cfg::CG) + tx * 4;
            if (VEC && mn_interior) {
                const v4<T> old = *reinterpret_cast<const v4<T>*>(Cin + (long)row * ldci + col);
                v4<T> nv;
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    nv[e] = R::add(old[e], R::finish(acc[r][g * 4 + e]));
                    diff |= bits_of(nv[e]) != bits_of(old[e]);
                }
                *reinterpret_cast<v4<T>*>(Cout + (long)row * ldco + col) = nv;
            } else {
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    if (col + e >= n) break;
                    const T old = Cin[(long)row * ldci + col + e];
                    const T nv = R::add(old, R::finish(acc[r][g * 4 + e]));
                    diff |= bits_of(nv) != bits_of(old);
                    Cout[(long)row * ldco + col + e] = nv;
                }
            }
        }
    }
    if (changed != nullptr && __any(diff)) {
        if ((threadIdx.x & 63) == 0) *changed = 1;
    }
}

using CfgL = GemmCfg<128, 128, 16, 8, 8>;  // large problems: 256 threads, 8x8 per thread
using CfgM = GemmCfg<64, 64, 16, 4, 4>;    // mid-size: 256 threads, 4x4 per thread
using CfgS = GemmCfg<32, 32, 16, 4, 4>;    // small / latency-bound: 64 threads

template <typename Cfg, typename T, int SR>
static hipError_t launch_cfg(const GemmArgs& a, hipStream_t s) {
    const int nbm = (a.m + Cfg::BM - 1) / Cfg::BM;
    const int nbn = (a.n + Cfg::BN - 1) / Cfg::BN;
    const long nb = (long)nbm * nbn;
    if (nb == 0) return hipSuccess;
    if (nb > 0x7FFFFFFFL) return hipErrorInvalidValue;
    const bool vec = (a.lda % 4 == 0) && (a.ldb % 4 == 0) && (a.ldci % 4 == 0) &&
                     (a.ldco % 4 == 0) && (((uintptr_t)a.A | (uintptr_t)a.B |
                                            (uintptr_t)a.Cin | (uintptr_t)a.Cout) % 16 == 0);
    dim3 grid((unsigned)nb), block(Cfg::NT);
    if (vec)
        hipLaunchKernelGGL((tropical_gemm_kernel<Cfg, T, SR, true>), grid, block, Cfg::lds_bytes,
                           s, a.m, a.n, a.k, (const T*)a.A, a.lda, (const T*)a.B, a.ldb,
                           (const T*)a.Cin, a.ldci, (T*)a.Cout, a.ldco, a.changed);
    else
        hipLaunchKernelGGL((tropical_gemm_kernel<Cfg, T, SR, false>), grid, block,
                           Cfg::lds_bytes, s, a.m, a.n, a.k, (const T*)a.A, a.lda,
                           (const T*)a.B, a.ldb, (const T*)a.Cin, a.ldci, (T*)a.Cout, a.ldco,
                           a.changed);
    return hipGetLastError();
}

template <typename T, int SR>
static hipError_t launch_typed(const GemmArgs& a, int cfg, hipStream_t s) {
    if (cfg < 0) cfg = pick_gemm_cfg(a.m, a.n, a.k);
    switch (cfg) {
        case GEMM_CFG_L: return launch_cfg<CfgL, T, SR>(a, s);
        case GEMM_CFG_M: return launch_cfg<CfgM, T, SR>(a, s);
        case GEMM_CFG_S: return launch_cfg<CfgS, T, SR>(a, s);
        default: return hipErrorInvalidValue;
    }
}

int pick_gemm_cfg(int m, int n, int /*k*/) {
    // Enough 128x128 tiles to give every CU two workgroups -> large tiles
    // (best arithmetic intensity); otherwise trade intensity for parallelism.
    const long tl = (long)((m + 127) / 128) * ((n + 127) / 128);
    if (tl >= 512) return GEMM_CFG_L;
    const long tmid = (long)((m + 63) / 64) * ((n + 63) / 64);
    if (tmid >= 256) return GEMM_CFG_M;
    return GEMM_CFG_S;
}

hipError_t launch_gemm(int sr, int dt, const GemmArgs& a, int cfg, hipStream_t s) {
    if (dt == BTAS_FLOAT32)
        return sr == BTAS_MIN_PLUS ? launch_typed<float, BTAS_MIN_PLUS>(a, cfg, s)
                                   : launch_typed<float, BTAS_MAX_PLUS>(a, cfg, s);
    return sr == BTAS_MIN_PLUS ? launch_typed<int32_t, BTAS_MIN_PLUS>(a, cfg, s)
                               : launch_typed<int32_t, BTAS_MAX_PLUS>(a, cfg, s);
}

}  // namespace btas
