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
//    the bound is VALU issue.  Each term costs one add; two terms are folded
//    into the accumulator with one three-input min/max (v_min3_* / v_max3_*).
//  * A workgroup owns a BM x BN macro-tile of C; each thread owns a TM x TN
//    register tile split into 4-wide groups so that LDS reads are 128-bit.
//  * A (BM x BK) and B (BK x BN) are staged row-major in padded LDS,
//    double-buffered: the next k-block is fetched from HBM into registers
//    while the current one is consumed, one barrier per block.
//  * Ragged m/n/k edges are filled with the absent value, which never wins
//    the (+)-reduction, so tile boundaries need no special compute path.
//  * Workgroup ids are remapped so that each XCD (own L2) receives a
//    contiguous band of tiles, then swizzled in groups of tile rows so that
//    co-resident workgroups share A and B panels.
//  * int32 operands that all fit in +-(2^23-1) run on the binary32 pipeline
//    (exact; see gemm_tile.h).  The choice is made per launch on the device
//    from a flag written by a range scan or by the previous squaring step, so
//    the host never waits for it.
#include <hip/hip_runtime.h>

#include <type_traits>

#include "gemm_tile.h"
#include "kernels.h"

namespace btas {

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
__global__ __launch_bounds__(Cfg::NT) void tropical_gemm_kernel(TileArgs<T> a,
                                                                 const int* wide_in) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const int nbm = (a.m + Cfg::BM - 1) / Cfg::BM;
    const int nbn = (a.n + Cfg::BN - 1) / Cfg::BN;
    int tm, tn;
    tile_of(blockIdx.x, nbm * nbn, nbm, nbn, tm, tn);
    if constexpr (std::is_same_v<T, int32_t>) {
        if (wide_in != nullptr && *wide_in == 0) {
            GemmTile<Cfg, T, float, SR, VEC>::run(a, tm * Cfg::BM, tn * Cfg::BN, smem_raw);
            return;
        }
    }
    GemmTile<Cfg, T, T, SR, VEC>::run(a, tm * Cfg::BM, tn * Cfg::BN, smem_raw);
}

template <typename Cfg, typename T, int SR>
static hipError_t launch_cfg(const GemmArgs& g, hipStream_t s) {
    const int nbm = (g.m + Cfg::BM - 1) / Cfg::BM;
    const int nbn = (g.n + Cfg::BN - 1) / Cfg::BN;
    const long nb = (long)nbm * nbn;
    if (nb == 0) return hipSuccess;
    if (nb > 0x7FFFFFFFL) return hipErrorInvalidValue;
    const bool vec = (g.lda % 4 == 0) && (g.ldb % 4 == 0) && (g.ldci % 4 == 0) &&
                     (g.ldco % 4 == 0) && (((uintptr_t)g.A | (uintptr_t)g.B |
                                            (uintptr_t)g.Cin | (uintptr_t)g.Cout) % 16 == 0);
    TileArgs<T> a{g.m, g.n, g.k, (const T*)g.A, g.lda, (const T*)g.B, g.ldb, (const T*)g.Cin,
                  g.ldci, (T*)g.Cout, g.ldco, g.changed, g.wide_out};
    dim3 grid((unsigned)nb), block(Cfg::NT);
    if (vec)
        hipLaunchKernelGGL((tropical_gemm_kernel<Cfg, T, SR, true>), grid, block, Cfg::lds_bytes,
                           s, a, g.wide_in);
    else
        hipLaunchKernelGGL((tropical_gemm_kernel<Cfg, T, SR, false>), grid, block,
                           Cfg::lds_bytes, s, a, g.wide_in);
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
