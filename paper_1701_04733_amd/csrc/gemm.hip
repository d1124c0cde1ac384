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
//    while the current one is consumed, one barrier per block.  Products
//    whose 128x128 tiles are all full load the next k-block straight into
//    LDS instead (no staging registers): fp32, and int32 on the
//    binary32-exact path (each lane converts the elements its own load
//    wrote, in LDS, before the block's barrier).  Large such products whose
//    full 256x256 tiles fill rounds of one per CU use a 256x256 tile of 1024
//    threads instead: half the panel traffic per output, and the panels a
//    CU shares are read in step.
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

#include <algorithm>
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

// WIDE_ONLY: the launch that follows a direct-load int32 launch; it does the
// product only when the operands left the binary32-exact range.
template <typename Cfg, typename T, int SR, bool VEC, bool WIDE_ONLY = false>
__global__ __launch_bounds__(Cfg::NT) void tropical_gemm_kernel(TileArgs<T> a,
                                                                 const int* wide_in) {
    if constexpr (WIDE_ONLY) {
        if (*wide_in == 0) return;
    }
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

// Every tile full and 16-byte aligned: direct global -> LDS loads.  fp32, or
// int32 on the binary32-exact path (wide_in non-null: the workgroups return
// at once when the operands left that range, and the WIDE_ONLY launch of the
// staged kernel that follows does the product).
template <typename Cfg, int SR, typename T = float>
__global__ __launch_bounds__(Cfg::NT) __attribute__((amdgpu_waves_per_eu(4))) void tropical_gemm_direct_kernel(
    TileArgs<T> a, const int* wide_in) {
    if constexpr (std::is_same_v<T, int32_t>) {
        if (*wide_in != 0) return;
    }
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const int nbm = a.m / Cfg::BM, nbn = a.n / Cfg::BN;
    int tm, tn;
    tile_of(blockIdx.x, nbm * nbn, nbm, nbn, tm, tn);
    GemmTileDirect<Cfg, SR, T>::run(a, tm * Cfg::BM, tn * Cfg::BN, smem_raw);
}

// Split-K on the direct-load tile (fp32, every 128x128 tile full): for
// products with fewer tiles than the device holds workgroups (4 per CU), k
// is cut into S chunks so that about a whole number of rounds of workgroups
// runs; blockIdx.x = tile * S + chunk, the chunk's partial product goes to
// ws[chunk] (m x n, leading dimension n) and splitk_reduce_kernel combines
// them with Cin (bit-identical: the (+) is exact).
template <typename Cfg, int SR>
__global__ __launch_bounds__(Cfg::NT) __attribute__((amdgpu_waves_per_eu(4))) void tropical_gemm_direct_splitk_kernel(
    TileArgs<float> a, int S, int kc, float* ws) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const int nbn = a.n / Cfg::BN;
    const int tile = blockIdx.x / S, chunk = blockIdx.x - tile * S;
    const int tm = tile / nbn, tn = tile - tm * nbn;
    const int k0 = chunk * kc;
    TileArgs<float> p = a;
    p.A = a.A + k0;
    p.B = a.B + (long)k0 * a.ldb;
    p.k = min(kc, a.k - k0);
    p.Cin = nullptr;
    p.ldci = 0;
    p.Cout = ws + (long)chunk * a.m * a.n;
    p.ldco = a.n;
    p.changed = nullptr;
    p.wide_out = nullptr;
    GemmTileDirect<Cfg, SR>::run(p, tm * Cfg::BM, tn * Cfg::BN, smem_raw);
}

// Split-K: blockIdx.x = tile * S + chunk; the chunk's partial product goes to
// ws[chunk] (m x n, leading dimension n), Cin is not read.
template <typename Cfg, typename T, int SR, bool VEC>
__global__ __launch_bounds__(Cfg::NT) void tropical_gemm_splitk_kernel(TileArgs<T> a, int S, int kc,
                                                                        T* ws, const int* wide_in) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const int nbm = (a.m + Cfg::BM - 1) / Cfg::BM;
    const int nbn = (a.n + Cfg::BN - 1) / Cfg::BN;
    const int tile = blockIdx.x / S, chunk = blockIdx.x - tile * S;
    const int tm = tile / nbn, tn = tile - tm * nbn;
    (void)nbm;
    const int k0 = chunk * kc;
    TileArgs<T> p = a;
    p.A = a.A + k0;
    p.B = a.B + (long)k0 * a.ldb;
    p.k = min(kc, a.k - k0);
    p.Cin = nullptr;
    p.ldci = 0;
    p.Cout = ws + (long)chunk * a.m * a.n;
    p.ldco = a.n;
    p.changed = nullptr;
    p.wide_out = nullptr;
    if constexpr (std::is_same_v<T, int32_t>) {
        if (wide_in != nullptr && *wide_in == 0) {
            GemmTile<Cfg, T, float, SR, VEC>::run(p, tm * Cfg::BM, tn * Cfg::BN, smem_raw);
            return;
        }
    }
    GemmTile<Cfg, T, T, SR, VEC>::run(p, tm * Cfg::BM, tn * Cfg::BN, smem_raw);
}

// Cout = Cin (+) (+)_s ws[s]; sets the changed / wide flags like the tile epilogue.
template <typename T, int SR>
__global__ __launch_bounds__(256) void splitk_reduce_kernel(int m, int n, int S, const T* ws,
                                                             const T* Cin, long ldci, T* Cout,
                                                             long ldco, int* changed, int* wide_out) {
    using R = Ring<SR, T>;
    const long total = (long)m * n;
    bool diff = false, wide = false;
    for (long e = (long)blockIdx.x * blockDim.x + threadIdx.x; e < total;
         e += (long)gridDim.x * blockDim.x) {
        const long i = e / n, j = e - i * n;
        T acc = R::absent();
        for (int s = 0; s < S; ++s) acc = R::add(acc, ws[(long)s * total + e]);
        const T old = Cin[i * ldci + j];
        const T nv = R::add(old, acc);
        Cout[i * ldco + j] = nv;
        diff |= bits_of(nv) != bits_of(old);
        if constexpr (std::is_same_v<T, int32_t>)
            wide |= nv != R::absent() && (nv > FP32_EXACT_MAX || nv < -FP32_EXACT_MAX);
    }
    if (changed != nullptr && __any(diff) && (threadIdx.x & 63) == 0) *changed = 1;
    if (wide_out != nullptr && __any(wide) && (threadIdx.x & 63) == 0) *wide_out = 1;
}

// The XL tile runs one workgroup per CU (256 at once): products whose full
// 256x256 tiles fill their rounds of 256 to at least 90% take it.  A ragged
// last round leaves CUs idle that 128x128 tiles (four per CU) would still
// occupy: fp32 n=4096 (256 tiles) 72.4 against 68.4 Top/s, n=5120 (400)
// 58.5 against 62.6, n=8192 (1024) 73-75 against 71-72.
constexpr long XL_SLOTS = 256;
static bool xl_fills(long tiles) {
    if (tiles < XL_SLOTS) return false;
    const long rounds = (tiles + XL_SLOTS - 1) / XL_SLOTS;
    return tiles * 10 >= rounds * XL_SLOTS * 9;
}

template <typename Cfg>
static long tiles_for(int m, int n) {
    return (long)((m + Cfg::BM - 1) / Cfg::BM) * ((n + Cfg::BN - 1) / Cfg::BN);
}

// Tile configuration and split-K factor for an m x n x k product.  The aim
// is enough work to occupy the GPU: at least ~512 workgroups of 256 threads
// (two per CU).  Large outputs use 128x128 tiles; mid-size outputs 64x64
// tiles, with k split into chunks of at least 32 when there are fewer than
// 512 of them; tiny outputs (m or n <= 48) 32x32 tiles of 64 threads with
// k split the same way.
GemmPlan plan_gemm(int m, int n, int k) {
    GemmPlan p{GEMM_CFG_L, 1};
    if (tiles_for<CfgL>(m, n) >= 512) return p;
    const long tm = tiles_for<CfgM>(m, n);
    if (tm >= 512) {
        p.cfg = GEMM_CFG_M;
        return p;
    }
    if (m > 48 && n > 48) {
        p.cfg = GEMM_CFG_M;
        long S = (512 + tm - 1) / tm;
        S = std::min<long>(S, k / 32);
        p.splits = (int)std::max<long>(1, std::min<long>(S, 64));
        return p;
    }
    p.cfg = GEMM_CFG_S;
    const long ts = tiles_for<CfgS>(m, n);
    long S = (2048 + ts - 1) / ts;  // 64-thread workgroups: aim at 2048 of them
    S = std::min<long>(S, k / 32);
    p.splits = (int)std::max<long>(1, std::min<long>(S, 64));
    return p;
}

// Workgroups of the 128x128 direct tile that the device holds at once (256
// CUs, four per CU).
constexpr long DIRECT_SLOTS = 1024;

// Split factor of the direct-load split-K path for an m x n x k fp32 product
// whose 128x128 tiles are all full (0: not used): when there are fewer tiles
// than DIRECT_SLOTS, the S (2..16, chunks of at least 256 k, at least three
// quarters of a round of workgroups) whose tiles * S fills the last round of
// workgroups best.  Smaller products keep the 64x64 split-K plan.
static int direct_split(int m, int n, int k) {
    if (m % CfgL::BM || n % CfgL::BN || k % CfgL::BK || m == 0 || n == 0) return 0;
    const long tiles = tiles_for<CfgL>(m, n);
    if (tiles >= DIRECT_SLOTS || k < 512) return 0;
    int best = 0;
    double best_fill = 0;
    for (int S = 2; S <= 16; ++S) {
        int kc = (k + S - 1) / S;
        kc = (kc + CfgL::BK - 1) / CfgL::BK * CfgL::BK;
        if (kc < 256 || (k + kc - 1) / kc != S) continue;
        const long wgs = tiles * S;
        if (wgs * 4 < DIRECT_SLOTS * 3) continue;  // at least three quarters of one round
        const double fill = (double)wgs / (double)(((wgs + DIRECT_SLOTS - 1) / DIRECT_SLOTS) * DIRECT_SLOTS);
        if (fill > best_fill + 0.02) {
            best_fill = fill;
            best = S;
        }
    }
    return best;
}

size_t gemm_splitk_bytes(int m, int n, int k) {
    const GemmPlan p = plan_gemm(m, n, k);
    const size_t staged = p.splits > 1 ? (size_t)p.splits * m * n * 4 : 0;
    const size_t direct = (size_t)direct_split(m, n, k) * m * n * 4;
    return staged > direct ? staged : direct;
}

template <typename Cfg, typename T, int SR>
static hipError_t launch_cfg(const GemmArgs& g, int S, hipStream_t s) {
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
    if (S > 1 && (g.ws == nullptr || (size_t)S * g.m * g.n * 4 > g.ws_bytes)) S = 1;
    if (S > 1) {
        // chunk length: a multiple of BK, so every chunk but the last is full
        int kc = (g.k + S - 1) / S;
        kc = (kc + Cfg::BK - 1) / Cfg::BK * Cfg::BK;
        S = (g.k + kc - 1) / kc;
        const bool vec_s = vec && g.n % 4 == 0 && (uintptr_t)g.ws % 16 == 0;
        dim3 grid((unsigned)(nb * S)), block(Cfg::NT);
        if (vec_s)
            hipLaunchKernelGGL((tropical_gemm_splitk_kernel<Cfg, T, SR, true>), grid, block,
                               Cfg::lds_bytes, s, a, S, kc, (T*)g.ws, g.wide_in);
        else
            hipLaunchKernelGGL((tropical_gemm_splitk_kernel<Cfg, T, SR, false>), grid, block,
                               Cfg::lds_bytes, s, a, S, kc, (T*)g.ws, g.wide_in);
        long rb = ((long)g.m * g.n + 1023) / 1024;
        rb = std::max<long>(1, std::min<long>(rb, 4096));
        hipLaunchKernelGGL((splitk_reduce_kernel<T, SR>), dim3((unsigned)rb), dim3(256), 0, s, g.m,
                           g.n, S, (const T*)g.ws, (const T*)g.Cin, g.ldci, (T*)g.Cout, g.ldco,
                           g.changed, g.wide_out);
        return hipGetLastError();
    }
    dim3 grid((unsigned)nb), block(Cfg::NT);
    if constexpr (std::is_same_v<Cfg, CfgL>) {
        const bool full = vec && g.m % Cfg::BM == 0 && g.n % Cfg::BN == 0 && g.k % Cfg::BK == 0;
        // full 256x256 tiles that fill their rounds (one per CU): the XL tile
        const long nbx = (long)(g.m / CfgXL::BM) * (g.n / CfgXL::BN);
        const bool xl = full && g.m % CfgXL::BM == 0 && g.n % CfgXL::BN == 0 && xl_fills(nbx);
        if constexpr (std::is_same_v<T, float>) {
            if (xl) {
                hipLaunchKernelGGL((tropical_gemm_direct_kernel<CfgXL, SR>), dim3((unsigned)nbx),
                                   dim3(CfgXL::NT), (GemmTileDirect<CfgXL, SR>::lds_bytes), s, a, nullptr);
                return hipGetLastError();
            }
            if (full) {
                hipLaunchKernelGGL((tropical_gemm_direct_kernel<Cfg, SR>), grid, block,
                                   (GemmTileDirect<Cfg, SR>::lds_bytes), s, a, nullptr);
                return hipGetLastError();
            }
        } else {
            // int32: the direct kernel runs the binary32-exact case and the
            // staged kernel the wide one; the flag picks one on the device.
            if (full && g.wide_in != nullptr) {
                if (xl)
                    hipLaunchKernelGGL((tropical_gemm_direct_kernel<CfgXL, SR, T>), dim3((unsigned)nbx),
                                       dim3(CfgXL::NT), (GemmTileDirect<CfgXL, SR, T>::lds_bytes), s, a,
                                       g.wide_in);
                else
                    hipLaunchKernelGGL((tropical_gemm_direct_kernel<Cfg, SR, T>), grid, block,
                                       (GemmTileDirect<Cfg, SR, T>::lds_bytes), s, a, g.wide_in);
                hipLaunchKernelGGL((tropical_gemm_kernel<Cfg, T, SR, true, true>), grid, block,
                                   Cfg::lds_bytes, s, a, g.wide_in);
                return hipGetLastError();
            }
        }
    }
    if (vec)
        hipLaunchKernelGGL((tropical_gemm_kernel<Cfg, T, SR, true>), grid, block, Cfg::lds_bytes,
                           s, a, g.wide_in);
    else
        hipLaunchKernelGGL((tropical_gemm_kernel<Cfg, T, SR, false>), grid, block,
                           Cfg::lds_bytes, s, a, g.wide_in);
    return hipGetLastError();
}

template <int SR>
static hipError_t launch_direct_split(const GemmArgs& g, int S, hipStream_t s) {
    int kc = (g.k + S - 1) / S;
    kc = (kc + CfgL::BK - 1) / CfgL::BK * CfgL::BK;
    S = (g.k + kc - 1) / kc;
    TileArgs<float> a{g.m, g.n, g.k, (const float*)g.A, g.lda, (const float*)g.B, g.ldb, (const float*)g.Cin,
                      g.ldci, (float*)g.Cout, g.ldco, g.changed, g.wide_out};
    const long nb = tiles_for<CfgL>(g.m, g.n);
    hipLaunchKernelGGL((tropical_gemm_direct_splitk_kernel<CfgL, SR>), dim3((unsigned)(nb * S)),
                       dim3(CfgL::NT), (GemmTileDirect<CfgL, SR>::lds_bytes), s, a, S, kc, (float*)g.ws);
    long rb = ((long)g.m * g.n + 1023) / 1024;
    rb = std::max<long>(1, std::min<long>(rb, 4096));
    hipLaunchKernelGGL((splitk_reduce_kernel<float, SR>), dim3((unsigned)rb), dim3(256), 0, s, g.m, g.n, S,
                       (const float*)g.ws, (const float*)g.Cin, g.ldci, (float*)g.Cout, g.ldco, g.changed,
                       g.wide_out);
    return hipGetLastError();
}

template <typename T, int SR>
static hipError_t launch_typed(const GemmArgs& a, int cfg, hipStream_t s) {
    if constexpr (std::is_same_v<T, float>) {
        // mid-size fp32 products with full 128x128 tiles: direct loads, k split
        const bool vec = (a.lda % 4 == 0) && (a.ldb % 4 == 0) && (a.ldci % 4 == 0) && (a.ldco % 4 == 0) &&
                         (((uintptr_t)a.A | (uintptr_t)a.B | (uintptr_t)a.Cin | (uintptr_t)a.Cout |
                           (uintptr_t)a.ws) % 16 == 0);
        const int S = cfg < 0 && vec ? direct_split(a.m, a.n, a.k) : 0;
        if (S > 1 && a.ws != nullptr && (size_t)S * a.m * a.n * 4 <= a.ws_bytes)
            return launch_direct_split<SR>(a, S, s);
    }
    GemmPlan p = plan_gemm(a.m, a.n, a.k);
    if (cfg >= 0 && cfg != p.cfg) p = GemmPlan{cfg, 1};  // a forced configuration does not split
    switch (p.cfg) {
        case GEMM_CFG_L: return launch_cfg<CfgL, T, SR>(a, p.splits, s);
        case GEMM_CFG_M: return launch_cfg<CfgM, T, SR>(a, p.splits, s);
        case GEMM_CFG_S: return launch_cfg<CfgS, T, SR>(a, p.splits, s);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_gemm(int sr, int dt, const GemmArgs& a, int cfg, hipStream_t s) {
    if (dt == BTAS_FLOAT32)
        return sr == BTAS_MIN_PLUS ? launch_typed<float, BTAS_MIN_PLUS>(a, cfg, s)
                                   : launch_typed<float, BTAS_MAX_PLUS>(a, cfg, s);
    return sr == BTAS_MIN_PLUS ? launch_typed<int32_t, BTAS_MIN_PLUS>(a, cfg, s)
                               : launch_typed<int32_t, BTAS_MAX_PLUS>(a, cfg, s);
}

}  // namespace btas
