// APSP by blocked (three-phase) Floyd-Warshall.
//
// The relaxations of the paper's sequential algorithm (Algorithm 2: for every
// pivot z, d(x,y) <- d(x,y) (+) d(x,z) (.) d(z,y)), grouped by pivot blocks of
// FW_B = 64 consecutive vertices so that all but a thin strip of the work is a
// tropical matrix product.  For pivot block K:
//   1. one workgroup relaxes the diagonal block (K,K) in registers, pivot by
//      pivot;
//   2. one workgroup per other block of block-row K and of block-column K
//      relaxes it in registers against the finished diagonal block;
//   3. every block (I,J) with I != K and J != K gets
//        D_IJ <- D_IJ (+) D_IK (.) D_KJ
//      from blocks that this phase does not change: a tropical GEMM update.
// Pivot blocks are taken in groups (four for fp32 when n is a multiple of
// 128, else pairs) so that phase 3 of the whole group, outside the group's
// own block-rows and block-columns, runs as one k=256 (k=128) product on
// 128x128 tiles (the product kernels' large tile, direct LDS loads for fp32
// when n is a multiple of 128), with thin k=64 strip updates before and after
// it that keep the sequential order's values exactly (fw_typed).  O(n^3)
// work, against O(n^3 log n) for repeated squaring.  In exact arithmetic
// every order gives the shortest distances; in binary32 the result is that
// of the blocked order with blocks of 64, which the grouping does not change
// (min is exact, so one pass over 256 rounded terms equals four passes over
// 64).
//
// Within one pivot z, the entries of row z and column z are relaxed against
// d(z,z) = 0, which leaves them unchanged, so every other entry may be
// relaxed concurrently from the pivot's row and column as they stood before
// it (graphs without negative cycles; with one, the result is unspecified).
#include <hip/hip_runtime.h>

#include <cstdlib>
#include <type_traits>

#include "fw_schedule.h"
#include "gemm_tile.h"
#include "kernels.h"
#include "semiring.h"

namespace btas {

namespace {


// d <- d (+) a (.) b (min-plus).
template <typename T>
__device__ __forceinline__ T relax(T a, T b, T d) {
    using R = Ring<BTAS_MIN_PLUS, T>;
    return R::add(d, R::finish(R::mul(a, b)));
}

// The same without mapping the sum back to the absent value: for int32 with
// canonical operands (finite, or the absent value itself) a sum that
// involves the absent value is >= 2^30, so an accumulator that only ever
// takes minima of such sums holds either the exact finite value or some
// value >= 2^30 that stands for "absent"; R::finish maps it back once where
// it is read as an operand or stored.  Every entry ends equal to relax's.
// (float32: R::finish is the identity and this is relax.)
template <typename T>
__device__ __forceinline__ T relax_raw(T a, T b, T d) {
    using R = Ring<BTAS_MIN_PLUS, T>;
    return R::add(d, R::mul(a, b));
}

// Calls f(std::integral_constant<int, I>) for I = B .. E-1: a loop whose index
// is a constant in every copy of the body (register arrays stay in registers
// where #pragma unroll would give up on a body this large).
template <int B, int E, typename F>
__device__ __forceinline__ void static_for(F&& f) {
    if constexpr (B < E) {
        f(std::integral_constant<int, B>{});
        static_for<B + 1, E>(f);
    }
}

// Phases 1 and 2: four waves per 64x64 block, the block in registers.  Lane
// l of wave w holds 16 entries v[0..15] of line l (a row or a column of the
// block), the 16 lines 16w..16w+15 of the other direction.  At pivot z the
// entries of the pivot's line that a wave needs sit in its lane z
// (readlane); the other operand is one value per lane.  The pivot loop is a
// static_for, so register indices are constants.  The registers accumulate
// with relax_raw: the readlane value is wave-uniform, so mapping it back to
// the absent value is scalar work, and a term costs one add and one min on
// the vector unit.

template <typename T>
__device__ __forceinline__ T lane_value(T x, int lane) {
    return __builtin_bit_cast(T, __builtin_amdgcn_readlane(__builtin_bit_cast(int, x), lane));
}

// Phase 1: the diagonal block of pivot block kb, pivots in ascending order.
// NW waves, E = 64/NW rows each: lane j of wave w holds column j, rows E*w+r.
// d(i,z) for the wave's rows is in its lane z; d(z,j) is row z, held by wave
// z/E, passed through LDS.
template <typename T, int NW = 4>
__device__ __forceinline__ void phase1_block(int n, T* D, long ld, int kb) {
    using R = Ring<BTAS_MIN_PLUS, T>;
    constexpr int E = FW_B / NW;
    __shared__ T rowz[2][FW_B];
    const int k0 = kb * FW_B, ks = n - k0 < FW_B ? n - k0 : FW_B;
    const int j = threadIdx.x % 64, w = threadIdx.x / 64;
    T v[E];
#pragma unroll
    for (int r = 0; r < E; ++r) {
        const int i = E * w + r;
        v[r] = (i < ks && j < ks) ? D[(long)(k0 + i) * ld + k0 + j] : R::absent();
    }
    static_for<0, FW_B>([&](auto zc) {
        constexpr int z = decltype(zc)::value;
        if (z < ks) {
            if (w == z / E) rowz[z & 1][j] = R::finish(v[z % E]);
            __syncthreads();  // this slot is written again two pivots later
            const T dzj = rowz[z & 1][j];
#pragma unroll
            for (int r = 0; r < E; ++r) v[r] = relax_raw(R::finish(lane_value(v[r], z)), dzj, v[r]);
        }
    });
#pragma unroll
    for (int r = 0; r < E; ++r) {
        const int i = E * w + r;
        if (i < ks && j < ks) D[(long)(k0 + i) * ld + k0 + j] = R::finish(v[r]);
    }
}

constexpr int FW_P1_WAVES = 16;  // phase 1 of single graphs: 16 waves, 4 rows each

template <typename T>
__global__ __launch_bounds__(FW_P1_WAVES * 64) void fw_phase1_kernel(int n, T* D, long ld, int kb) {
    phase1_block<T, FW_P1_WAVES>(n, D, ld, kb);
}

// Phase 2: workgroup b < nb-1 takes block (kb, J) of block-row kb, the others
// block (I, kb) of block-column kb (J, I skip kb); each relaxes its block
// against the finished diagonal block, pivots in ascending order.
//   block-row:    own(x,j) <- own(x,j) (+) dia(x,z) (.) own(z,j): lane x holds
//                 row x, columns E*w+c; own(z,j) is in lane z;
//   block-column: own(i,x) <- own(i,x) (+) own(i,z) (.) dia(z,x): lane x holds
//                 column x, rows E*w+c; own(i,z) is in lane z.
// NW waves per block, E = 64/NW entries per lane.  The per-lane operand
// L[z][x] (dia(x,z), resp. dia(z,x)) is constant, so no wave waits for
// another after the set-up.
template <typename T, int NW = 4>
__device__ __forceinline__ void phase2_block(int n, T* D, long ld, int kb, int nb, int bid) {
    constexpr int E = FW_B / NW;
    using R = Ring<BTAS_MIN_PLUS, T>;
    constexpr int LP = FW_B + 1;  // the transposed fill walks a column
    __shared__ T L[FW_B][LP];
    const int k0 = kb * FW_B, ks = n - k0 < FW_B ? n - k0 : FW_B;
    const bool row = bid < nb - 1;
    int b = row ? bid : bid - (nb - 1);
    b += b >= kb ? 1 : 0;
    const int o0 = b * FW_B, os = n - o0 < FW_B ? n - o0 : FW_B;
    const int x = threadIdx.x % 64, w = threadIdx.x / 64;
    for (int e = threadIdx.x; e < FW_B * FW_B; e += NW * 64) {
        const int i = e / FW_B, c = e % FW_B;
        const T d = (i < ks && c < ks) ? D[(long)(k0 + i) * ld + k0 + c] : R::absent();
        if (row)
            L[c][i] = d;
        else
            L[i][c] = d;
    }
    T v[E];
#pragma unroll
    for (int c = 0; c < E; ++c) {
        const int o = E * w + c;
        if (row)
            v[c] = (x < ks && o < os) ? D[(long)(k0 + x) * ld + o0 + o] : R::absent();
        else
            v[c] = (o < os && x < ks) ? D[(long)(o0 + o) * ld + k0 + x] : R::absent();
    }
    __syncthreads();
    static_for<0, FW_B>([&](auto zc) {
        constexpr int z = decltype(zc)::value;
        if (z < ks) {
            const T lz = L[z][x];
#pragma unroll
            for (int c = 0; c < E; ++c) v[c] = relax_raw(lz, R::finish(lane_value(v[c], z)), v[c]);
        }
    });
#pragma unroll
    for (int c = 0; c < E; ++c) {
        const int o = E * w + c;
        if (row) {
            if (x < ks && o < os) D[(long)(k0 + x) * ld + o0 + o] = R::finish(v[c]);
        } else {
            if (o < os && x < ks) D[(long)(o0 + o) * ld + k0 + x] = R::finish(v[c]);
        }
    }
}

constexpr int FW_P2_WAVES = 16;  // phase 2 of single graphs: 16 waves per block

template <typename T>
__global__ __launch_bounds__(FW_P2_WAVES * 64) void fw_phase2_kernel(int n, T* D, long ld, int kb, int nb) {
    phase2_block<T, FW_P2_WAVES>(n, D, ld, kb, nb, (int)blockIdx.x);
}

// fp32 with n a multiple of 64: every block full, direct LDS loads.
// The k=64 strip updates on the direct-load path: four waves per 64x64
// block, 4x4 outputs per thread.  (With one wave per block and 8x8 outputs
// per lane each workgroup ran 64^3 terms through one SIMD, 22-40 us per
// launch.)
using FwStripCfg = GemmCfg<64, 64, 16, 4, 4>;

template <int SR>
__global__ __launch_bounds__(FwStripCfg::NT) void fw_band_direct_kernel(
    int n, float* D, long ld, BandSel u) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    int I, J;
    select_band(u, blockIdx.x, I, J);
    const int k0 = u.kb * FW_B;
    TileArgs<float> a{n, n, FW_B, D + k0, ld, D + (long)k0 * ld, ld, D, ld, D, ld, nullptr, nullptr};
    GemmTileDirect<FwStripCfg, SR>::run(a, I * FW_B, J * FW_B, smem_raw);
}

template <int SR>
__global__ __launch_bounds__(FwStripCfg::NT) void fw_update_direct_kernel(
    int n, float* D, long ld, UpdateSel u) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    int I, J;
    select_block(u, blockIdx.x, I, J);
    const int k0 = u.kb * FW_B;
    TileArgs<float> a{n, n, FW_B, D + k0, ld, D + (long)k0 * ld, ld, D, ld, D, ld, nullptr, nullptr};
    GemmTileDirect<FwStripCfg, SR>::run(a, I * FW_B, J * FW_B, smem_raw);
}

// General: the staged one-wave tile with bounds checks.
template <typename T, bool VEC>
__global__ __launch_bounds__(64) void fw_update_kernel(int n, T* D, long ld, UpdateSel u) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    int I, J;
    select_block(u, blockIdx.x, I, J);
    const int k0 = u.kb * FW_B, ks = n - k0 < FW_B ? n - k0 : FW_B;
    TileArgs<T> a{n, n, ks, D + k0, ld, D + (long)k0 * ld, ld, D, ld, D, ld, nullptr, nullptr};
    GemmTile<GemmCfg<64, 64, 8, 8, 8>, T, T, BTAS_MIN_PLUS, VEC>::run(a, I * FW_B, J * FW_B, smem_raw);
}

template <int SR>
__global__ __launch_bounds__(CfgL::NT) __attribute__((amdgpu_waves_per_eu(4))) void fw_pair_direct_kernel(
    int n, float* D, long ld, int sb, int nb2) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    int m0, n0;
    pair_tile(blockIdx.x, sb, nb2, m0, n0);
    const int k0 = sb * 2 * FW_B;
    TileArgs<float> a{n, n, 2 * FW_B, D + k0, ld, D + (long)k0 * ld, ld, D, ld, D, ld, nullptr, nullptr};
    GemmTileDirect<CfgL, SR>::run(a, m0, n0, smem_raw);
}

template <int SR>
__global__ __launch_bounds__(CfgL::NT) __attribute__((amdgpu_waves_per_eu(4))) void fw_quad_direct_kernel(
    int n, float* D, long ld, int q, int nt) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    int m0, n0;
    quad_tile(blockIdx.x, q, nt, m0, n0);
    const int k0 = q * 4 * FW_B;
    TileArgs<float> a{n, n, 4 * FW_B, D + k0, ld, D + (long)k0 * ld, ld, D, ld, D, ld, nullptr, nullptr};
    GemmTileDirect<CfgL, SR>::run(a, m0, n0, smem_raw);
}

template <typename T, bool VEC>
__global__ __launch_bounds__(CfgL::NT) void fw_pair_kernel(int n, T* D, long ld, int sb, int nb2) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    int m0, n0;
    pair_tile(blockIdx.x, sb, nb2, m0, n0);
    const int k0 = sb * 2 * FW_B, ks = n - k0 < 2 * FW_B ? n - k0 : 2 * FW_B;
    TileArgs<T> a{n, n, ks, D + k0, ld, D + (long)k0 * ld, ld, D, ld, D, ld, nullptr, nullptr};
    GemmTile<CfgL, T, T, BTAS_MIN_PLUS, VEC>::run(a, m0, n0, smem_raw);
}

constexpr int FW_QUAD_MIN_N = 8192;

template <typename T>
struct FwLaunch {
    int n, nb;
    T* D;
    long ld;
    hipStream_t s;
    bool vec;

    void phase12(int kb) const {
        hipLaunchKernelGGL(fw_phase1_kernel<T>, dim3(1), dim3(FW_P1_WAVES * 64), 0, s, n, D, ld, kb);
        if (nb > 1)
            hipLaunchKernelGGL(fw_phase2_kernel<T>, dim3(2 * (nb - 1)), dim3(FW_P2_WAVES * 64), 0, s, n, D, ld, kb,
                               nb);
    }

    void update(const UpdateSel& u) const {
        const unsigned blocks = update_blocks(u);
        if (blocks == 0) return;
        if constexpr (std::is_same_v<T, float>) {
            if (vec && n % FW_B == 0) {
                using DT = GemmTileDirect<FwStripCfg, BTAS_MIN_PLUS>;
                hipLaunchKernelGGL((fw_update_direct_kernel<BTAS_MIN_PLUS>), dim3(blocks), dim3(FwStripCfg::NT),
                                   DT::lds_bytes, s, n, D, ld, u);
                return;
            }
        }
        using ST = GemmCfg<64, 64, 8, 8, 8>;
        if (vec)
            hipLaunchKernelGGL((fw_update_kernel<T, true>), dim3(blocks), dim3(64), ST::lds_bytes, s,
                               n, D, ld, u);
        else
            hipLaunchKernelGGL((fw_update_kernel<T, false>), dim3(blocks), dim3(64), ST::lds_bytes,
                               s, n, D, ld, u);
    }

    // fp32 with every 128x128 tile full and n >= FW_QUAD_MIN_N: groups of
    // four pivot blocks.  Each group adds two strip launches and three times
    // the strip work of two pairs, which its k=256 update repays only on
    // large graphs (n=16384: 141 against 146-147 ms; n=8192: 21.6 against
    // 21.9; n=4096: 5.4-5.5 against 5.3).  BTAS_FW_GROUP=2 or 4 forces pairs
    // or groups of four.
    bool quads() const {
        if constexpr (!std::is_same_v<T, float>) return false;
        if (!vec || n % (2 * FW_B) != 0) return false;
        const char* e = getenv("BTAS_FW_GROUP");
        if (e && e[0] == '2') return false;
        if (e && e[0] == '4') return true;
        return n >= FW_QUAD_MIN_N;
    }

    // (only reached when quads() holds: fp32, every 128x128 tile full)
    void band(const BandSel& u) const {
        if constexpr (std::is_same_v<T, float>) {
            const long blocks = band_blocks(u);
            if (blocks <= 0) return;
            using DT = GemmTileDirect<FwStripCfg, BTAS_MIN_PLUS>;
            hipLaunchKernelGGL((fw_band_direct_kernel<BTAS_MIN_PLUS>), dim3((unsigned)blocks), dim3(FwStripCfg::NT),
                               DT::lds_bytes, s, n, D, ld, u);
        }
    }

    void quad_update(int q) const {
        if constexpr (std::is_same_v<T, float>) {
            const int nt = n / (2 * FW_B);
            const unsigned tiles = (unsigned)((long)(nt - 2) * (nt - 2));
            if (tiles == 0) return;
            using DT = GemmTileDirect<CfgL, BTAS_MIN_PLUS>;
            hipLaunchKernelGGL((fw_quad_direct_kernel<BTAS_MIN_PLUS>), dim3(tiles), dim3(CfgL::NT),
                               DT::lds_bytes, s, n, D, ld, q, nt);
        }
    }

    void pair_update(int sb) const {
        const int nb2 = (n + 2 * FW_B - 1) / (2 * FW_B);
        const unsigned tiles = (unsigned)((long)(nb2 - 1) * (nb2 - 1));
        if (tiles == 0) return;
        if constexpr (std::is_same_v<T, float>) {
            if (vec && n % (2 * FW_B) == 0) {
                using DT = GemmTileDirect<CfgL, BTAS_MIN_PLUS>;
                hipLaunchKernelGGL((fw_pair_direct_kernel<BTAS_MIN_PLUS>), dim3(tiles), dim3(CfgL::NT),
                                   DT::lds_bytes, s, n, D, ld, sb, nb2);
                return;
            }
        }
        if (vec)
            hipLaunchKernelGGL((fw_pair_kernel<T, true>), dim3(tiles), dim3(CfgL::NT), CfgL::lds_bytes,
                               s, n, D, ld, sb, nb2);
        else
            hipLaunchKernelGGL((fw_pair_kernel<T, false>), dim3(tiles), dim3(CfgL::NT), CfgL::lds_bytes,
                               s, n, D, ld, sb, nb2);
    }
};

// The launches of fw_schedule (fw_schedule.h), in order on one stream.  The
// sequential blocked order's effects are kept exactly; only the updates of
// entries outside a pair's (group's) rows and columns are fused, which leaves
// every entry the same min of the same rounded terms.
template <typename T>
hipError_t fw_typed(int n, T* D, long ld, hipStream_t s) {
    const int nb = (n + FW_B - 1) / FW_B;
    const FwLaunch<T> L{n, nb, D, ld, s, ld % 4 == 0 && (uintptr_t)D % 16 == 0};
    for (const FwStep& st : fw_schedule(nb, L.quads())) {
        switch (st.kind) {
            case FW_PHASE12: L.phase12(st.kb); break;
            case FW_UPDATE: L.update(st.u); break;
            case FW_BAND: L.band(st.b); break;
            case FW_PAIR: L.pair_update(st.q); break;
            case FW_QUAD: L.quad_update(st.q); break;
        }
    }
    return hipGetLastError();
}

// ---- many graphs at once: one launch per phase and pivot block for all ----
// graphs that still have that pivot block (work items name a graph and a
// block index within that graph's phase).

// D <- I (+) W, rows 64r .. 64r+63 of one graph per workgroup.
template <typename T>
__global__ __launch_bounds__(256) void fwb_init_kernel(const FwGraph* __restrict__ gs,
                                                       const FwItem* __restrict__ items) {
    const FwItem it = items[blockIdx.x];
    const FwGraph g = gs[it.graph];
    const T* W = (const T*)g.W;
    T* D = (T*)g.D;
    const int r0 = it.idx * FW_B, rows = g.n - r0 < FW_B ? g.n - r0 : FW_B;
    for (long e = threadIdx.x; e < (long)rows * g.n; e += 256) {
        const int i = r0 + (int)(e / g.n), j = (int)(e % g.n);
        T w = W[(long)i * g.ldw + j];
        if (i == j && w > (T)0) w = (T)0;
        D[(long)i * g.ldd + j] = w;
    }
}

constexpr int FWB_P_WAVES = 8;  // phases 1-2 of batched graphs (4: 5.61 ms, 16: 5.95 ms on the 4096-graph workload)

template <typename T>
__global__ __launch_bounds__(FWB_P_WAVES * 64) void fwb_phase1_kernel(const FwGraph* __restrict__ gs,
                                                                      const FwItem* __restrict__ items, int kb) {
    const FwItem it = items[blockIdx.x];
    const FwGraph g = gs[it.graph];
    phase1_block<T, FWB_P_WAVES>(g.n, (T*)g.D, g.ldd, kb);
}

template <typename T>
__global__ __launch_bounds__(FWB_P_WAVES * 64) void fwb_phase2_kernel(const FwGraph* __restrict__ gs,
                                                                      const FwItem* __restrict__ items, int kb) {
    const FwItem it = items[blockIdx.x];
    const FwGraph g = gs[it.graph];
    phase2_block<T, FWB_P_WAVES>(g.n, (T*)g.D, g.ldd, kb, g.nb, it.idx);
}

// Updates of many small graphs on the four-wave 64x64 tile (4x4 per thread);
// with k = 64 per tile more waves per tile hide the loads better than the
// one-wave tile (measured 7.0 against 7.5 ms on 4096 graphs of 16..512).
// mode 0: phase 3 of pivot block kb (every block outside its row and
// column); mode 1: kb's update of block-row and block-column kb+1; mode 2:
// kb's update of block-row and block-column kb-1 (the pair schedule's strips).
template <typename T, bool VEC>
__global__ __launch_bounds__(256) void fwb_update_kernel(const FwGraph* __restrict__ gs,
                                                        const FwItem* __restrict__ items, int kb,
                                                        int mode) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const FwItem it = items[blockIdx.x];
    const FwGraph g = gs[it.graph];
    const UpdateSel u = mode == 0 ? UpdateSel{kb, g.nb, -1, -1}
                                  : UpdateSel{kb, g.nb, mode == 1 ? kb + 1 : kb - 1, kb};
    int I, J;
    select_block(u, it.idx, I, J);
    T* D = (T*)g.D;
    const int k0 = kb * FW_B, ks = g.n - k0 < FW_B ? g.n - k0 : FW_B;
    TileArgs<T> a{g.n, g.n, ks, D + k0, g.ldd, D + (long)k0 * g.ldd, g.ldd, D, g.ldd, D, g.ldd,
                  nullptr, nullptr};
    GemmTile<CfgM, T, T, BTAS_MIN_PLUS, VEC>::run(a, I * FW_B, J * FW_B, smem_raw);
}

// The pair update of many graphs: 128x128 tiles outside tile-row and
// tile-column kb/2, k = the 128 pivots of blocks kb and kb+1.
template <typename T, bool VEC>
__global__ __launch_bounds__(CfgL::NT) void fwb_pair_kernel(const FwGraph* __restrict__ gs,
                                                           const FwItem* __restrict__ items, int kb) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const FwItem it = items[blockIdx.x];
    const FwGraph g = gs[it.graph];
    const int sb = kb / 2, nb2 = (g.n + 2 * FW_B - 1) / (2 * FW_B);
    int m0, n0;
    pair_tile(it.idx, sb, nb2, m0, n0);
    T* D = (T*)g.D;
    const int k0 = sb * 2 * FW_B, ks = g.n - k0 < 2 * FW_B ? g.n - k0 : 2 * FW_B;
    TileArgs<T> a{g.n, g.n, ks, D + k0, g.ldd, D + (long)k0 * g.ldd, g.ldd, D, g.ldd, D, g.ldd,
                  nullptr, nullptr};
    GemmTile<CfgL, T, T, BTAS_MIN_PLUS, VEC>::run(a, m0, n0, smem_raw);
}

template <typename T, bool VEC>
void fwb_launch_update(const FwGraph* gs, const FwItem* items, int nitems, int kb, int mode,
                       hipStream_t s) {
    hipLaunchKernelGGL((fwb_update_kernel<T, VEC>), dim3(nitems), dim3(256), CfgM::lds_bytes, s, gs,
                       items, kb, mode);
}

template <typename T, bool VEC>
void fwb_launch_pair(const FwGraph* gs, const FwItem* items, int nitems, int kb, hipStream_t s) {
    hipLaunchKernelGGL((fwb_pair_kernel<T, VEC>), dim3(nitems), dim3(CfgL::NT), CfgL::lds_bytes, s,
                       gs, items, kb);
}

template <typename T>
hipError_t fwb_typed(int phase, const FwGraph* gs, const FwItem* items, int nitems, int kb, bool vec,
                     hipStream_t s) {
    if (nitems <= 0) return hipSuccess;
    switch (phase) {
        case FWB_INIT:
            hipLaunchKernelGGL(fwb_init_kernel<T>, dim3(nitems), dim3(256), 0, s, gs, items);
            break;
        case FWB_PHASE1:
            hipLaunchKernelGGL(fwb_phase1_kernel<T>, dim3(nitems), dim3(FWB_P_WAVES * 64), 0, s, gs, items, kb);
            break;
        case FWB_PHASE2:
            hipLaunchKernelGGL(fwb_phase2_kernel<T>, dim3(nitems), dim3(FWB_P_WAVES * 64), 0, s, gs, items, kb);
            break;
        case FWB_PHASE3:
        case FWB_STRIP_NEXT:
        case FWB_STRIP_PREV: {
            const int mode = phase == FWB_PHASE3 ? 0 : (phase == FWB_STRIP_NEXT ? 1 : 2);
            if (vec)
                fwb_launch_update<T, true>(gs, items, nitems, kb, mode, s);
            else
                fwb_launch_update<T, false>(gs, items, nitems, kb, mode, s);
            break;
        }
        case FWB_PAIR:
            if (vec)
                fwb_launch_pair<T, true>(gs, items, nitems, kb, s);
            else
                fwb_launch_pair<T, false>(gs, items, nitems, kb, s);
            break;
        default:
            return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace

hipError_t launch_fw_batched(int dt, int phase, const FwGraph* graphs, const FwItem* items, int nitems,
                             int kb, bool vec, hipStream_t s) {
    return dt == BTAS_FLOAT32 ? fwb_typed<float>(phase, graphs, items, nitems, kb, vec, s)
                              : fwb_typed<int32_t>(phase, graphs, items, nitems, kb, vec, s);
}

int fw_block_size() { return FW_B; }

hipError_t launch_floyd_warshall(int dt, int n, void* D, long ld, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    if (dt == BTAS_FLOAT32) return fw_typed<float>(n, (float*)D, ld, s);
    return fw_typed<int32_t>(n, (int32_t*)D, ld, s);
}

}  // namespace btas
