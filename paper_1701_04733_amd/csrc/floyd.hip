// APSP by blocked (three-phase) Floyd-Warshall.
//
// The relaxations of the paper's sequential algorithm (Algorithm 2: for every
// pivot z, d(x,y) <- d(x,y) (+) d(x,z) (.) d(z,y)), grouped by pivot blocks of
// FW_B = 64 consecutive vertices so that all but a thin strip of the work is a
// tropical matrix product.  For pivot block K:
//   1. one workgroup relaxes the diagonal block (K,K) in LDS, pivot by pivot;
//   2. one workgroup per other block of block-row K and of block-column K
//      relaxes it in LDS against the finished diagonal block, pivot by pivot;
//   3. every block (I,J) with I != K and J != K gets
//        D_IJ <- D_IJ (+) D_IK (.) D_KJ
//      from blocks that this phase does not change: a tropical GEMM update with
//      k = 64, run by the one-wave 64x64 tile of the product kernels (direct
//      LDS loads for fp32 when n is a multiple of 64).
// O(n^3) work in n/64 rounds of three launches, against O(n^3 log n) for
// repeated squaring.  In exact arithmetic every order gives the shortest
// distances; in binary32 the result is that of this order and block size.
//
// Within one pivot z, the entries of row z and column z are relaxed against
// d(z,z) = 0, which leaves them unchanged, so every other entry may be
// relaxed concurrently with one barrier per pivot (graphs without negative
// cycles; with one, the result is unspecified).
#include <hip/hip_runtime.h>

#include <type_traits>

#include "gemm_tile.h"
#include "kernels.h"
#include "semiring.h"

namespace btas {

namespace {

constexpr int FW_B = 64;      // pivot block edge
constexpr int FW_NT = 256;    // threads of the phase-1/2 workgroups
constexpr int FW_PER = FW_B * FW_B / FW_NT;  // block entries per thread

// d <- d (+) a (.) b (min-plus).
template <typename T>
__device__ __forceinline__ T relax(T a, T b, T d) {
    using R = Ring<BTAS_MIN_PLUS, T>;
    return R::add(d, R::finish(R::mul(a, b)));
}

template <typename T>
__device__ __forceinline__ void load_block(T (*dst)[FW_B], const T* D, long ld, int r0, int c0,
                                           int rows, int cols) {
    for (int e = threadIdx.x; e < FW_B * FW_B; e += FW_NT) {
        const int i = e / FW_B, j = e % FW_B;
        dst[i][j] = (i < rows && j < cols) ? D[(long)(r0 + i) * ld + c0 + j]
                                           : Ring<BTAS_MIN_PLUS, T>::absent();
    }
}

template <typename T>
__device__ __forceinline__ void store_block(const T (*src)[FW_B], T* D, long ld, int r0, int c0,
                                            int rows, int cols) {
    for (int e = threadIdx.x; e < FW_B * FW_B; e += FW_NT) {
        const int i = e / FW_B, j = e % FW_B;
        if (i < rows && j < cols) D[(long)(r0 + i) * ld + c0 + j] = src[i][j];
    }
}

// Phase 1: the diagonal block of pivot block kb, pivots in ascending order.
// Thread t owns entries (t/64 + 4r, t%64): a wave shares the row, so the
// column-z operand is a broadcast and the row-z operand 64 consecutive words.
template <typename T>
__global__ __launch_bounds__(FW_NT) void fw_phase1_kernel(int n, T* D, long ld, int kb) {
    __shared__ T blk[FW_B][FW_B];
    const int k0 = kb * FW_B, ks = n - k0 < FW_B ? n - k0 : FW_B;
    load_block(blk, D, ld, k0, k0, ks, ks);
    __syncthreads();
    const int i0 = threadIdx.x / FW_B, j = threadIdx.x % FW_B;
    for (int z = 0; z < ks; ++z) {
        const T bz = blk[z][j];
#pragma unroll
        for (int r = 0; r < FW_PER; ++r) {
            const int i = i0 + r * (FW_NT / FW_B);
            blk[i][j] = relax(blk[i][z], bz, blk[i][j]);
        }
        __syncthreads();
    }
    store_block(blk, D, ld, k0, k0, ks, ks);
}

// Phase 2: workgroup w < nb-1 takes block (kb, J) of block-row kb, the others
// block (I, kb) of block-column kb (J, I skip kb); each relaxes its block
// against the finished diagonal block, pivots in ascending order.
template <typename T>
__global__ __launch_bounds__(FW_NT) void fw_phase2_kernel(int n, T* D, long ld, int kb, int nb) {
    __shared__ T dia[FW_B][FW_B];
    __shared__ T own[FW_B][FW_B];
    const int k0 = kb * FW_B, ks = n - k0 < FW_B ? n - k0 : FW_B;
    const bool row = blockIdx.x < (unsigned)(nb - 1);
    int b = row ? blockIdx.x : blockIdx.x - (nb - 1);
    b += b >= kb ? 1 : 0;
    const int o0 = b * FW_B, os = n - o0 < FW_B ? n - o0 : FW_B;
    const int r0 = row ? k0 : o0, c0 = row ? o0 : k0;
    const int rows = row ? ks : os, cols = row ? os : ks;
    load_block(dia, D, ld, k0, k0, ks, ks);
    load_block(own, D, ld, r0, c0, rows, cols);
    __syncthreads();
    const int i0 = threadIdx.x / FW_B, j = threadIdx.x % FW_B;
    for (int z = 0; z < ks; ++z) {
        if (row) {
            // own(i,j) <- own(i,j) (+) dia(i,z) (.) own(z,j)
            const T bz = own[z][j];
#pragma unroll
            for (int r = 0; r < FW_PER; ++r) {
                const int i = i0 + r * (FW_NT / FW_B);
                own[i][j] = relax(dia[i][z], bz, own[i][j]);
            }
        } else {
            // own(i,j) <- own(i,j) (+) own(i,z) (.) dia(z,j)
            const T bz = dia[z][j];
#pragma unroll
            for (int r = 0; r < FW_PER; ++r) {
                const int i = i0 + r * (FW_NT / FW_B);
                own[i][j] = relax(own[i][z], bz, own[i][j]);
            }
        }
        __syncthreads();
    }
    store_block(own, D, ld, r0, c0, rows, cols);
}

// Tile (I, J) of phase 3 for workgroup t of (nb-1)^2 (I, J skip kb).
__device__ __forceinline__ void phase3_tile(int t, int kb, int nb, int& m0, int& n0) {
    int I = t / (nb - 1), J = t % (nb - 1);
    I += I >= kb ? 1 : 0;
    J += J >= kb ? 1 : 0;
    m0 = I * FW_B;
    n0 = J * FW_B;
}

// Phase 3, fp32 with n a multiple of 64: every tile full, direct LDS loads.
template <int SR>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(4))) void fw_phase3_direct_kernel(
    int n, float* D, long ld, int kb, int nb) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    int m0, n0;
    phase3_tile(blockIdx.x, kb, nb, m0, n0);
    const int k0 = kb * FW_B;
    TileArgs<float> a{n, n, FW_B, D + k0, ld, D + (long)k0 * ld, ld, D, ld, D, ld, nullptr, nullptr};
    GemmTileDirect<GemmCfg<64, 64, 8, 8, 8>, SR>::run(a, m0, n0, smem_raw);
}

// Phase 3, general: the staged one-wave tile with bounds checks.
template <typename T, bool VEC>
__global__ __launch_bounds__(64) void fw_phase3_kernel(int n, T* D, long ld, int kb, int nb) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    int m0, n0;
    phase3_tile(blockIdx.x, kb, nb, m0, n0);
    const int k0 = kb * FW_B, ks = n - k0 < FW_B ? n - k0 : FW_B;
    TileArgs<T> a{n, n, ks, D + k0, ld, D + (long)k0 * ld, ld, D, ld, D, ld, nullptr, nullptr};
    GemmTile<GemmCfg<64, 64, 8, 8, 8>, T, T, BTAS_MIN_PLUS, VEC>::run(a, m0, n0, smem_raw);
}

template <typename T>
hipError_t fw_typed(int n, T* D, long ld, hipStream_t s) {
    const int nb = (n + FW_B - 1) / FW_B;
    const bool vec = ld % 4 == 0 && (uintptr_t)D % 16 == 0;
    const bool direct = std::is_same_v<T, float> && vec && n % FW_B == 0;
    using DT = GemmTileDirect<GemmCfg<64, 64, 8, 8, 8>, BTAS_MIN_PLUS>;
    using ST = GemmCfg<64, 64, 8, 8, 8>;
    for (int kb = 0; kb < nb; ++kb) {
        hipLaunchKernelGGL(fw_phase1_kernel<T>, dim3(1), dim3(FW_NT), 0, s, n, D, ld, kb);
        if (nb > 1) {
            hipLaunchKernelGGL(fw_phase2_kernel<T>, dim3(2 * (nb - 1)), dim3(FW_NT), 0, s, n, D, ld,
                               kb, nb);
            const unsigned tiles = (unsigned)((long)(nb - 1) * (nb - 1));
            if constexpr (std::is_same_v<T, float>) {
                if (direct) {
                    hipLaunchKernelGGL((fw_phase3_direct_kernel<BTAS_MIN_PLUS>), dim3(tiles), dim3(64),
                                       DT::lds_bytes, s, n, D, ld, kb, nb);
                    continue;
                }
            }
            if (vec)
                hipLaunchKernelGGL((fw_phase3_kernel<T, true>), dim3(tiles), dim3(64), ST::lds_bytes,
                                   s, n, D, ld, kb, nb);
            else
                hipLaunchKernelGGL((fw_phase3_kernel<T, false>), dim3(tiles), dim3(64), ST::lds_bytes,
                                   s, n, D, ld, kb, nb);
        }
    }
    return hipGetLastError();
}

}  // namespace

int fw_block_size() { return FW_B; }

hipError_t launch_floyd_warshall(int dt, int n, void* D, long ld, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    if (dt == BTAS_FLOAT32) return fw_typed<float>(n, (float*)D, ld, s);
    return fw_typed<int32_t>(n, (int32_t*)D, ld, s);
}

}  // namespace btas
