// Tropical product with witnesses: C <- C (+) A (.) B, and for every entry
// whose value strictly improves, K <- the smallest p whose term A_ip (.) B_pj
// attains it (the min over k of the Sec. IV product listing, with its
// argument).  The same kernel computes successor matrices of APSP:
// S_ij = the smallest u != i minimising W_iu (.) D_uj (i != j), S_ii = i,
// -1 where every term is absent.
//
// Ties are decided on the terms' values in the kernel's arithmetic (binary32
// adds for float32, clamped int32 adds mapped back to the absent value for
// int32), which is the arithmetic of the value-only product, so C is the same
// as that product's and K is unique.
//
// A 64x64 output tile per 256-thread workgroup, 4x4 outputs per thread, k in
// blocks of 16 staged through LDS.  Each witness block of 64 terms (four
// k-blocks; 32 for successors) is reduced per output with three-way min/max
// (the cost of the value-only product); an output whose block extreme
// strictly beats its running best takes it and remembers the block (a
// compare and two selects per output and block).  The index search is
// deferred: after the k loop each output rereads, from global memory, the
// terms of the one block that holds its final value and takes the first
// index attaining it.  Ties across blocks keep the earliest block (strict
// comparison), ties inside it the earliest index, so the witness is the
// smallest p, as with a search inside the loop, which measured 2.9 VALU
// instructions per term against the 1.5 of the value product: a wave had to
// search a block whenever any of its 64 lanes improved there.
#include <hip/hip_runtime.h>

#include <type_traits>

#include "kernels.h"
#include "semiring.h"

namespace btas {

namespace {

constexpr int WT_BM = 64, WT_BN = 64, WT_BK = 16;
// k-blocks per witness block: 4 (64 terms) for the product, 2 (32 terms) for
// successors, whose every entry runs the deferred search (8192^3 product:
// 17.5 ms with 32-term blocks, 17.0 with 64, 16.9 with 128; dense successors
// n=16384: 135, 141, 239 ms).
template <bool SUCC>
constexpr int wt_wb() { return SUCC ? 2 : 4; }
constexpr int WT_NT = 256;
constexpr int WT_TM = 4, WT_TN = 4;
constexpr int WT_VW = WT_BM * WT_BK / WT_NT;  // staged elements per thread and operand
constexpr int WT_APAD = 4;  // As rows padded: transposed stores hit 64 banks
static_assert(WT_VW >= 1 && WT_VW <= 4 && WT_BK % 2 == 0, "staging layout");

template <typename T>
struct WitnessArgs {
    int m, n, k;
    const T* A;
    long lda;
    const T* B;
    long ldb;
    T* C;        // read and written in product mode; unused for successors
    long ldc;
    int32_t* K;  // witnesses (product mode) or successors
    long ldk;
};

template <int SR, typename T>
__device__ __forceinline__ bool better(T x, T y) {
    if constexpr (SR == BTAS_MIN_PLUS) return x < y;
    else return x > y;
}

// blockIdx -> (tile row, tile col): consecutive workgroups go to different
// XCDs, so each XCD gets a contiguous range of tiles, walked in groups of 8
// tile rows so that neighbouring workgroups share B panels in that XCD's L2.
__device__ __forceinline__ void wt_tile_of(int bid, int nb, int nbm, int nbn, int& tm, int& tn) {
    constexpr int NXCD = 8, GROUP_M = 8;
    const int per = nb / NXCD;
    if (bid < per * NXCD) bid = (bid % NXCD) * per + bid / NXCD;
    const int group = GROUP_M * nbn;
    const int gid = bid / group;
    const int first_m = gid * GROUP_M;
    const int gsz = min(nbm - first_m, GROUP_M);
    const int in_g = bid - gid * group;
    tm = first_m + in_g % gsz;
    tn = in_g / gsz;
}

// SUCC: successor mode (A = W with its diagonal treated as absent, B = D,
// output S); otherwise the witness product.
template <typename T, int SR, bool VEC, bool SUCC>
__global__ __launch_bounds__(WT_NT) void witness_gemm_kernel(WitnessArgs<T> a) {
    using R = Ring<SR, T>;
    __shared__ __align__(16) T As[WT_BK][WT_BM + WT_APAD];
    __shared__ __align__(16) T Bs[WT_BK][WT_BN];

    const int nbm = (a.m + WT_BM - 1) / WT_BM, nbn = (a.n + WT_BN - 1) / WT_BN;
    int tm, tn;
    wt_tile_of(blockIdx.x, nbm * nbn, nbm, nbn, tm, tn);
    const int m0 = tm * WT_BM, n0 = tn * WT_BN;
    const int tid = threadIdx.x, tx = tid % 16, ty = tid / 16;

    // staging: each thread moves WT_VW consecutive elements of A (row ar,
    // columns ac..) and of B (row br, columns bc..) per k-block
    typedef T V __attribute__((ext_vector_type(WT_VW)));
    const int ar = tid / (WT_BK / WT_VW), ac = (tid % (WT_BK / WT_VW)) * WT_VW;
    const int br = tid / (WT_BN / WT_VW), bc = (tid % (WT_BN / WT_VW)) * WT_VW;
    T ra[WT_VW], rb[WT_VW];

    auto load = [&](int k0) {
        const int gi = m0 + ar, gp = k0 + ac;
        if (VEC && gi < a.m && gp + WT_VW <= a.k) {
            const V v = *reinterpret_cast<const V*>(a.A + (long)gi * a.lda + gp);
#pragma unroll
            for (int q = 0; q < WT_VW; ++q) ra[q] = v[q];
        } else {
#pragma unroll
            for (int q = 0; q < WT_VW; ++q)
                ra[q] = (gi < a.m && gp + q < a.k) ? a.A[(long)gi * a.lda + gp + q] : R::absent();
        }
        if constexpr (SUCC) {
#pragma unroll
            for (int q = 0; q < WT_VW; ++q)
                if (gi == gp + q) ra[q] = R::absent();
        }
        const int gk = k0 + br, gj = n0 + bc;
        if (VEC && gk < a.k && gj + WT_VW <= a.n) {
            const V v = *reinterpret_cast<const V*>(a.B + (long)gk * a.ldb + gj);
#pragma unroll
            for (int q = 0; q < WT_VW; ++q) rb[q] = v[q];
        } else {
#pragma unroll
            for (int q = 0; q < WT_VW; ++q)
                rb[q] = (gk < a.k && gj + q < a.n) ? a.B[(long)gk * a.ldb + gj + q] : R::absent();
        }
    };

    T acc[WT_TM][WT_TN];
    int blk[WT_TM][WT_TN];  // witness block where acc was first attained, -1 while absent
    T bm[WT_TM][WT_TN];     // extreme of the current witness block
    constexpr int WT_WB = wt_wb<SUCC>();
#pragma unroll
    for (int r = 0; r < WT_TM; ++r)
#pragma unroll
        for (int c = 0; c < WT_TN; ++c) {
            acc[r][c] = R::absent();
            blk[r][c] = -1;
        }

    const int nkb = (a.k + WT_BK - 1) / WT_BK;
    if (nkb > 0) load(0);
    for (int kb = 0; kb < nkb; ++kb) {
        const int k0 = kb * WT_BK;
        __syncthreads();
#pragma unroll
        for (int q = 0; q < WT_VW; ++q) {
            As[ac + q][ar] = ra[q];
            Bs[br][bc + q] = rb[q];
        }
        __syncthreads();
        if (kb + 1 < nkb) load(k0 + WT_BK);

        // block extreme of every output over the 32 terms of this witness
        // block (two k-blocks)
        if (kb % WT_WB == 0) {
#pragma unroll
            for (int r = 0; r < WT_TM; ++r)
#pragma unroll
                for (int c = 0; c < WT_TN; ++c) bm[r][c] = R::absent();
        }
// (two k-pairs per iteration: a full unroll hoists every LDS read and
        // doubles the register count)
#pragma unroll 2
        for (int kk = 0; kk < WT_BK; kk += 2) {
            const auto a0 = *reinterpret_cast<const HIP_vector_type<T, 4>*>(&As[kk][ty * WT_TM]);
            const auto a1 = *reinterpret_cast<const HIP_vector_type<T, 4>*>(&As[kk + 1][ty * WT_TM]);
            const auto b0 = *reinterpret_cast<const HIP_vector_type<T, 4>*>(&Bs[kk][tx * WT_TN]);
            const auto b1 = *reinterpret_cast<const HIP_vector_type<T, 4>*>(&Bs[kk + 1][tx * WT_TN]);
            const T av0[4] = {a0.x, a0.y, a0.z, a0.w}, av1[4] = {a1.x, a1.y, a1.z, a1.w};
            const T bv0[4] = {b0.x, b0.y, b0.z, b0.w}, bv1[4] = {b1.x, b1.y, b1.z, b1.w};
#pragma unroll
            for (int r = 0; r < WT_TM; ++r)
#pragma unroll
                for (int c = 0; c < WT_TN; ++c)
                    bm[r][c] = R::add3(bm[r][c], R::mul(av0[r], bv0[c]), R::mul(av1[r], bv1[c]));
        }

        // at the end of a witness block, outputs whose block extreme strictly
        // beats the running best take it and remember the block
        if (kb % WT_WB == WT_WB - 1 || kb + 1 == nkb) {
#pragma unroll
            for (int r = 0; r < WT_TM; ++r)
#pragma unroll
                for (int c = 0; c < WT_TN; ++c) {
                    const T v = R::finish(bm[r][c]);
                    const bool imp = better<SR>(v, acc[r][c]);
                    acc[r][c] = imp ? v : acc[r][c];
                    blk[r][c] = imp ? kb / WT_WB : blk[r][c];
                }
        }
    }

#pragma unroll
    for (int r = 0; r < WT_TM; ++r) {
        const int i = m0 + ty * WT_TM + r;
        if (i >= a.m) continue;
#pragma unroll
        for (int c = 0; c < WT_TN; ++c) {
            const int j = n0 + tx * WT_TN + c;
            if (j >= a.n) continue;
            bool store;
            if constexpr (SUCC) {
                store = i != j;
                if (i == j) a.K[(long)i * a.ldk + j] = i;
            } else {
                store = blk[r][c] >= 0 && better<SR>(acc[r][c], a.C[(long)i * a.ldc + j]);
            }
            if (!store) continue;
            // the first index of the remembered block whose term equals the
            // value (a finite value is the raw block extreme, which one of the
            // block's terms attains)
            int first = -1;
            if (blk[r][c] >= 0) {
                const int p0 = blk[r][c] * (WT_WB * WT_BK);
                for (int q = WT_WB * WT_BK - 1; q >= 0; --q) {
                    const int p = p0 + q;
                    if (p >= a.k) continue;
                    T x = a.A[(long)i * a.lda + p];
                    if (SUCC && i == p) x = R::absent();
                    if (R::mul(x, a.B[(long)p * a.ldb + j]) == acc[r][c]) first = p;
                }
            }
            if constexpr (SUCC) {
                a.K[(long)i * a.ldk + j] = first;
            } else {
                a.C[(long)i * a.ldc + j] = acc[r][c];
                a.K[(long)i * a.ldk + j] = first;
            }
        }
    }
}

template <typename T, int SR, bool SUCC>
hipError_t launch_typed(WitnessArgs<T> a, hipStream_t s) {
    if (a.m <= 0 || a.n <= 0) return hipSuccess;
    const long tiles = (long)((a.m + WT_BM - 1) / WT_BM) * ((a.n + WT_BN - 1) / WT_BN);
    if (tiles > 0x7FFFFFFFL) return hipErrorInvalidValue;
    const bool vec = a.lda % 4 == 0 && a.ldb % 4 == 0 && (uintptr_t)a.A % 16 == 0 &&
                     (uintptr_t)a.B % 16 == 0;
    if (vec)
        hipLaunchKernelGGL((witness_gemm_kernel<T, SR, true, SUCC>), dim3((unsigned)tiles),
                           dim3(WT_NT), 0, s, a);
    else
        hipLaunchKernelGGL((witness_gemm_kernel<T, SR, false, SUCC>), dim3((unsigned)tiles),
                           dim3(WT_NT), 0, s, a);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_gemm_witness(int sr, int dt, int m, int n, int k, const void* A, long lda,
                               const void* B, long ldb, void* C, long ldc, int32_t* K, long ldk,
                               hipStream_t s) {
    if (dt == BTAS_FLOAT32) {
        WitnessArgs<float> a{m, n, k, (const float*)A, lda, (const float*)B, ldb, (float*)C, ldc, K, ldk};
        return sr == BTAS_MIN_PLUS ? launch_typed<float, BTAS_MIN_PLUS, false>(a, s)
                                   : launch_typed<float, BTAS_MAX_PLUS, false>(a, s);
    }
    WitnessArgs<int32_t> a{m, n, k, (const int32_t*)A, lda, (const int32_t*)B, ldb, (int32_t*)C, ldc, K, ldk};
    return sr == BTAS_MIN_PLUS ? launch_typed<int32_t, BTAS_MIN_PLUS, false>(a, s)
                               : launch_typed<int32_t, BTAS_MAX_PLUS, false>(a, s);
}

hipError_t launch_successors(int dt, int n, const void* W, long ldw, const void* D, long ldd,
                             int32_t* S, long lds, hipStream_t s) {
    if (dt == BTAS_FLOAT32) {
        WitnessArgs<float> a{n, n, n, (const float*)W, ldw, (const float*)D, ldd, nullptr, 0, S, lds};
        return launch_typed<float, BTAS_MIN_PLUS, true>(a, s);
    }
    WitnessArgs<int32_t> a{n, n, n, (const int32_t*)W, ldw, (const int32_t*)D, ldd, nullptr, 0, S, lds};
    return launch_typed<int32_t, BTAS_MIN_PLUS, true>(a, s);
}

}  // namespace btas
