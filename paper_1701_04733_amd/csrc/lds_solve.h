// A whole APSP solve of one small graph (n <= 64) by one workgroup of 1024
// threads, both ping-pong matrices in LDS (internal).
//
//   D_0 = I (+) W;  for t = 1..nsq:  D_t = D_{t-1} (+) D_{t-1} (.) D_{t-1}
//
// (Sec. III repeated squaring) with a workgroup barrier between squarings.
// Lane j of wave w computes column j of rows w, w+16, w+32, w+48: per four k
// it reads the column's four entries once and each row's four entries as one
// 16-byte broadcast read.  The early-exit decision is the OR of the
// workgroup's change bits.  The terms and the per-output mapping of int32
// sums are those of every other squaring kernel, so the bits are the same.
#pragma once

#include <hip/hip_runtime.h>

#include "gemm_tile.h"
#include "semiring.h"

namespace btas {

constexpr int LDS_SOLVE_MAX_N = 64;
constexpr int LDS_SOLVE_NT = 1024;
constexpr int LDS_SOLVE_LS = LDS_SOLVE_MAX_N + 4;  // row stride: 16-byte aligned rows

// Shared memory of one solve.
template <typename T>
struct LdsSolveBuffers {
    T buf[2][LDS_SOLVE_MAX_N * LDS_SOLVE_LS];
};

// Every thread of the workgroup calls it; returns the squarings run.  D may
// equal W (in place); D is written only after W has been read.
template <typename T>
__device__ int lds_solve_graph(int n, const T* __restrict__ W, long ldw, T* D, long ldd, int nsq,
                               int early, LdsSolveBuffers<T>& sm) {
    using R = Ring<BTAS_MIN_PLUS, T>;
    T (&buf)[2][LDS_SOLVE_MAX_N * LDS_SOLVE_LS] = sm.buf;
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
    return steps;
}

}  // namespace btas
