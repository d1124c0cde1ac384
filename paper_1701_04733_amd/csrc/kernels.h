// Host-side launchers of the tropical kernels (internal to libbtas).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "btas.h"

namespace btas {

// Cout <- Cin (+) A (.) B ; `changed` (device int, may be null) is set to 1
// when some output differs bitwise from its Cin value.
struct GemmArgs {
    int m, n, k;
    const void* A;
    long lda;
    const void* B;
    long ldb;
    const void* Cin;
    long ldci;
    void* Cout;
    long ldco;
    int* changed;
    // int32 only (ignored for float32): wide_in points at a device flag that
    // is 0 when every finite element of A and B fits in +-FP32_EXACT_MAX (the
    // product then runs exactly on the binary32 pipeline); wide_out, if not
    // null, is set to 1 when a finite output element does not fit.
    const int* wide_in;
    int* wide_out;
    // Optional split-K workspace (device, ws_bytes bytes).  When the output has
    // too few tiles to fill the GPU and k is long, the k range is cut into S
    // chunks whose partial products go to ws and a reduce pass (+)-combines
    // them with Cin.  Exact: (+) is associative, commutative and idempotent.
    void* ws;
    size_t ws_bytes;
};

// Split-K workspace that launch_gemm may use for an m x n x k product.
size_t gemm_splitk_bytes(int m, int n, int k);

enum { GEMM_CFG_L = 0, GEMM_CFG_M = 1, GEMM_CFG_S = 2, GEMM_NUM_CFGS = 3 };

struct GemmPlan {
    int cfg;     // GEMM_CFG_*
    int splits;  // split-K chunks (1: none)
};
// Configuration launch_gemm uses for an m x n x k product (cfg < 0).
GemmPlan plan_gemm(int m, int n, int k);
hipError_t launch_gemm(int sr, int dt, const GemmArgs& a, int cfg, hipStream_t s);

// y <- y (+) A (.) x
hipError_t launch_gemv(int sr, int dt, int m, int n, const void* A, long lda, const void* x,
                       long incx, void* y, long incy, hipStream_t s);

// Level 1.  op: 0 = vadd (z = x (+) y), 1 = vmul (z = x (.) y).
hipError_t launch_vec_binary(int op, int sr, int dt, int n, const void* x, long incx,
                             const void* y, long incy, void* z, long incz, hipStream_t s);
// y <- y (+) alpha (.) x ; alpha passed by bits.
hipError_t launch_axpy(int sr, int dt, int n, uint32_t alpha_bits, const void* x, long incx,
                       void* y, long incy, hipStream_t s);
// result <- (+)_i x_i (.) y_i via a two-pass reduction through `partials`
// (at least dot_partials_needed(n) elements of 4 bytes).
int dot_partials_needed(int n);
hipError_t launch_dot(int sr, int dt, int n, const void* x, long incx, const void* y, long incy,
                      void* partials, void* result, hipStream_t s);

// APSP helpers.
// dst <- I (+) W  (copy with dst_ii = min(W_ii, 0)); dst may equal W.  For
// int32, `wide` (may be null) is set to 1 if a finite element of dst exceeds
// +-FP32_EXACT_MAX.
hipError_t launch_apsp_init(int dt, int n, const void* W, long ldw, void* dst, long ldd,
                            int* wide, hipStream_t s);
// int32: flag <- 1 if a finite element (not the semiring's absent value) of the
// m x n matrix exceeds +-FP32_EXACT_MAX.
hipError_t launch_range_scan(int sr, int m, int n, const void* X, long ld, int* flag,
                             hipStream_t s);
// flag[0..count) <- 0 (a kernel, not a memset, so it is safe inside graphs).
hipError_t launch_clear_flags(int* flag, int count, hipStream_t s);
// flag <- 1 if some D_ii < 0.
hipError_t launch_neg_diag_check(int dt, int n, const void* D, long ldd, int* flag,
                                 hipStream_t s);
// Either semiring: dst <- I (+) W (dst_ii = min(W_ii, 0), resp. max(W_ii, 0));
// flag <- 1 if some D_ii is past 0 on the improving side (min-plus: < 0,
// max-plus: > 0).
hipError_t launch_closure_init(int sr, int dt, int n, const void* W, long ldw, void* dst, long ldd,
                               int* wide, hipStream_t s);
hipError_t launch_diag_check(int sr, int dt, int n, const void* D, long ldd, int* flag,
                             hipStream_t s);
// Zero `words` 64-bit words at p (8-byte aligned).
hipError_t launch_zero_words(void* p, size_t words, hipStream_t s);
// Copy an n-column, m-row matrix between leading dimensions (4-byte elements).
hipError_t launch_copy_matrix(int m, int n, const void* src, long lds, void* dst, long ldd,
                              hipStream_t s);
// Whole APSP solve in one launch (n <= RESIDENT_MAX_N): D_0 = I (+) W, then
// T squarings (or fewer with early exit); n <= 64: one workgroup with both
// matrices in LDS; larger n: a cooperative launch with a device-wide barrier
// between squarings, ping-ponging between D and ws (n x n, leading
// dimension n).  The result ends in D.  flags (device, 2 + 2 *
// RESIDENT_MAX_GRID words): [0] <- epoch on a barrier timeout, [1] <- the
// number of squarings run, [2..] the barrier's arrival words, tagged with
// epoch (1 .. 2^24 - 1, larger than the tag of every word already there:
// zero the words before the first epoch and whenever the count restarts).
// latch: a pinned host word also set to 1 on a barrier timeout (never
// cleared by the kernel).  allow_u16 (int32, 64 < n): square in the packed
// 16-bit mode when the weights pass its gate (checked on the device; ws
// then needs resident_ws_bytes).  num_cus: compute units of the device; spin_limit:
// polls per barrier wait before giving up (negative: every wait reports a
// timeout at once, for tests of the error path).  tagws (may be null): a
// buffer of resident_tag_bytes() that only these launches write, zeroed
// like the arrival words; with it, a solve whose grid has one workgroup per
// 16x16 tile runs the tagged mode (no device-wide barrier).  Without it, a
// fixed-T solve of that shape waits per squaring for the workgroups of its
// row and column panels only.
constexpr int RESIDENT_MAX_N = 500;  // keeps the workgroup's LDS within 64 KB
constexpr int RESIDENT_MAX_GRID = 1024;  // (500 / 16 rounded up)^2 tiles
constexpr int RESIDENT_TAG_STEPS = 32;   // squarings the tagged mode's change words cover
size_t resident_tag_bytes();
// Up to this size the single-launch solve beats one launch per squaring on
// MI355X (measured latency, int32 ER graphs of mean degree 12.75, fixed T:
// n=8 23 us vs 34 us, n=64 48 vs 93 (one workgroup, n <= 64); tagged mode:
// n=129 64 vs 155, n=256 79 vs 171, n=288 132 vs 216, n=352 139 vs 240;
// with the device-wide barrier, n=400 322 vs 251).
constexpr int AUTO_SINGLE_LAUNCH_MIN_N = 1;
constexpr int AUTO_SINGLE_LAUNCH_N = 352;
constexpr int AUTO_SINGLE_LAUNCH_BARRIER_N = 256;  // without the tagged mode (barrier: n=320 235 vs 212)
size_t resident_lds_bytes(int n);
// Bytes of `ws` a single-launch solve uses: the n x n int32/fp32 partner and,
// for int32 graphs that take the cooperative launch (64 < n <= RESIDENT_MAX_N),
// two n x round_up(n, 8) matrices of 16-bit distances for the packed mode.
size_t resident_ws_bytes(int dt, int n);
// Set in flags[1] (beside the step count) by a solve that ran the packed
// 16-bit mode.
constexpr int RESIDENT_PACKED16_BIT = 1 << 16;
// Fixed workspace of the no-allocation APSP entry point (per GPU): the
// ping-pong partner (n*n*4 bytes, so n <= NOALLOC_MAX_N) and, in what is left,
// split-K partial products.
constexpr size_t NOALLOC_SCRATCH_BYTES = (size_t)32 << 20;
constexpr int NOALLOC_MAX_N = 2896;
static_assert((size_t)NOALLOC_MAX_N * NOALLOC_MAX_N * 4 <= NOALLOC_SCRATCH_BYTES &&
                  (size_t)(NOALLOC_MAX_N + 1) * (NOALLOC_MAX_N + 1) * 4 > NOALLOC_SCRATCH_BYTES,
              "NOALLOC_MAX_N is the largest n whose partner matrix fits");
hipError_t launch_apsp_resident(int dt, int n, const void* W, long ldw, void* D, long ldd,
                                void* ws, void* tagws, int T, bool early, int* flags, int* latch,
                                int num_cus, int spin_limit, bool allow_u16, unsigned epoch,
                                hipStream_t s);
// Blocked Floyd-Warshall in place on D (n x n, leading dimension ld), which
// holds I (+) W: pivot blocks of fw_block_size() vertices, three launches per
// block (diagonal block, its block-row and block-column, the rest).
int fw_block_size();
hipError_t launch_floyd_warshall(int dt, int n, void* D, long ld, hipStream_t s);
// Blocked FW of many graphs: per graph its input, output (may be the input
// with the same ld: in place), size and pivot-block count; work items name a
// graph and a block index.  phase 0: D <- I (+) W, item idx = 64-row block;
// phase 1: diagonal block kb (idx unused); phase 2: the 2(nb-1) panel blocks
// of kb (idx); phase 3: the (nb-1)^2 other blocks (idx).  vec: every graph's
// ldd is a multiple of 4 and D 16-byte aligned.
struct FwGraph {
    const void* W;
    long ldw;
    void* D;
    long ldd;
    int n;
    int nb;
};
struct FwItem {
    int graph;
    int idx;
};
// Launch kinds of the batched blocked Floyd-Warshall (items name a graph and
// a block or tile index within that launch's list for the graph): D = I (+) W
// by 64-row slabs; phases 1 and 2 of pivot block kb; phase 3 of kb (every
// block outside its row and column); kb's update of block-row and
// block-column kb+1 (STRIP_NEXT) or kb-1 (STRIP_PREV); and the k=128 update of
// the 128x128 tiles outside tile-row and tile-column kb/2 (PAIR, kb even).
enum FwbPhase { FWB_INIT, FWB_PHASE1, FWB_PHASE2, FWB_PHASE3, FWB_STRIP_NEXT, FWB_STRIP_PREV, FWB_PAIR };
hipError_t launch_fw_batched(int dt, int phase, const FwGraph* graphs, const FwItem* items, int nitems,
                             int kb, bool vec, hipStream_t s);

// Sparse-aware APSP squarings (csrc/sparse.hip), min-plus.  count: rownnz[i]
// = finite entries of row i of D, counters[0] += total.  build: row pointers
// (n + 1) and the CSR of D (capacity >= the total), counters[1] += the
// squaring's term count.  square: E = D (+) D (.) D from the CSR, row by row
// (LDS of sparse_step_lds_bytes(n) per workgroup), changed / wide_out flags
// as in the dense product.
size_t sparse_step_lds_bytes(int n);
// skip_diag: leave out the diagonal (a graph's edges without self loops).
hipError_t launch_sparse_count(int dt, int n, const void* D, long ld, int* rownnz,
                               unsigned long long* counters, hipStream_t s, bool skip_diag = false);
hipError_t launch_sparse_build(int dt, int n, const void* D, long ld, const int* rownnz, int* rowptr,
                               int* cols, void* vals, unsigned long long* counters, hipStream_t s,
                               bool skip_diag = false);
// Successors from the CSR of W without its diagonal (column order kept):
// the same S as launch_successors, one row per workgroup, |row i| terms per
// entry instead of n.
hipError_t launch_sparse_successors(int dt, int n, const int* rowptr, const int* cols,
                                    const void* vals, const void* D, long ldd, int32_t* S, long lds,
                                    hipStream_t s);
hipError_t launch_sparse_square(int dt, int n, const void* D, long ld, void* E, long lde,
                                const int* rowptr, const int* cols, const void* vals, int* changed,
                                int* wide_out, hipStream_t s);

// Maximum cycle mean of a max-plus matrix by Karp's theorem (csrc/maxplus.hip).
// maxabs: *out = max |A_ij| over present int32 entries (atomicMax, clear first).
// cycle_mean: ws of cycle_mean_ws_bytes(n) bytes; the n max-plus products
// x_{k+1} = A (x) x_k as one cooperative launch (n <= 4096 and n/16 <=
// num_cus; *uses_err = 1, and after synchronising the word at
// cycle_mean_error_word(n, ws) is nonzero if a barrier wait timed out) or n
// gemv launches (*uses_err = 0); then result[0..1] = the int32 fraction in
// lowest terms (den = 0: no cycle), result[2] = the bits of lambda as a
// binary64 (-inf: no cycle).
size_t cycle_mean_ws_bytes(int n);
hipError_t launch_cycle_mean_maxabs(int n, const void* A, long lda, int* out, hipStream_t s);
hipError_t launch_cycle_mean(int dt, int n, const void* A, long lda, void* ws, long long* result,
                             int num_cus, int* uses_err, hipStream_t s);
const int* cycle_mean_error_word(int n, const void* ws);

// Tropical product with witnesses (csrc/witness.hip): C <- C (+) A (.) B and,
// where an entry strictly improves, K <- the smallest p attaining it.
hipError_t launch_gemm_witness(int sr, int dt, int m, int n, int k, const void* A, long lda,
                               const void* B, long ldb, void* C, long ldc, int32_t* K, long ldk,
                               hipStream_t s);
// Successors of a (min-plus) distance matrix: S_ii = i; for i != j the
// smallest u != i minimising W_iu (.) D_uj, -1 if every term is absent.
hipError_t launch_successors(int dt, int n, const void* W, long ldw, const void* D, long ldd,
                             int32_t* S, long lds, hipStream_t s);
// Domain scan (BTAS_VALIDATE=1): flag <- 1 if some element of the m x n matrix
// is not a legal (.) operand of the semiring.
hipError_t launch_domain_scan(int sr, int dt, int m, int n, const void* X, long ld, int* flag,
                              hipStream_t s);

}  // namespace btas
