/*
 * btas.h -- Basic Tropical Algebra Subroutines for AMD Instinct MI355X (gfx950).
 *
 * A BLAS-style C ABI for tropical linear algebra over the max-plus and
 * min-plus semirings (Sec. I, eqs. (1)-(4)):
 *     max-plus:  x (+) y = max(x, y),   x (.) y = x + y
 *     min-plus:  x (+) y = min(x, y),   x (.) y = x + y
 * and for all-pairs shortest paths by repeated min-plus squaring of the
 * weighted adjacency matrix (Sec. III).  The library is motivated as the
 * tropical counterpart of the standard vector and matrix routines of BLAS
 * (Abstract; Sec. II); no signatures are given there, so these follow BLAS
 * conventions.
 *
 * General rules
 *  - Every call returns btas_status_t; nothing throws across the ABI.
 *  - Matrices are row-major with a leading dimension (elements between the
 *    starts of consecutive rows), as the adjacency matrix of Sec. IV is
 *    indexed.  Column-major callers use (A (.) B)^T = B^T (.) A^T.
 *  - Matrix and vector pointers are DEVICE pointers owned by the caller; the
 *    library never frees or retains them past the call's stream work.  Only
 *    btas_tropical_axpy's alpha and the *_out / counts arguments explicitly
 *    documented as host memory are host pointers.
 *  - Element types: BTAS_INT32 (int32_t) and BTAS_FLOAT32 (IEEE binary32).
 *  - Absent values (the (+)-identity): for int32, BTAS_I32_INF in min-plus and
 *    BTAS_I32_NEG_INF in max-plus; they absorb under (.) (saturating, never
 *    wrapping).  For float32, +inf / -inf.  Finite int32 operands of (.) must
 *    satisfy |x| <= BTAS_I32_FINITE_MAX; float32 operands must not be NaN and
 *    must not be the other semiring's infinity.  Out-of-domain input gives
 *    unspecified values (no fault); with the environment variable
 *    BTAS_VALIDATE=1 it is detected and reported as BTAS_ERR_DOMAIN before
 *    any output is written.
 *  - float32: each (.) is one IEEE binary32 round-to-nearest-even addition,
 *    denormals preserved, no contraction; since min/max are exact and
 *    rounding is monotone the result does not depend on reduction order and
 *    is bit-reproducible.
 *  - Calls are asynchronous on the handle's stream unless stated otherwise.
 *    A handle must be used by one host thread at a time.
 *  - Errors: arguments are checked before anything is launched (as BLAS's
 *    xerbla does); btas_last_error(h) then names the offending argument.
 *    A HIP launch or synchronisation failure is BTAS_ERR_DEVICE.
 *  - Degenerate sizes: a zero output size is a no-op returning BTAS_OK; a
 *    zero reduction length leaves the accumulator unchanged (the (+) over an
 *    empty set is the identity).
 */
#ifndef BTAS_H
#define BTAS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum { BTAS_MIN_PLUS = 0, BTAS_MAX_PLUS = 1 } btas_semiring_t;
typedef enum { BTAS_INT32 = 0, BTAS_FLOAT32 = 1 } btas_dtype_t;

typedef enum {
    BTAS_OK = 0,
    BTAS_ERR_INVALID_ARG = 1, /* bad size, leading dimension, stride, enum or null pointer */
    BTAS_ERR_ALIAS = 2,       /* output overlaps an input where that is not allowed       */
    BTAS_ERR_DOMAIN = 3,      /* an element outside the domain (BTAS_VALIDATE=1 scans; a
                                 few entry points check their own ranges always)           */
    BTAS_ERR_OOM = 4,         /* device workspace allocation failed                      */
    BTAS_ERR_DEVICE = 5,      /* HIP runtime error (launch, copy, synchronisation)         */
    BTAS_ERR_UNSUPPORTED = 6, /* combination not provided                                  */
    BTAS_WARN_NEG_CYCLE = 7,  /* APSP result has some D_ii < 0 (result unspecified)        */
    BTAS_WARN_POS_CYCLE = 8   /* max-plus closure has some D_ii > 0 (result unspecified)   */
} btas_status_t;

#define BTAS_I32_INF ((int32_t)0x7FFFFFFF)      /* min-plus absent value, +INF  */
#define BTAS_I32_NEG_INF ((int32_t)-0x7FFFFFFF) /* max-plus absent value, -INF  */
#define BTAS_I32_FINITE_MAX ((1 << 29) - 1)     /* |finite (.) operand| bound   */

typedef struct btas_ctx *btas_handle_t;

/* Create a handle bound to HIP device `device` (made current for the call).
 * The handle starts on the default (null) stream and owns its workspace.
 * h: host pointer receiving the handle.  Errors: INVALID_ARG (null h, bad
 * device), DEVICE. */
btas_status_t btas_create(btas_handle_t *h, int device);

/* Release the handle and its workspace (synchronises its stream first). */
btas_status_t btas_destroy(btas_handle_t h);

/* Use `hip_stream` (a hipStream_t, borrowed, not owned; NULL = default
 * stream) for all later work of this handle.  The handle's workspaces (the
 * APSP partner matrix, split-K partials, the single launch's tag buffer and
 * barrier words) serve every call on it, so work still running on the
 * previous stream must be ordered before the new stream's (for example by
 * btas_synchronize) by the caller. */
btas_status_t btas_set_stream(btas_handle_t h, void *hip_stream);

/* Block the host until the handle's stream has drained.  Returns
 * BTAS_ERR_DEVICE on a HIP error, or (once) when an earlier asynchronous
 * single-launch APSP solve on this handle hit the bound of one of its waits
 * on other workgroups (see BTAS_APSP_SINGLE_LAUNCH); every other entry point reports that latched
 * error too, on its next call, instead of doing its work. */
btas_status_t btas_synchronize(btas_handle_t h);

/* Static text for a status code. */
const char *btas_status_string(btas_status_t s);

/* Text describing the last failure on this handle ("" if none).  Valid until
 * the next call on the handle. */
const char *btas_last_error(btas_handle_t h);

/* Library version string. */
const char *btas_version(void);

/* ---------------------------------------------------------------------------
 * Level 3 -- tropical matrix product with accumulate (Sec. IV, min-plus form
 * of the matrix-product listing):  C <- C (+) A (.) B, i.e.
 *     c_ij <- c_ij (+) ( (+)_p  a_ip (.) b_pj ).
 * A is m x k (lda >= max(1,k)), B is k x n (ldb >= max(1,n)), C is m x n
 * (ldc >= max(1,n)), all row-major device arrays of dtype `dt`.  C is read
 * and written; it must not overlap A or B (BTAS_ERR_ALIAS).  Pass C filled
 * with the absent value for a plain product.  Any int32 value is accepted in
 * C (it is only (+)-combined).
 */
btas_status_t btas_tropical_gemm(btas_handle_t h, btas_semiring_t sr, btas_dtype_t dt,
                                 int m, int n, int k,
                                 const void *A, int lda, const void *B, int ldb,
                                 void *C, int ldc);

/* Level 2 -- y <- y (+) A (.) x, i.e. y_i <- y_i (+) (+)_j a_ij (.) x_j.
 * A is m x n row-major (lda >= max(1,n)); x has n elements with stride incx
 * >= 1; y has m elements with stride incy >= 1.  y must not overlap A or x. */
btas_status_t btas_tropical_gemv(btas_handle_t h, btas_semiring_t sr, btas_dtype_t dt,
                                 int m, int n, const void *A, int lda,
                                 const void *x, int incx, void *y, int incy);

/* Level 1 (strides >= 1, n >= 0).  z may equal x or y exactly (elementwise
 * in place) but must not partially overlap them. */
/* z_i = x_i (+) y_i */
btas_status_t btas_tropical_vadd(btas_handle_t h, btas_semiring_t sr, btas_dtype_t dt, int n,
                                 const void *x, int incx, const void *y, int incy,
                                 void *z, int incz);
/* z_i = x_i (.) y_i */
btas_status_t btas_tropical_vmul(btas_handle_t h, btas_semiring_t sr, btas_dtype_t dt, int n,
                                 const void *x, int incx, const void *y, int incy,
                                 void *z, int incz);
/* *result_dev = (+)_i x_i (.) y_i  (one element of dtype dt in device
 * memory; n = 0 stores the absent value). */
btas_status_t btas_tropical_dot(btas_handle_t h, btas_semiring_t sr, btas_dtype_t dt, int n,
                                const void *x, int incx, const void *y, int incy,
                                void *result_dev);
/* y_i <- y_i (+) alpha (.) x_i; alpha_host points to one host element of
 * dtype dt, read during the call. */
btas_status_t btas_tropical_axpy(btas_handle_t h, btas_semiring_t sr, btas_dtype_t dt, int n,
                                 const void *alpha_host, const void *x, int incx,
                                 void *y, int incy);

/* ---------------------------------------------------------------------------
 * All-pairs shortest paths by repeated min-plus squaring (Sec. III).
 *   D_0 = I (+) W   (I: 0 on the diagonal, absent elsewhere; so D_ii =
 *                    min(W_ii, 0)),
 *   D_t = D_{t-1} (+) D_{t-1} (.) D_{t-1}   for t = 1..T,
 *   T   = ceil(log2(n-1)) for n > 2, else 0,
 * each step reading only the previous step's matrix (out-of-place).  W and D
 * are n x n row-major device matrices (ldw, ldd >= max(1,n)); D may equal W
 * (in place) but must not partially overlap it.  Only min-plus is provided
 * (BTAS_ERR_UNSUPPORTED is never returned for valid dtypes).
 * Flags:
 *   BTAS_APSP_EARLY_EXIT: stop after the first step whose output equals its
 *     input bit for bit (that step is counted).  Same result as fixed T.
 *     Reads a device flag back after every step (host synchronisation).
 *     On this path, for 4096 <= n <= 16384, a squaring whose input has at
 *     most n^2/8 finite entries and whose term count makes it cheaper runs
 *     as a sparse product (the input compressed to rows of finite entries,
 *     each output row accumulated in LDS); the result is bit-identical (the
 *     same min of the same rounded terms).  Its workspace (n^2 + 8n bytes)
 *     is kept by the handle; if it cannot be allocated the step runs dense.
 *     BTAS_SPARSE_STEPS=0 in the environment disables it; =force uses it
 *     for any n <= 16384 while the density limit holds.
 *   BTAS_APSP_CHECK_NEG_CYCLE: after the last step, return
 *     BTAS_WARN_NEG_CYCLE if some D_ii < 0 (synchronises).
 *   BTAS_APSP_GRAPH: capture the whole fixed-T solve into a hipGraph on the
 *     first call with a given (dtype, n, W, ldw, D, ldd) and replay it on later
 *     calls (one launch per solve; for latency-bound small n).  The handle
 *     keeps one such graph.  Not combinable with EARLY_EXIT.
 *   BTAS_APSP_SINGLE_LAUNCH: for n <= 500, run the whole solve (init, every
 *     squaring, and with EARLY_EXIT the stop test) as one kernel launch: one
 *     workgroup with the matrices in LDS for n <= 64, else a cooperative
 *     launch.  When every 16x16 output tile can have a resident workgroup of
 *     its own, squarings are ordered by the data alone: each workgroup
 *     re-reads the entries of D_{t-1} it needs until their tags (64-bit words
 *     of value and launch/step tag, in a tag buffer the handle allocates once,
 *     about 4 MB) say they are current, and early exit reads one change word
 *     per workgroup and squaring; otherwise a device-wide barrier separates
 *     squarings.  No per-step
 *     launches and no host round trip, also with EARLY_EXIT (the host then
 *     synchronises only if steps_out is not NULL).  Larger n ignore the flag.
 *     Not combinable with GRAPH.  BTAS_ERR_DEVICE if the device cannot launch
 *     it cooperatively, or if a wait on other workgroups timed out (D is then not
 *     valid): reported by this call when steps_out is not NULL, else latched
 *     on the handle and reported by its next call or btas_synchronize.  The
 *     environment variable BTAS_TEST_SPIN_LIMIT, read by btas_create, sets
 *     the bound of each wait in polls (a negative value reports a timeout at
 *     every wait, for tests of this path).  Calls without GRAPH take this path
 *     for n <= 352 (n <= 256 in btas_apsp_squaring_noalloc) even without the flag (it is the faster one there), unless the
 *     environment variable BTAS_SINGLE_LAUNCH=0 is set; such a call whose
 *     cooperative launch is refused runs one launch per squaring instead.
 * steps_out: host int receiving the number of squarings executed (may be
 * NULL; when non-NULL the call synchronises).  Integer contract: all finite
 * path lengths must stay within +-BTAS_I32_FINITE_MAX.  The handle keeps an
 * n x n workspace matrix between calls (grown on demand).
 */
#define BTAS_APSP_EARLY_EXIT 1u
#define BTAS_APSP_CHECK_NEG_CYCLE 2u
#define BTAS_APSP_GRAPH 4u
#define BTAS_APSP_SINGLE_LAUNCH 8u
btas_status_t btas_apsp_squaring(btas_handle_t h, btas_dtype_t dt, int n,
                                 const void *W, int ldw, void *D, int ldd,
                                 unsigned flags, int *steps_out);

/* The same solve as btas_apsp_squaring, for callers that cannot allocate
 * device memory during the call (code under stream capture, tight serving
 * loops, harnesses that forbid hipMalloc).  The call allocates nothing: the
 * ping-pong partner matrix and split-K partial products live in a fixed
 * 32 MiB device array held by the library on each GPU it runs on until the
 * process ends, so n <= 2896 (larger n: BTAS_ERR_INVALID_ARG, nothing
 * launched).  The caller passes W and D as for btas_apsp_squaring; flags as
 * there except BTAS_APSP_GRAPH (BTAS_ERR_INVALID_ARG: capture allocates); the
 * sparse first squarings are not used (same result).  Every call on one GPU
 * shares that GPU's array: calls that may overlap in time on the same GPU
 * (other handles or streams) race and must be serialised by the caller.  The
 * array keeps the last call's contents; nothing in it has to start at zero.
 * Without the handle's tag buffer (which this call does not allocate), a
 * single-launch solve here orders fixed-T squarings by per-workgroup words
 * of the row and column panels, and early exit by device-wide barriers.
 * Results are bit-identical to btas_apsp_squaring's. */
btas_status_t btas_apsp_squaring_noalloc(btas_handle_t h, btas_dtype_t dt, int n,
                                         const void *W, int ldw, void *D, int ldd,
                                         unsigned flags, int *steps_out);

/* Number of squarings T for n vertices (0 for n <= 2). */
int btas_apsp_num_steps(int n);

/* 1 if the last btas_apsp_squaring / _noalloc call on this handle that read
 * its step count (steps_out not NULL) ran the single-launch solve on packed
 * 16-bit distances (Sec. I semirings evaluated two lanes per 32-bit
 * register), else 0.  With BTAS_U16=1 in the environment that mode is taken
 * on the device, for int32 graphs of 64 < n <= 500 solved by the single
 * launch, when every finite off-diagonal weight lies in
 * [0, floor(65534 / (2 (n - 1)))] and no diagonal weight is negative: every
 * distance then fits 15 bits and every sum of two fits 16, so the result has
 * the same bits as the int32 squarings.  It is off by default: at n=256 it
 * measured slower than the int32 squarings (the solve is bound by load and
 * synchronisation latency, not by bytes or instructions; the packed mode
 * keeps a device-wide barrier after its gate and between squarings). */
int btas_apsp_last_packed16(btas_handle_t h);

/* ---------------------------------------------------------------------------
 * Batched APSP: `count` independent solves of btas_apsp_squaring (fixed
 * T(n_i) squarings each, same bits as one call per graph), executed as ONE
 * hipGraph launch on the handle's stream.  The paper names host-device
 * transfer and latency as what limits matrix-product formulations (Sec. V);
 * this entry point keeps all graphs resident and issues no host round trip
 * between squarings.
 *   n, W, ldw, D, ldd: HOST arrays of length count; W[i] and D[i] are device
 *   pointers to n[i] x n[i] row-major matrices with leading dimensions
 *   ldw[i], ldd[i] >= max(1, n[i]).  Every W[i] is read before any D[j] is
 *   written, so D[i] may equal W[i]; two outputs must not overlap
 *   (BTAS_ERR_ALIAS).  flags: 0 (every graph runs its T(n_i) squarings) or
 *   BTAS_APSP_EARLY_EXIT: each squaring records per graph whether it changed
 *   D, and the next squaring's tiles of a graph that did not change return at
 *   once (the fixpoint then sits in both of its buffers).  Decided on the
 *   device inside the captured graph, no host round trip; the results are
 *   identical to flags = 0.  Any other flag: BTAS_ERR_UNSUPPORTED.
 * The first call with a given argument set builds a plan (device workspace of
 * two padded n_i x n_i buffers per graph, work lists, per-size-bucket tile
 * shapes chosen by timing every candidate shape of btas_tile_shape_t on this
 * device, the captured graph) and synchronises; later calls with identical
 * arguments only launch the graph (asynchronous).  The environment variable
 * BTAS_BATCHED_TILE=128, 64, mixed, w64, wmix or w64d forces one tile shape;
 * BTAS_AUTOTUNE=0 uses a cost model instead of timing.  A batch of one or two
 * graphs of n <= 352, whose earlier outputs do not overlap later inputs, is
 * solved instead by one btas_apsp_squaring single launch per graph (faster
 * at that size, same bits; no plan, unless BTAS_SINGLE_LAUNCH=0).
 */
btas_status_t btas_apsp_squaring_batched(btas_handle_t h, btas_dtype_t dt, int count,
                                         const int *n, const void *const *W, const int *ldw,
                                         void *const *D, const int *ldd, unsigned flags);

/* All-pairs shortest paths by blocked Floyd-Warshall: the relaxations of the
 * paper's sequential algorithm (Sec. IV, Algorithm 2), d(x,y) <- d(x,y) (+)
 * d(x,z) (.) d(z,y) for every pivot z, grouped into pivot blocks of 64
 * vertices (diagonal block, then its block-row and block-column, then every
 * other block as a tropical product with k = 64).  Consecutive pivot blocks
 * are fused in pairs (in fours for fp32 with n a multiple of 128 and
 * n >= 8192) into one k = 128 (k = 256) product over the blocks outside
 * their own rows and columns, with strip updates that keep the values of
 * the unfused order exactly.  O(n^3) work instead of
 * the O(n^3 log n) of repeated squaring.  D (leading dimension ldd) receives
 * the result of I (+) W (the same reading of the diagonal as
 * btas_apsp_squaring); W == D (same ld) runs in place, any other overlap is
 * BTAS_ERR_ALIAS.  No workspace.  int32 results are the exact distances (equal
 * to btas_apsp_squaring's); binary32 results are those of this relaxation
 * order and block size (one rounding per relaxation), within the rounding
 * bound of the exact distances, and may differ from squaring's in the last
 * bits.  Graphs must have no negative cycle (checked with flags =
 * BTAS_APSP_CHECK_NEG_CYCLE, which synchronises); flags may be 0 or that.
 * Asynchronous otherwise. */
btas_status_t btas_apsp_floyd_warshall(btas_handle_t h, btas_dtype_t dt, int n, const void *W,
                                       int ldw, void *D, int ldd, unsigned flags);

/* Blocked Floyd-Warshall (btas_apsp_floyd_warshall, pivot blocks of 64) of
 * `count` independent graphs in one captured hipGraph: D[i] <- the result for
 * I (+) W[i] (n[i] x n[i], row-major, leading dimensions ldw[i], ldd[i];
 * device pointers in host arrays).  Pivot blocks go in pairs (the pair
 * schedule of btas_apsp_floyd_warshall, which gives the same values as its
 * groups of four); each step of the pair schedule (phases 1 and 2
 * of a block, a strip update, the k=128 update of a pair) is one launch
 * over all graphs that have it, so the graph holds at most
 * 1 + 8 * ceil(max_i ceil(n_i / 64) / 2) launches.  int32 results are the exact
 * distances, bit-identical to btas_apsp_squaring and
 * btas_apsp_squaring_batched; binary32 results equal btas_apsp_floyd_warshall
 * graph by graph.  D[i] may be W[i] with ldd[i] == ldw[i] (in place); any
 * other overlap of an output with any input or output is BTAS_ERR_ALIAS.
 * flags must be 0.  Graphs must have no negative cycle (not checked; the
 * result is unspecified otherwise).  The first call with an argument set
 * builds and captures the plan (synchronises); identical later calls only
 * launch it (asynchronous).  The handle keeps one such plan. */
btas_status_t btas_apsp_floyd_warshall_batched(btas_handle_t h, btas_dtype_t dt, int count,
                                               const int *n, const void *const *W, const int *ldw,
                                               void *const *D, const int *ldd, unsigned flags);

/* Closure (I (+) W)^(2^s) by repeated squaring over either semiring of
 * Sec. I: D_0 = I (+) W (I: 0 on the diagonal, the absent value elsewhere),
 * D_t = D_{t-1} (+) D_{t-1} (.) D_{t-1} for t = 1..T = ceil(log2(n-1)), as in
 * Sec. III.  Min-plus is btas_apsp_squaring (shortest distances; this call
 * forwards to it).  Max-plus gives the heaviest walks of up to n-1 edges; for
 * a graph without positive cycles, such as the precedence DAG of a schedule,
 * these are the longest paths (critical paths: D_ij is the latest start
 * offset of j after i).  W absent entries: BTAS_I32_NEG_INF or -inf for
 * max-plus.  Layout, in-place rule (W == D with ldw == ldd), aliasing and
 * workspace as btas_apsp_squaring.  flags: BTAS_APSP_EARLY_EXIT (stop at the
 * first unchanged step; host round trip per step) and
 * BTAS_APSP_CHECK_NEG_CYCLE, which for max-plus reports a positive cycle (some
 * D_ii > 0, result unspecified) as BTAS_WARN_POS_CYCLE.  int32 finite values
 * along the way must stay within BTAS_I32_FINITE_MAX. */
btas_status_t btas_tropical_closure(btas_handle_t h, btas_semiring_t sr, btas_dtype_t dt, int n,
                                    const void *W, int ldw, void *D, int ldd, unsigned flags,
                                    int *steps_out);

/* Maximum cycle mean of the max-plus matrix A (n x n, row-major, lda; A_vu the
 * weight of edge v -> u, absent BTAS_I32_NEG_INF / -inf): the largest mean
 * weight of a cycle, which is the max-plus eigenvalue of A and the cycle time
 * of the discrete-event system x(k+1) = A (x) x(k) (an application of the
 * max-plus algebra of Sec. I).  Computed by Karp's theorem from the walk
 * table x_0 = 0, x_{k+1} = A (x) x_k (n max-plus gemv launches, the table in
 * the handle's workspace, (n+1) * n * 4 + 24 n bytes):
 *   lambda = max_v min_{k<n, x_k(v) present} (x_n(v) - x_k(v)) / (n - k).
 * int32: *num / *den is lambda exactly, in lowest terms (den > 0), and
 * *lambda its binary64 rounding; den = 0 and lambda = -inf when A has no
 * cycle.  n * max|A_ij| must not exceed BTAS_I32_FINITE_MAX (walk weights
 * stay in the domain), else BTAS_ERR_DOMAIN (checked always).  float32: walk
 * weights are maxima of single binary32 adds and the ratios are evaluated in
 * binary64 as ((double)x_n - (double)x_k) / (n - k); *num = *den = 0.  Output
 * pointers are host pointers, each may be NULL.  Synchronises. */
btas_status_t btas_maxplus_cycle_mean(btas_handle_t h, btas_dtype_t dt, int n, const void *A,
                                      int lda, int64_t *num, int64_t *den, double *lambda);

/* Tropical product with witnesses: C <- C (+) A (.) B as btas_tropical_gemm
 * (the Sec. IV product, whose inner step is a min (max) over k), and K
 * records that step's argument: for every entry whose value strictly
 * improves (smaller for min-plus, larger for max-plus), K[i*ldk+j] <- the
 * smallest p whose term A_ip (.) B_pj equals the new value.  Entries that do
 * not strictly improve keep C and K unchanged, so K needs no initialisation
 * where C is the (+)-identity and callers may chain products over k-slices.
 * Ties between terms are decided on the terms' values as the product
 * computes them (one binary32 add per term; int32 terms exact inside the
 * domain bound, absent values absorbing), so C equals btas_tropical_gemm's
 * result bit for bit and K is unique.  A, B, C row-major as in
 * btas_tropical_gemm; K is an m x n int32 device matrix (leading dimension
 * ldk >= max(1,n)), caller-owned; C or K overlapping any other operand, or
 * each other, is BTAS_ERR_ALIAS.  No workspace, no split-K, asynchronous.
 * k must fit in int32 (it does). */
btas_status_t btas_tropical_gemm_witness(btas_handle_t h, btas_semiring_t sr, btas_dtype_t dt,
                                         int m, int n, int k, const void *A, int lda,
                                         const void *B, int ldb, void *C, int ldc, int32_t *K,
                                         int ldk);

/* Successor (next-hop) matrix of an APSP result, min-plus: S[i*lds+i] = i,
 * and for i != j, S[i*lds+j] = the smallest u != i minimising W_iu (.) D_uj,
 * or -1 when every such term is absent.  It is the witness of the product
 * W' (.) D, W' being W with its diagonal absent (the min over k of the
 * Sec. IV product, taken once on the solved matrix).  With D the shortest
 * distances of W (btas_apsp_squaring, btas_apsp_floyd_warshall) and every
 * edge weight positive, S_ij is the first vertex after i on a shortest path
 * to j and following S from i reaches j; int32 walks have exactly length
 * D_ij.  Zero-weight cycles can make a walk loop.  W, D as in
 * btas_apsp_squaring (n x n, leading dimensions ldw, ldd; W and D may be the
 * same matrix only if the caller wants the successors of D itself); S is an
 * n x n int32 device matrix, leading dimension lds >= max(1,n),
 * caller-owned, and must not overlap W or D (BTAS_ERR_ALIAS).  For n >= 256
 * and W with at most n^2/32 edges off the diagonal (counted first, one host
 * round trip) the argmin runs over each row's edges only, |row i| terms per
 * entry, from a compressed copy of W in the handle's workspace; otherwise
 * one witness product of n^3 terms.  Same S either way.  BTAS_SPARSE_STEPS=0
 * forces the product, =force the edge lists at any n. */
btas_status_t btas_apsp_successors(btas_handle_t h, btas_dtype_t dt, int n, const void *W, int ldw,
                                   const void *D, int ldd, int32_t *S, int lds);

/* Describe the handle's current batched plan: number of kernel launches in
 * its graph and the algorithmic work, sum_i T(n_i) * n_i^3 terms (host
 * outputs, either may be NULL).  INVALID_ARG if no plan exists. */
btas_status_t btas_batched_plan_info(btas_handle_t h, int *num_launches, double *total_terms);

/* How the batched path cuts a graph's n x n output into work items.  The
 * block shapes give each tile a workgroup of four waves, the wave shapes a
 * single wave; one plan uses shapes of one family only. */
typedef enum {
    BTAS_TILES_128 = 0,    /* 128x128 tiles, ragged edge padded to 128 */
    BTAS_TILES_64 = 1,     /* 64x64 tiles (four waves, 4x4 outputs per thread) */
    BTAS_TILES_MIXED = 2,  /* 128x128 on the multiple-of-128 core, 64x64 on the edge */
    BTAS_TILES_W64 = 3,    /* 64x64 tiles, one wave, 8x8 outputs per thread */
    BTAS_TILES_WMIX = 4,   /* one-wave 64x64 on the multiple-of-64 core, 32x32 on the edge */
    BTAS_TILES_W64_DIRECT = 5  /* one-wave 64x64 tiles over the matrix padded to a multiple of
                                  64 with the absent value, operands loaded straight into LDS;
                                  when n mod 64 is 1..32 the last row and column strips use
                                  64x32, 32x64 and 32x32 tiles (work up to n rounded to 32) */
} btas_tile_shape_t;

/* The btas_tile_shape_t the handle's most recent batched plan used for graphs
 * of n vertices of dtype dt, or -1 if that size bucket has not been planned. */
int btas_batched_tile_choice(btas_handle_t h, btas_dtype_t dt, int n);

/* ---------------------------------------------------------------------------
 * Serving: a request loop for APSP solves of mixed sizes.  The paper points to
 * latency and host-device traffic as the limits of matrix-product methods
 * (Sec. V); the server keeps every request's distance matrix on the device
 * from admission to release and overlaps the squarings (Sec. III) of all
 * admitted requests in shared launches.
 *
 * A server owns an engine thread, a stream and a device memory pool of
 * budget_bytes.  Requests are admitted in arrival order while the pool can
 * hold their two padded n x n matrices and edges; admitted requests are
 * densified on the device (D_0 = I (+) W from the COO edge list; duplicate
 * edges keep the lightest) and then advanced one squaring at a time:
 *   BTAS_SERVE_CONTINUOUS: every engine iteration issues ONE grouped launch
 *     holding, for each active request, the next tiles of its current
 *     squaring up to quantum_terms (tile rows x tile cols x n) of work
 *     (<= 0 selects 6e10); requests admitted while others run join the next
 *     iteration (continuous batching).  Two such engines (lanes) run side by
 *     side on their own streams: one for requests of at most 1024 vertices
 *     (the environment variable BTAS_SERVE_SMALL_N changes the bound; 0
 *     keeps one lane) and one for the others, sharing the memory pool, so
 *     small requests do not wait for the large ones' launches.  Admission is
 *     in arrival order within each lane.  BTAS_SERVE_LAUNCH_TERMS (unset: no
 *     cap) caps a large-lane launch at about that many terms, split evenly
 *     over its requests: lower p50 at overload, at some cost in p99 and
 *     throughput;
 *   BTAS_SERVE_FIFO: one request at a time, each squaring one plain GEMM
 *     launch (the one-solve-per-launch baseline).
 * Results are identical in both modes and to btas_apsp_squaring.  Times are
 * seconds on the server's steady clock (btas_server_now).  The server is
 * thread-safe: submit/wait/result/release may be called from any thread.
 */
typedef struct btas_server *btas_server_t;
#define BTAS_SERVE_CONTINUOUS 0
#define BTAS_SERVE_FIFO 1

typedef struct {           /* counts and times are summed over the lanes   */
    long iterations;        /* engine iterations run                        */
    long launches;          /* kernel launches issued for squarings          */
    double busy_seconds;    /* engine time spent with work on the device     */
    size_t pool_bytes, pool_used_bytes, pool_peak_bytes;
    int active, pending;    /* requests on the device / waiting for memory   */
} btas_server_stats_t;

/* dt: element type of every request.  Errors: INVALID_ARG, OOM (pool), DEVICE. */
btas_status_t btas_server_create(btas_server_t *srv, int device, btas_dtype_t dt,
                                 size_t budget_bytes, int mode, double quantum_terms);
/* Stops the engine after its current iteration and frees everything. */
btas_status_t btas_server_destroy(btas_server_t srv);
/* Seconds since the server was created. */
double btas_server_now(btas_server_t srv);
/* Queue one solve.  rows/cols/w: HOST arrays of nnz edges (copied before
 * return; 0 <= rows, cols < n else INVALID_ARG; weights must be legal (.)
 * operands else DOMAIN).  flags: 0 or BTAS_APSP_EARLY_EXIT.  arrival: the
 * request's arrival time on the server clock (latency is measured from it;
 * < 0 means now).  *id receives the request id.  OOM if the request can never
 * fit the pool. */
btas_status_t btas_server_submit(btas_server_t srv, int n, int nnz, const int32_t *rows,
                                 const int32_t *cols, const void *w, unsigned flags,
                                 double arrival, int64_t *id);
/* Wait until request id is done (timeout_s < 0: forever); *done = 1 if so. */
btas_status_t btas_server_wait(btas_server_t srv, int64_t id, double timeout_s, int *done);
/* Device pointer, leading dimension and executed squarings of a finished
 * request's distance matrix; valid until btas_server_release. */
btas_status_t btas_server_result(btas_server_t srv, int64_t id, const void **D_dev, int *ldd,
                                 int *steps);
/* Copy a finished request's n x n distance matrix to the device matrix D
 * (leading dimension ldd >= n); synchronous.  Do not release the request
 * concurrently. */
btas_status_t btas_server_copy_result(btas_server_t srv, int64_t id, void *D, int ldd);
/* Arrival, admission and completion times of a request (-1 if not yet). */
btas_status_t btas_server_times(btas_server_t srv, int64_t id, double *arrival,
                                double *admitted, double *done);
/* Return a finished request's memory to the pool. */
btas_status_t btas_server_release(btas_server_t srv, int64_t id);
btas_status_t btas_server_stats(btas_server_t srv, btas_server_stats_t *out);

#ifdef __cplusplus
}
#endif

#endif /* BTAS_H */
