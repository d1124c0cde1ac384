/*
 * Plain CPU oracle for tropical (min,+)/(max,+) linear algebra and for
 * all-pairs shortest paths by repeated min-plus squaring.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, obviously-correct
 * statement of what the GPU library must compute.  Only the test suite, the
 * smoke check and the CPU-baseline leg of the benchmark may load it.  It
 * shares no header, constant, helper or kernel with the HIP library: its
 * sentinels and domain bounds are declared here, independently.
 *
 * Arithmetic policy (the readings of the paper that this file fixes):
 *  - Semirings (Sec. I, eqs. (1)-(4)): max-plus  x(+)y = max(x,y), x(.)y = x+y;
 *    min-plus  x(+)y = min(x,y), x(.)y = x+y.
 *  - int32: exact integer arithmetic carried in int64.  The absent value is a
 *    sentinel that absorbs under (.): +INF = 0x7FFFFFFF for min-plus,
 *    -INF = -0x7FFFFFFF for max-plus.  Finite operands of (.) must satisfy
 *    |x| <= 2^29-1; anything else is reported as a domain error instead of
 *    being computed.
 *  - float32: every (.) is computed in binary64 and the (+)-reduction is done
 *    on binary64 values; the result is rounded to binary32 once per output.
 *    Because rounding is monotone, min_k RN32(a+b) = RN32(min_k (a+b)), and
 *    because 53 >= 2*24+2, rounding a binary64 sum of two binary32 values to
 *    binary32 equals rounding the exact sum (double rounding is innocuous
 *    for one addition).  So this is the exact definition "one IEEE binary32
 *    add per term, then min/max", evaluated without binary32 arithmetic.
 *  - A matrix that is an input to a later step (the distance matrix of the
 *    squaring loop) is held in binary32 between steps, as the method stores it.
 *
 * Layouts are row-major with leading dimensions; vectors take strides.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

/* ---- this file's own constants (independent of the GPU library) ---- */
#define OR_INF32 ((int32_t)0x7FFFFFFF)       /* min-plus absent value */
#define OR_NINF32 ((int32_t)(-0x7FFFFFFF))   /* max-plus absent value */
#define OR_FINITE_MAX ((1 << 29) - 1)        /* domain bound on (.) operands */
#define OR_INF64 INT64_MAX
#define OR_NINF64 INT64_MIN

#define OR_OK 0
#define OR_EARG 1
#define OR_EDOMAIN 2
#define OR_WNEGCYCLE 3

#define OR_MIN_PLUS 0
#define OR_MAX_PLUS 1

/* ---------------- scalar semiring, int32 (Sec. I eqs. (1)-(4)) -------- */

/* A (.) operand is legal when it is the semiring's absent value or a finite
 * value inside the domain bound.  The other infinity is illegal. */
static int i32_operand_ok(int sr, int32_t x) {
    if (sr == OR_MIN_PLUS && x == OR_INF32) return 1;
    if (sr == OR_MAX_PLUS && x == OR_NINF32) return 1;
    return x >= -OR_FINITE_MAX && x <= OR_FINITE_MAX;
}

/* Lift an int32 element to the int64 carrier (sentinel -> int64 extreme). */
static int64_t i32_lift(int sr, int32_t x) {
    if (sr == OR_MIN_PLUS && x == OR_INF32) return OR_INF64;
    if (sr == OR_MAX_PLUS && x == OR_NINF32) return OR_NINF64;
    return (int64_t)x;
}

/* x (.) y: the absent value absorbs; otherwise the exact sum. */
static int64_t i64_otimes(int sr, int64_t x, int64_t y) {
    if (sr == OR_MIN_PLUS) {
        if (x == OR_INF64 || y == OR_INF64) return OR_INF64;
    } else {
        if (x == OR_NINF64 || y == OR_NINF64) return OR_NINF64;
    }
    return x + y;
}

/* x (+) y: min for min-plus, max for max-plus. */
static int64_t i64_oplus(int sr, int64_t x, int64_t y) {
    if (sr == OR_MIN_PLUS) return x < y ? x : y;
    return x > y ? x : y;
}

/* Back to int32; a finite value that does not fit is a domain error. */
static int i64_store(int sr, int64_t v, int32_t *out) {
    if (sr == OR_MIN_PLUS && v == OR_INF64) { *out = OR_INF32; return OR_OK; }
    if (sr == OR_MAX_PLUS && v == OR_NINF64) { *out = OR_NINF32; return OR_OK; }
    if (v < INT32_MIN || v > INT32_MAX) return OR_EDOMAIN;
    *out = (int32_t)v;
    return OR_OK;
}

/* (+)-identity of the semiring in the int64 carrier. */
static int64_t i64_zero(int sr) { return sr == OR_MIN_PLUS ? OR_INF64 : OR_NINF64; }

/* ---------------- scalar semiring, float32 via binary64 --------------- */

static int f32_operand_ok(int sr, float x) {
    if (isnan(x)) return 0;
    if (sr == OR_MIN_PLUS && isinf(x) && x < 0) return 0;
    if (sr == OR_MAX_PLUS && isinf(x) && x > 0) return 0;
    return 1;
}

static double f64_oplus(int sr, double x, double y) {
    if (sr == OR_MIN_PLUS) return y < x ? y : x;
    return y > x ? y : x;
}

static double f64_zero(int sr) { return sr == OR_MIN_PLUS ? INFINITY : -INFINITY; }

static int sr_ok(int sr) { return sr == OR_MIN_PLUS || sr == OR_MAX_PLUS; }

/* ---------------- domain scans ---------------- */

static int scan_i32(int sr, long rows, long cols, const int32_t *X, long ld) {
    for (long i = 0; i < rows; ++i)
        for (long j = 0; j < cols; ++j)
            if (!i32_operand_ok(sr, X[i * ld + j])) return 0;
    return 1;
}

static int scan_f32(int sr, long rows, long cols, const float *X, long ld) {
    for (long i = 0; i < rows; ++i)
        for (long j = 0; j < cols; ++j)
            if (!f32_operand_ok(sr, X[i * ld + j])) return 0;
    return 1;
}

int or_num_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

void or_set_num_threads(int t) {
#ifdef _OPENMP
    if (t > 0) omp_set_num_threads(t);
#else
    (void)t;
#endif
}

/* ============ Level 3: C <- C (+) A (.) B  (Sec. IV, min-plus product) ===
 * The matrix-product listing of Sec. IV replaces + by min and x by + :
 *     z(i,j) <- min( z(i,j), min_k ( x(i,k) + y(k,j) ) ).
 * Max-plus is the same with max.  A is m x k, B is k x n, C is m x n.
 * C is an accumulator: it is only (+)-combined, never an operand of (.),
 * so any int32 value is accepted there.  Rows are independent, so they are
 * distributed over threads; the order of the k-reduction is the definition's
 * order and cannot change a min/max anyway.
 */
int or_gemm_i32(int sr, long m, long n, long k, const int32_t *A, long lda,
                const int32_t *B, long ldb, int32_t *C, long ldc) {
    if (!sr_ok(sr) || m < 0 || n < 0 || k < 0) return OR_EARG;
    if (!scan_i32(sr, m, k, A, lda) || !scan_i32(sr, k, n, B, ldb)) return OR_EDOMAIN;
    int status = OR_OK;
#pragma omp parallel for schedule(dynamic, 1)
    for (long i = 0; i < m; ++i) {
        for (long j = 0; j < n; ++j) {
            int64_t acc = i64_zero(sr);
            for (long p = 0; p < k; ++p) {
                int64_t term = i64_otimes(sr, i32_lift(sr, A[i * lda + p]),
                                          i32_lift(sr, B[p * ldb + j]));
                acc = i64_oplus(sr, acc, term);
            }
            int64_t c = i32_lift(sr, C[i * ldc + j]);
            int32_t out;
            if (i64_store(sr, i64_oplus(sr, c, acc), &out) != OR_OK) {
#pragma omp atomic write
                status = OR_EDOMAIN;
                continue;
            }
            C[i * ldc + j] = out;
        }
    }
    return status;
}

int or_gemm_f32(int sr, long m, long n, long k, const float *A, long lda,
                const float *B, long ldb, float *C, long ldc) {
    if (!sr_ok(sr) || m < 0 || n < 0 || k < 0) return OR_EARG;
    if (!scan_f32(sr, m, k, A, lda) || !scan_f32(sr, k, n, B, ldb)) return OR_EDOMAIN;
#pragma omp parallel for schedule(dynamic, 1)
    for (long i = 0; i < m; ++i) {
        for (long j = 0; j < n; ++j) {
            double acc = f64_zero(sr);
            for (long p = 0; p < k; ++p) {
                double term = (double)A[i * lda + p] + (double)B[p * ldb + j];
                acc = f64_oplus(sr, acc, term);
            }
            acc = f64_oplus(sr, (double)C[i * ldc + j], acc);
            C[i * ldc + j] = (float)acc;
        }
    }
    return OR_OK;
}

/* ============ Level 2: y <- y (+) A (.) x ============ */
int or_gemv_i32(int sr, long m, long n, const int32_t *A, long lda,
                const int32_t *x, long incx, int32_t *y, long incy) {
    if (!sr_ok(sr) || m < 0 || n < 0 || incx < 1 || incy < 1) return OR_EARG;
    for (long j = 0; j < n; ++j)
        if (!i32_operand_ok(sr, x[j * incx])) return OR_EDOMAIN;
    if (!scan_i32(sr, m, n, A, lda)) return OR_EDOMAIN;
    for (long i = 0; i < m; ++i) {
        int64_t acc = i64_zero(sr);
        for (long j = 0; j < n; ++j)
            acc = i64_oplus(sr, acc, i64_otimes(sr, i32_lift(sr, A[i * lda + j]),
                                                 i32_lift(sr, x[j * incx])));
        int32_t out;
        if (i64_store(sr, i64_oplus(sr, i32_lift(sr, y[i * incy]), acc), &out) != OR_OK)
            return OR_EDOMAIN;
        y[i * incy] = out;
    }
    return OR_OK;
}

int or_gemv_f32(int sr, long m, long n, const float *A, long lda,
                const float *x, long incx, float *y, long incy) {
    if (!sr_ok(sr) || m < 0 || n < 0 || incx < 1 || incy < 1) return OR_EARG;
    if (!scan_f32(sr, m, n, A, lda)) return OR_EDOMAIN;
    for (long j = 0; j < n; ++j)
        if (!f32_operand_ok(sr, x[j * incx])) return OR_EDOMAIN;
    for (long i = 0; i < m; ++i) {
        double acc = f64_zero(sr);
        for (long j = 0; j < n; ++j)
            acc = f64_oplus(sr, acc, (double)A[i * lda + j] + (double)x[j * incx]);
        y[i * incy] = (float)f64_oplus(sr, (double)y[i * incy], acc);
    }
    return OR_OK;
}

/* ============ Level 1 ============
 * z = x (+) y, z = x (.) y, dot = (+)_i x_i (.) y_i (empty: the (+)-identity),
 * y <- y (+) alpha (.) x.
 */
int or_vadd_i32(int sr, long n, const int32_t *x, long incx, const int32_t *y,
                long incy, int32_t *z, long incz) {
    if (!sr_ok(sr) || n < 0 || incx < 1 || incy < 1 || incz < 1) return OR_EARG;
    for (long i = 0; i < n; ++i) {
        int64_t v = i64_oplus(sr, i32_lift(sr, x[i * incx]), i32_lift(sr, y[i * incy]));
        if (i64_store(sr, v, &z[i * incz]) != OR_OK) return OR_EDOMAIN;
    }
    return OR_OK;
}

int or_vadd_f32(int sr, long n, const float *x, long incx, const float *y,
                long incy, float *z, long incz) {
    if (!sr_ok(sr) || n < 0 || incx < 1 || incy < 1 || incz < 1) return OR_EARG;
    for (long i = 0; i < n; ++i)
        z[i * incz] = (float)f64_oplus(sr, (double)x[i * incx], (double)y[i * incy]);
    return OR_OK;
}

int or_vmul_i32(int sr, long n, const int32_t *x, long incx, const int32_t *y,
                long incy, int32_t *z, long incz) {
    if (!sr_ok(sr) || n < 0 || incx < 1 || incy < 1 || incz < 1) return OR_EARG;
    for (long i = 0; i < n; ++i) {
        if (!i32_operand_ok(sr, x[i * incx]) || !i32_operand_ok(sr, y[i * incy]))
            return OR_EDOMAIN;
        int64_t v = i64_otimes(sr, i32_lift(sr, x[i * incx]), i32_lift(sr, y[i * incy]));
        if (i64_store(sr, v, &z[i * incz]) != OR_OK) return OR_EDOMAIN;
    }
    return OR_OK;
}

int or_vmul_f32(int sr, long n, const float *x, long incx, const float *y,
                long incy, float *z, long incz) {
    if (!sr_ok(sr) || n < 0 || incx < 1 || incy < 1 || incz < 1) return OR_EARG;
    for (long i = 0; i < n; ++i) {
        if (!f32_operand_ok(sr, x[i * incx]) || !f32_operand_ok(sr, y[i * incy]))
            return OR_EDOMAIN;
        z[i * incz] = (float)((double)x[i * incx] + (double)y[i * incy]);
    }
    return OR_OK;
}

int or_dot_i32(int sr, long n, const int32_t *x, long incx, const int32_t *y,
               long incy, int32_t *result) {
    if (!sr_ok(sr) || n < 0 || incx < 1 || incy < 1) return OR_EARG;
    int64_t acc = i64_zero(sr);
    for (long i = 0; i < n; ++i) {
        if (!i32_operand_ok(sr, x[i * incx]) || !i32_operand_ok(sr, y[i * incy]))
            return OR_EDOMAIN;
        acc = i64_oplus(sr, acc, i64_otimes(sr, i32_lift(sr, x[i * incx]),
                                            i32_lift(sr, y[i * incy])));
    }
    return i64_store(sr, acc, result);
}

int or_dot_f32(int sr, long n, const float *x, long incx, const float *y,
               long incy, float *result) {
    if (!sr_ok(sr) || n < 0 || incx < 1 || incy < 1) return OR_EARG;
    double acc = f64_zero(sr);
    for (long i = 0; i < n; ++i) {
        if (!f32_operand_ok(sr, x[i * incx]) || !f32_operand_ok(sr, y[i * incy]))
            return OR_EDOMAIN;
        acc = f64_oplus(sr, acc, (double)x[i * incx] + (double)y[i * incy]);
    }
    *result = (float)acc;
    return OR_OK;
}

int or_axpy_i32(int sr, long n, int32_t alpha, const int32_t *x, long incx,
                int32_t *y, long incy) {
    if (!sr_ok(sr) || n < 0 || incx < 1 || incy < 1) return OR_EARG;
    if (!i32_operand_ok(sr, alpha)) return OR_EDOMAIN;
    for (long i = 0; i < n; ++i) {
        if (!i32_operand_ok(sr, x[i * incx])) return OR_EDOMAIN;
        int64_t t = i64_otimes(sr, i32_lift(sr, alpha), i32_lift(sr, x[i * incx]));
        int64_t v = i64_oplus(sr, i32_lift(sr, y[i * incy]), t);
        if (i64_store(sr, v, &y[i * incy]) != OR_OK) return OR_EDOMAIN;
    }
    return OR_OK;
}

int or_axpy_f32(int sr, long n, float alpha, const float *x, long incx,
                float *y, long incy) {
    if (!sr_ok(sr) || n < 0 || incx < 1 || incy < 1) return OR_EARG;
    if (!f32_operand_ok(sr, alpha)) return OR_EDOMAIN;
    for (long i = 0; i < n; ++i) {
        if (!f32_operand_ok(sr, x[i * incx])) return OR_EDOMAIN;
        double t = (double)alpha + (double)x[i * incx];
        y[i * incy] = (float)f64_oplus(sr, (double)y[i * incy], t);
    }
    return OR_OK;
}

/* ============ APSP by repeated min-plus squaring (Sec. III) ============
 * D_0 = I (+) W, where I is the tropical identity (0 on the diagonal, +INF
 * elsewhere); then D_t = D_{t-1} (+) D_{t-1} (.) D_{t-1}, each step reading
 * only the previous step's matrix.  After T = ceil(log2(n-1)) steps (0 when
 * n <= 2) every path of up to n-1 edges has been considered.  With early
 * exit, stop after the first step whose result equals its input bit for bit
 * (that step is counted); every later step would be the identity map.
 */
int or_apsp_steps(long n) {
    if (n <= 2) return 0;
    int t = 0;
    long reach = 1;
    while (reach < n - 1) { reach *= 2; ++t; }
    return t;
}

int or_apsp_i32(long n, const int32_t *W, long ldw, int32_t *D, long ldd,
                int early_exit, int check_neg_cycle, int *steps_out) {
    if (n < 0 || (n > 0 && (ldw < n || ldd < n))) return OR_EARG;
    if (steps_out) *steps_out = 0;
    if (n == 0) return OR_OK;
    int32_t *cur = (int32_t *)malloc(sizeof(int32_t) * n * n);
    int32_t *nxt = (int32_t *)malloc(sizeof(int32_t) * n * n);
    if (!cur || !nxt) { free(cur); free(nxt); return OR_EARG; }
    for (long i = 0; i < n; ++i)
        for (long j = 0; j < n; ++j) cur[i * n + j] = W[i * ldw + j];
    for (long i = 0; i < n; ++i)               /* I (+) W */
        if (cur[i * n + i] > 0) cur[i * n + i] = 0;
    int T = or_apsp_steps(n), steps = 0, status = OR_OK;
    for (int t = 0; t < T; ++t) {
        memcpy(nxt, cur, sizeof(int32_t) * n * n);            /* C = D */
        status = or_gemm_i32(OR_MIN_PLUS, n, n, n, cur, n, cur, n, nxt, n);
        if (status != OR_OK) break;
        ++steps;
        int same = memcmp(nxt, cur, sizeof(int32_t) * n * n) == 0;
        int32_t *tmp = cur; cur = nxt; nxt = tmp;
        if (early_exit && same) break;
    }
    if (status == OR_OK) {
        for (long i = 0; i < n; ++i)
            for (long j = 0; j < n; ++j) D[i * ldd + j] = cur[i * n + j];
        if (check_neg_cycle)
            for (long i = 0; i < n; ++i)
                if (cur[i * n + i] < 0) { status = OR_WNEGCYCLE; break; }
    }
    if (steps_out) *steps_out = steps;
    free(cur); free(nxt);
    return status;
}

int or_apsp_f32(long n, const float *W, long ldw, float *D, long ldd,
                int early_exit, int check_neg_cycle, int *steps_out) {
    if (n < 0 || (n > 0 && (ldw < n || ldd < n))) return OR_EARG;
    if (steps_out) *steps_out = 0;
    if (n == 0) return OR_OK;
    float *cur = (float *)malloc(sizeof(float) * n * n);
    float *nxt = (float *)malloc(sizeof(float) * n * n);
    if (!cur || !nxt) { free(cur); free(nxt); return OR_EARG; }
    for (long i = 0; i < n; ++i)
        for (long j = 0; j < n; ++j) cur[i * n + j] = W[i * ldw + j];
    for (long i = 0; i < n; ++i)
        if (cur[i * n + i] > 0.0f) cur[i * n + i] = 0.0f;
    int T = or_apsp_steps(n), steps = 0, status = OR_OK;
    for (int t = 0; t < T; ++t) {
        memcpy(nxt, cur, sizeof(float) * n * n);
        status = or_gemm_f32(OR_MIN_PLUS, n, n, n, cur, n, cur, n, nxt, n);
        if (status != OR_OK) break;
        ++steps;
        int same = memcmp(nxt, cur, sizeof(float) * n * n) == 0;
        float *tmp = cur; cur = nxt; nxt = tmp;
        if (early_exit && same) break;
    }
    if (status == OR_OK) {
        for (long i = 0; i < n; ++i)
            for (long j = 0; j < n; ++j) D[i * ldd + j] = cur[i * n + j];
        if (check_neg_cycle)
            for (long i = 0; i < n; ++i)
                if (cur[i * n + i] < 0.0f) { status = OR_WNEGCYCLE; break; }
    }
    if (steps_out) *steps_out = steps;
    free(cur); free(nxt);
    return status;
}

/* ============ Sequential Floyd-Warshall (Sec. IV, Algorithm 2) ==========
 * The paper's CPU method: for every pivot z, relax every pair (x,y) through
 * z.  The paper marks absent edges with 0 and skips x == y; here absent is
 * +INF and the diagonal starts at min(W_ii, 0), which is the same relaxation
 * without the ambiguity of a zero-weight edge.  Single-threaded, as in the
 * paper's CPU measurement.  The double version is for fp32-valued inputs
 * (exact when every path sum is an integer below 2^24).
 */
int or_fw_i32(long n, const int32_t *W, long ldw, int32_t *D, long ldd) {
    if (n < 0 || (n > 0 && (ldw < n || ldd < n))) return OR_EARG;
    if (!scan_i32(OR_MIN_PLUS, n, n, W, ldw)) return OR_EDOMAIN;
    int64_t *d = (int64_t *)malloc(sizeof(int64_t) * (n > 0 ? n * n : 1));
    if (!d) return OR_EARG;
    for (long i = 0; i < n; ++i)
        for (long j = 0; j < n; ++j) d[i * n + j] = i32_lift(OR_MIN_PLUS, W[i * ldw + j]);
    for (long i = 0; i < n; ++i)
        if (d[i * n + i] > 0) d[i * n + i] = 0;
    for (long z = 0; z < n; ++z)
        for (long x = 0; x < n; ++x) {
            if (d[x * n + z] == OR_INF64) continue;
            for (long y = 0; y < n; ++y) {
                if (d[z * n + y] == OR_INF64) continue;
                int64_t s = d[x * n + z] + d[z * n + y];
                if (s < d[x * n + y]) d[x * n + y] = s;
            }
        }
    int status = OR_OK;
    for (long i = 0; i < n && status == OR_OK; ++i)
        for (long j = 0; j < n; ++j)
            if (i64_store(OR_MIN_PLUS, d[i * n + j], &D[i * ldd + j]) != OR_OK) {
                status = OR_EDOMAIN;
                break;
            }
    free(d);
    return status;
}

int or_fw_f64(long n, const double *W, long ldw, double *D, long ldd) {
    if (n < 0 || (n > 0 && (ldw < n || ldd < n))) return OR_EARG;
    for (long i = 0; i < n; ++i)
        for (long j = 0; j < n; ++j) D[i * ldd + j] = W[i * ldw + j];
    for (long i = 0; i < n; ++i)
        if (D[i * ldd + i] > 0.0) D[i * ldd + i] = 0.0;
    for (long z = 0; z < n; ++z)
        for (long x = 0; x < n; ++x) {
            double dxz = D[x * ldd + z];
            if (isinf(dxz)) continue;
            for (long y = 0; y < n; ++y) {
                double s = dxz + D[z * ldd + y];
                if (s < D[x * ldd + y]) D[x * ldd + y] = s;
            }
        }
    return OR_OK;
}

/* ============ Blocked (three-phase) Floyd-Warshall ======================
 * The same relaxations as Algorithm 2 -- d(x,y) <- d(x,y) (+) d(x,z) (.) d(z,y)
 * for every pivot z -- grouped by pivot blocks of B consecutive vertices, the
 * order a tiled GPU implementation follows.  For pivot block K:
 *   1. the diagonal block (K,K), pivots of K in ascending order;
 *   2. every other block of block-row K and of block-column K, pivots of K in
 *      ascending order, reading the finished diagonal block;
 *   3. every block (I,J) with I != K and J != K:
 *        d(x,y) <- d(x,y) (+) (+)_{z in K} d(x,z) (.) d(z,y),
 *      reading blocks (I,K) and (K,J), which this phase does not change.
 * In exact arithmetic every order gives the shortest distances.  In binary32
 * the operands of a relaxation depend on the order, so the result is defined
 * by this order and by B (B >= n is sequential Floyd-Warshall; B = 1 as well).
 * int32: exact integers carried in int64, absent = +INF absorbing.  fp32: each
 * relaxation rounds the sum of two binary32 values to binary32 (computed in
 * binary64 and rounded once, which is the same number) and keeps the smaller.
 */
static void fwb_relax_i64(int64_t *d, long n, long x, long y, long z) {
    int64_t a = d[x * n + z], b = d[z * n + y];
    if (a == OR_INF64 || b == OR_INF64) return;
    if (a + b < d[x * n + y]) d[x * n + y] = a + b;
}

static void fwb_relax_f32(float *d, long n, long x, long y, long z) {
    float s = (float)((double)d[x * n + z] + (double)d[z * n + y]);
    if (s < d[x * n + y]) d[x * n + y] = s;
}

/* Runs the three phases with relax(d, n, x, y, z) over an n x n matrix. */
#define OR_FW_BLOCKED(RELAX)                                                     \
    do {                                                                         \
        long nb = (n + B - 1) / B;                                               \
        for (long K = 0; K < nb; ++K) {                                          \
            long k0 = K * B, k1 = k0 + B < n ? k0 + B : n;                       \
            for (long z = k0; z < k1; ++z) /* phase 1 */                         \
                for (long x = k0; x < k1; ++x)                                   \
                    for (long y = k0; y < k1; ++y) RELAX(d, n, x, y, z);         \
            for (long J = 0; J < nb; ++J) { /* phase 2: block-row K */           \
                if (J == K) continue;                                            \
                long j0 = J * B, j1 = j0 + B < n ? j0 + B : n;                   \
                for (long z = k0; z < k1; ++z)                                   \
                    for (long x = k0; x < k1; ++x)                               \
                        for (long y = j0; y < j1; ++y) RELAX(d, n, x, y, z);     \
            }                                                                    \
            for (long I = 0; I < nb; ++I) { /* phase 2: block-column K */        \
                if (I == K) continue;                                            \
                long i0 = I * B, i1 = i0 + B < n ? i0 + B : n;                   \
                for (long z = k0; z < k1; ++z)                                   \
                    for (long x = i0; x < i1; ++x)                               \
                        for (long y = k0; y < k1; ++y) RELAX(d, n, x, y, z);     \
            }                                                                    \
            for (long I = 0; I < nb; ++I) { /* phase 3 */                        \
                if (I == K) continue;                                            \
                long i0 = I * B, i1 = i0 + B < n ? i0 + B : n;                   \
                for (long J = 0; J < nb; ++J) {                                  \
                    if (J == K) continue;                                        \
                    long j0 = J * B, j1 = j0 + B < n ? j0 + B : n;               \
                    for (long z = k0; z < k1; ++z)                               \
                        for (long x = i0; x < i1; ++x)                           \
                            for (long y = j0; y < j1; ++y) RELAX(d, n, x, y, z); \
                }                                                                \
            }                                                                    \
        }                                                                        \
    } while (0)

int or_fw_blocked_i32(long n, const int32_t *W, long ldw, int32_t *D, long ldd, long B) {
    if (n < 0 || B < 1 || (n > 0 && (ldw < n || ldd < n))) return OR_EARG;
    if (!scan_i32(OR_MIN_PLUS, n, n, W, ldw)) return OR_EDOMAIN;
    int64_t *d = (int64_t *)malloc(sizeof(int64_t) * (n > 0 ? n * n : 1));
    if (!d) return OR_EARG;
    for (long i = 0; i < n; ++i)
        for (long j = 0; j < n; ++j) d[i * n + j] = i32_lift(OR_MIN_PLUS, W[i * ldw + j]);
    for (long i = 0; i < n; ++i)
        if (d[i * n + i] > 0) d[i * n + i] = 0;
    OR_FW_BLOCKED(fwb_relax_i64);
    int status = OR_OK;
    for (long i = 0; i < n && status == OR_OK; ++i)
        for (long j = 0; j < n; ++j)
            if (i64_store(OR_MIN_PLUS, d[i * n + j], &D[i * ldd + j]) != OR_OK) {
                status = OR_EDOMAIN;
                break;
            }
    free(d);
    return status;
}

int or_fw_blocked_f32(long n, const float *W, long ldw, float *D, long ldd, long B) {
    if (n < 0 || B < 1 || (n > 0 && (ldw < n || ldd < n))) return OR_EARG;
    if (!scan_f32(OR_MIN_PLUS, n, n, W, ldw)) return OR_EDOMAIN;
    float *d = (float *)malloc(sizeof(float) * (n > 0 ? n * n : 1));
    if (!d) return OR_EARG;
    for (long i = 0; i < n; ++i)
        for (long j = 0; j < n; ++j) d[i * n + j] = W[i * ldw + j];
    for (long i = 0; i < n; ++i)
        if (d[i * n + i] > 0.0f) d[i * n + i] = 0.0f;
    OR_FW_BLOCKED(fwb_relax_f32);
    for (long i = 0; i < n; ++i)
        for (long j = 0; j < n; ++j) D[i * ldd + j] = d[i * n + j];
    free(d);
    return OR_OK;
}

/* ============ Witnesses: which k attains each entry of a product ==========
 * The product listing of Sec. IV takes a min over k; these functions also
 * report the k.  For C <- C (+) A (.) B, an entry whose value strictly
 * improves (smaller for min-plus, larger for max-plus) gets in K the
 * smallest p whose term A_ip (.) B_pj equals the new value; an entry that
 * does not strictly improve keeps both C and K as they were.  Ties between
 * terms are decided on the terms' values in the data's own precision: exact
 * integers for int32 (absent values absorb), one binary32 add for float32
 * (the rounded value, Sec. I arithmetic as read for binary32).
 */
static int better_i64(int sr, int64_t x, int64_t y) { return sr == OR_MIN_PLUS ? x < y : x > y; }
static int better_f32(int sr, float x, float y) { return sr == OR_MIN_PLUS ? x < y : x > y; }

int or_gemm_witness_i32(int sr, long m, long n, long k, const int32_t *A, long lda,
                        const int32_t *B, long ldb, int32_t *C, long ldc, int32_t *K, long ldk) {
    if (!sr_ok(sr) || m < 0 || n < 0 || k < 0 || k > INT32_MAX) return OR_EARG;
    if (!scan_i32(sr, m, k, A, lda) || !scan_i32(sr, k, n, B, ldb)) return OR_EDOMAIN;
    int status = OR_OK;
#pragma omp parallel for schedule(dynamic, 1)
    for (long i = 0; i < m; ++i) {
        for (long j = 0; j < n; ++j) {
            int64_t best = i64_zero(sr);
            long arg = -1;
            for (long p = 0; p < k; ++p) {
                int64_t term = i64_otimes(sr, i32_lift(sr, A[i * lda + p]),
                                          i32_lift(sr, B[p * ldb + j]));
                if (better_i64(sr, term, best)) {
                    best = term;
                    arg = p;
                }
            }
            if (arg < 0 || !better_i64(sr, best, i32_lift(sr, C[i * ldc + j]))) continue;
            int32_t out;
            if (i64_store(sr, best, &out) != OR_OK) {
#pragma omp atomic write
                status = OR_EDOMAIN;
                continue;
            }
            C[i * ldc + j] = out;
            K[i * ldk + j] = (int32_t)arg;
        }
    }
    return status;
}

int or_gemm_witness_f32(int sr, long m, long n, long k, const float *A, long lda,
                        const float *B, long ldb, float *C, long ldc, int32_t *K, long ldk) {
    if (!sr_ok(sr) || m < 0 || n < 0 || k < 0 || k > INT32_MAX) return OR_EARG;
    if (!scan_f32(sr, m, k, A, lda) || !scan_f32(sr, k, n, B, ldb)) return OR_EDOMAIN;
#pragma omp parallel for schedule(dynamic, 1)
    for (long i = 0; i < m; ++i) {
        for (long j = 0; j < n; ++j) {
            float best = (float)f64_zero(sr);
            long arg = -1;
            for (long p = 0; p < k; ++p) {
                /* one binary32 add, evaluated exactly in binary64 and rounded */
                float term = (float)((double)A[i * lda + p] + (double)B[p * ldb + j]);
                if (better_f32(sr, term, best)) {
                    best = term;
                    arg = p;
                }
            }
            if (arg < 0 || !better_f32(sr, best, C[i * ldc + j])) continue;
            C[i * ldc + j] = best;
            K[i * ldk + j] = (int32_t)arg;
        }
    }
    return OR_OK;
}

/* Successor matrix of a distance matrix D (min-plus): S_ii = i, and for
 * i != j, S_ij is the smallest u != i minimising W_iu (.) D_uj (the first
 * hop of a shortest i -> j path when D holds the shortest distances and
 * every weight is positive), or -1 when every such term is absent.  It is
 * the witness of the product W' (.) D with W' = W off the diagonal. */
int or_successors_i32(long n, const int32_t *W, long ldw, const int32_t *D, long ldd,
                      int32_t *S, long lds) {
    if (n < 0 || n > INT32_MAX || (n > 0 && (ldw < n || ldd < n || lds < n))) return OR_EARG;
    if (!scan_i32(OR_MIN_PLUS, n, n, W, ldw) || !scan_i32(OR_MIN_PLUS, n, n, D, ldd))
        return OR_EDOMAIN;
#pragma omp parallel for schedule(dynamic, 1)
    for (long i = 0; i < n; ++i) {
        for (long j = 0; j < n; ++j) {
            int64_t best = OR_INF64;
            long arg = -1;
            for (long u = 0; u < n; ++u) {
                if (u == i) continue;
                int64_t term = i64_otimes(OR_MIN_PLUS, i32_lift(OR_MIN_PLUS, W[i * ldw + u]),
                                          i32_lift(OR_MIN_PLUS, D[u * ldd + j]));
                if (term < best) {
                    best = term;
                    arg = u;
                }
            }
            S[i * lds + j] = (int32_t)(i == j ? i : arg);
        }
    }
    return OR_OK;
}

int or_successors_f32(long n, const float *W, long ldw, const float *D, long ldd,
                      int32_t *S, long lds) {
    if (n < 0 || n > INT32_MAX || (n > 0 && (ldw < n || ldd < n || lds < n))) return OR_EARG;
    if (!scan_f32(OR_MIN_PLUS, n, n, W, ldw) || !scan_f32(OR_MIN_PLUS, n, n, D, ldd))
        return OR_EDOMAIN;
#pragma omp parallel for schedule(dynamic, 1)
    for (long i = 0; i < n; ++i) {
        for (long j = 0; j < n; ++j) {
            float best = INFINITY;
            long arg = -1;
            for (long u = 0; u < n; ++u) {
                if (u == i) continue;
                float term = (float)((double)W[i * ldw + u] + (double)D[u * ldd + j]);
                if (term < best) {
                    best = term;
                    arg = u;
                }
            }
            S[i * lds + j] = (int32_t)(i == j ? i : arg);
        }
    }
    return OR_OK;
}

/* ============ Closure over either semiring (Sec. I semirings, Sec. III) ===
 * (I (+) W)^(2^s) by repeated squaring, as or_apsp_* but for a chosen
 * semiring.  Min-plus gives shortest distances; max-plus gives the heaviest
 * walks of at most 2^s edges, which for a graph without positive cycles (a
 * DAG, as in critical-path scheduling) are the longest paths.  I holds 0 on
 * the diagonal and the absent value elsewhere, so D_ii starts at
 * min(W_ii, 0), resp. max(W_ii, 0).  With check set, a diagonal entry past 0
 * on the improving side (min-plus < 0, max-plus > 0) reports a cycle that
 * makes the closure diverge (OR_WNEGCYCLE).
 */
static int improves_zero_i32(int sr, int32_t x) { return sr == OR_MIN_PLUS ? x < 0 : x > 0; }
static int improves_zero_f32(int sr, float x) { return sr == OR_MIN_PLUS ? x < 0.0f : x > 0.0f; }

int or_closure_i32(int sr, long n, const int32_t *W, long ldw, int32_t *D, long ldd,
                   int early_exit, int check, int *steps_out) {
    if (!sr_ok(sr) || n < 0 || (n > 0 && (ldw < n || ldd < n))) return OR_EARG;
    if (steps_out) *steps_out = 0;
    if (n == 0) return OR_OK;
    int32_t *cur = (int32_t *)malloc(sizeof(int32_t) * n * n);
    int32_t *nxt = (int32_t *)malloc(sizeof(int32_t) * n * n);
    if (!cur || !nxt) { free(cur); free(nxt); return OR_EARG; }
    for (long i = 0; i < n; ++i)
        for (long j = 0; j < n; ++j) {
            int32_t w = W[i * ldw + j];
            if (i == j && improves_zero_i32(sr, 0 - w)) w = 0;   /* (+) with the identity's 0 */
            cur[i * n + j] = w;
        }
    int T = or_apsp_steps(n), steps = 0, status = OR_OK;
    for (int t = 0; t < T; ++t) {
        memcpy(nxt, cur, sizeof(int32_t) * n * n);
        status = or_gemm_i32(sr, n, n, n, cur, n, cur, n, nxt, n);
        if (status != OR_OK) break;
        ++steps;
        int same = memcmp(nxt, cur, sizeof(int32_t) * n * n) == 0;
        int32_t *tmp = cur; cur = nxt; nxt = tmp;
        if (early_exit && same) break;
    }
    if (status == OR_OK) {
        for (long i = 0; i < n; ++i)
            for (long j = 0; j < n; ++j) D[i * ldd + j] = cur[i * n + j];
        if (check)
            for (long i = 0; i < n; ++i)
                if (improves_zero_i32(sr, cur[i * n + i])) { status = OR_WNEGCYCLE; break; }
    }
    if (steps_out) *steps_out = steps;
    free(cur); free(nxt);
    return status;
}

int or_closure_f32(int sr, long n, const float *W, long ldw, float *D, long ldd,
                   int early_exit, int check, int *steps_out) {
    if (!sr_ok(sr) || n < 0 || (n > 0 && (ldw < n || ldd < n))) return OR_EARG;
    if (steps_out) *steps_out = 0;
    if (n == 0) return OR_OK;
    float *cur = (float *)malloc(sizeof(float) * n * n);
    float *nxt = (float *)malloc(sizeof(float) * n * n);
    if (!cur || !nxt) { free(cur); free(nxt); return OR_EARG; }
    for (long i = 0; i < n; ++i)
        for (long j = 0; j < n; ++j) {
            float w = W[i * ldw + j];
            if (i == j && improves_zero_f32(sr, -w)) w = 0.0f;
            cur[i * n + j] = w;
        }
    int T = or_apsp_steps(n), steps = 0, status = OR_OK;
    for (int t = 0; t < T; ++t) {
        memcpy(nxt, cur, sizeof(float) * n * n);
        status = or_gemm_f32(sr, n, n, n, cur, n, cur, n, nxt, n);
        if (status != OR_OK) break;
        ++steps;
        int same = memcmp(nxt, cur, sizeof(float) * n * n) == 0;
        float *tmp = cur; cur = nxt; nxt = tmp;
        if (early_exit && same) break;
    }
    if (status == OR_OK) {
        for (long i = 0; i < n; ++i)
            for (long j = 0; j < n; ++j) D[i * ldd + j] = cur[i * n + j];
        if (check)
            for (long i = 0; i < n; ++i)
                if (improves_zero_f32(sr, cur[i * n + i])) { status = OR_WNEGCYCLE; break; }
    }
    if (steps_out) *steps_out = steps;
    free(cur); free(nxt);
    return status;
}

/* ============ Maximum cycle mean (max-plus eigenvalue), Karp's theorem ====
 * For a max-plus matrix A (A_vu the weight of edge v -> u), the largest mean
 * weight of a cycle is the max-plus eigenvalue of A, the cycle time of the
 * system x(k+1) = A (x) x(k).  With x_0 = 0 (every vertex a start) and
 * x_{k+1} = A (x) x_k (x_k(v) = heaviest walk of exactly k edges from v):
 *     lambda = max over v with x_n(v) present of
 *              min over k < n with x_k(v) present of (x_n(v) - x_k(v)) / (n - k),
 * and no v has x_n(v) present iff the graph has no cycle.  int32: exact
 * integers, lambda returned as the fraction num/den in lowest terms (den = 0:
 * no cycle);
 * the walk weights x_k must stay within the domain bound (n * max|A| <=
 * 2^29 - 1).  float32: every x_{k+1}(v) is a max of single binary32 adds, and
 * lambda is evaluated in binary64 as ((double)x_n - (double)x_k) / (n - k)
 * (-inf: no cycle).
 */
int or_cycle_mean_i32(long n, const int32_t *A, long lda, int64_t *num, int64_t *den) {
    if (n < 0 || (n > 0 && lda < n)) return OR_EARG;
    if (!scan_i32(OR_MAX_PLUS, n, n, A, lda)) return OR_EDOMAIN;
    int64_t *x = (int64_t *)malloc(sizeof(int64_t) * (n + 1) * (n > 0 ? n : 1));
    if (!x) return OR_EARG;
    for (long v = 0; v < n; ++v) x[v] = 0;
    for (long k = 0; k < n; ++k)
        for (long v = 0; v < n; ++v) {
            int64_t best = OR_NINF64;
            for (long u = 0; u < n; ++u)
                best = i64_oplus(OR_MAX_PLUS, best,
                                 i64_otimes(OR_MAX_PLUS, i32_lift(OR_MAX_PLUS, A[v * lda + u]),
                                            x[k * n + u]));
            if (best != OR_NINF64 && (best > OR_FINITE_MAX || best < -OR_FINITE_MAX)) {
                free(x);
                return OR_EDOMAIN;
            }
            x[(k + 1) * n + v] = best;
        }
    int64_t bn = 0, bd = 0;  /* best lambda so far; bd = 0: none */
    for (long v = 0; v < n; ++v) {
        const int64_t xn = x[n * n + v];
        if (xn == OR_NINF64) continue;
        int64_t mn = 0, md = 0;  /* min over k */
        for (long k = 0; k < n; ++k) {
            const int64_t xk = x[k * n + v];
            if (xk == OR_NINF64) continue;
            const int64_t p = xn - xk, q = n - k;
            if (md == 0 || p * md < mn * q) { mn = p; md = q; }
        }
        if (md != 0 && (bd == 0 || mn * bd > bn * md)) { bn = mn; bd = md; }
    }
    if (bd != 0) {  /* lowest terms, so that the fraction is unique */
        int64_t a = bn < 0 ? -bn : bn, b = bd;
        while (b != 0) { const int64_t r = a % b; a = b; b = r; }
        if (a > 1) { bn /= a; bd /= a; }
    }
    *num = bn;
    *den = bd;
    free(x);
    return OR_OK;
}

int or_cycle_mean_f32(long n, const float *A, long lda, double *lambda) {
    if (n < 0 || (n > 0 && lda < n)) return OR_EARG;
    if (!scan_f32(OR_MAX_PLUS, n, n, A, lda)) return OR_EDOMAIN;
    float *x = (float *)malloc(sizeof(float) * (n + 1) * (n > 0 ? n : 1));
    if (!x) return OR_EARG;
    for (long v = 0; v < n; ++v) x[v] = 0.0f;
    for (long k = 0; k < n; ++k)
        for (long v = 0; v < n; ++v) {
            double best = -INFINITY;
            for (long u = 0; u < n; ++u) {
                double term = (double)A[v * lda + u] + (double)x[k * n + u];
                if (term > best) best = term;
            }
            x[(k + 1) * n + v] = (float)best;
        }
    double best = -INFINITY;
    for (long v = 0; v < n; ++v) {
        const float xn = x[n * n + v];
        if (xn == -INFINITY) continue;
        double mn = INFINITY;
        for (long k = 0; k < n; ++k) {
            const float xk = x[k * n + v];
            if (xk == -INFINITY) continue;
            const double r = ((double)xn - (double)xk) / (double)(n - k);
            if (r < mn) mn = r;
        }
        if (mn > best) best = mn;
    }
    *lambda = best;
    free(x);
    return OR_OK;
}
