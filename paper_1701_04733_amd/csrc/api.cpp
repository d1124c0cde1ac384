// C ABI of libbtas: handles, argument validation and dispatch to the HIP
// kernels.  See include/btas.h for the contract of every entry point.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <string>

#include "btas.h"
#include "context.h"
#include "kernels.h"

using namespace btas;

namespace {

const char* kVersion = "btas-gfx950 0.1.0";

// The no-allocation APSP entry point's workspace: one copy of this array per
// GPU, held until the process ends.  In host code its name is only a
// stand-in; kernels get the device address that btas_create looks up once
// per device (kept in scratch_addr).
__device__ __align__(256) unsigned char scratch[btas::NOALLOC_SCRATCH_BYTES];
constexpr int kMaxDevices = 64;
std::mutex scratch_mu;
void* scratch_addr[kMaxDevices];

// Device address of this device's copy of `scratch` (the device is
// current); nullptr if the runtime cannot name it.
void* scratch_for(int device) {
    if (device < 0 || device >= kMaxDevices) return nullptr;
    std::lock_guard<std::mutex> lk(scratch_mu);
    if (!scratch_addr[device]) {
        void* p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) == hipSuccess) scratch_addr[device] = p;
        else (void)hipGetLastError();
    }
    return scratch_addr[device];
}

bool sr_ok(btas_semiring_t sr) { return sr == BTAS_MIN_PLUS || sr == BTAS_MAX_PLUS; }
bool dt_ok(btas_dtype_t dt) { return dt == BTAS_INT32 || dt == BTAS_FLOAT32; }

btas_status_t check_common(btas_handle_t h, const char* fn, btas_semiring_t sr,
                           btas_dtype_t dt) {
    if (!h) return BTAS_ERR_INVALID_ARG;
    if (btas_status_t l = begin_call(h, fn); l != BTAS_OK) return l;
    if (!sr_ok(sr)) return fail(h, BTAS_ERR_INVALID_ARG, "%s: argument 2 (semiring=%d) unknown", fn, (int)sr);
    if (!dt_ok(dt)) return fail(h, BTAS_ERR_INVALID_ARG, "%s: argument 3 (dtype=%d) unknown", fn, (int)dt);
    return BTAS_OK;
}

btas_status_t sync_flags(btas_handle_t h, const char* fn, int count) {
    hipError_t e = hipMemcpyAsync(h->hflags, h->dflags, sizeof(int) * count,
                                  hipMemcpyDeviceToHost, h->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
    if (e != hipSuccess) return device_fail(h, fn, e);
    return BTAS_OK;
}

// BTAS_VALIDATE=1: scan operands of (.) for out-of-domain values.
btas_status_t validate_operands(btas_handle_t h, const char* fn, int sr, int dt,
                                const void* const* ptrs, const long* rows, const long* cols,
                                const long* lds, int count) {
    if (!h->validate) return BTAS_OK;
    int* flag = h->dflags + FLAG_CHECK;
    hipError_t e = btas::launch_clear_flags(flag, 1, h->stream);
    for (int i = 0; i < count && e == hipSuccess; ++i)
        e = btas::launch_domain_scan(sr, dt, (int)rows[i], (int)cols[i], ptrs[i], lds[i], flag,
                                     h->stream);
    if (e != hipSuccess) return device_fail(h, fn, e);
    btas_status_t st = sync_flags(h, fn, FLAG_CHECK + 1);
    if (st != BTAS_OK) return st;
    if (h->hflags[FLAG_CHECK]) return fail(h, BTAS_ERR_DOMAIN, "%s: an input element is outside the semiring's domain", fn);
    return BTAS_OK;
}

// The fixed-T squaring sequence (no host synchronisation): flag resets, D_0 =
// I (+) W, T squarings ping-ponging between D and the workspace so that the
// last one lands in D.
hipError_t enqueue_fixed_apsp(btas_handle_t h, btas_dtype_t dt, int n, const void* W, int ldw,
                              void* D, int ldd, int T, void* ws, void* skws, size_t skws_bytes,
                              hipStream_t s) {
    void* bufs[2] = {D, ws};
    long lds[2] = {ldd, n};
    int cur = (T % 2 == 0) ? 0 : 1;
    // int32: slot FLAG_STEP_WIDE + t records whether D_t left the binary32-exact
    // range; the init kernel fills slot 0 and step t reads slot t-1, writes slot t.
    int* wide = dt == BTAS_INT32 ? h->dflags + FLAG_STEP_WIDE : nullptr;
    hipError_t e = hipSuccess;
    if (wide) e = btas::launch_clear_flags(wide, T + 1, s);
    if (e == hipSuccess) e = btas::launch_apsp_init(dt, n, W, ldw, bufs[cur], lds[cur], wide, s);
    for (int t = 0; t < T && e == hipSuccess; ++t) {
        const int nxt = cur ^ 1;
        btas::GemmArgs a{n, n, n, bufs[cur], lds[cur], bufs[cur], lds[cur], bufs[cur], lds[cur],
                         bufs[nxt], lds[nxt], nullptr,
                         wide ? wide + t : nullptr, wide ? wide + t + 1 : nullptr,
                         skws, skws_bytes};
        e = btas::launch_gemm(BTAS_MIN_PLUS, dt, a, -1, s);
        cur = nxt;
    }
    return e;
}

// Sparse-aware squarings (early-exit path): while D is sparse enough, a
// squaring runs as a row-by-row sparse product with the same bits.
// Costs in units of one dense term (the product runs ~3.9e13 terms/s): a
// sparse term (a gathered load and an LDS atomic min) measured ~200; reading
// D and writing E once costs ~80 per matrix entry at the rates measured.
constexpr int SPARSE_MAX_N = 16384;         // the row accumulator (n entries) fits 64 KiB of LDS
constexpr int SPARSE_AUTO_MIN_N = 4096;     // measured: -5% at 2048, +9% at 4096, +12% at 8192
constexpr long SPARSE_DENSITY_DIV = 8;      // compress only while nnz <= n^2 / 8
constexpr double SPARSE_TERM_COST = 200.0;
constexpr double SPARSE_ENTRY_COST = 80.0;

enum class SparseMode { Off, Auto, Force };

SparseMode sparse_mode(int n) {
    const char* env = getenv("BTAS_SPARSE_STEPS");
    if ((env && env[0] == '0') || n > SPARSE_MAX_N) return SparseMode::Off;
    if (env && strcmp(env, "force") == 0) return SparseMode::Force;
    return n >= SPARSE_AUTO_MIN_N ? SparseMode::Auto : SparseMode::Off;
}

hipError_t ensure_sparse_ws(btas_handle_t h, size_t need) {
    if (h->sp_bytes >= need) return hipSuccess;
    hipError_t e = hipStreamSynchronize(h->stream);
    if (e != hipSuccess) return e;
    if (h->sp_ws) (void)hipFree(h->sp_ws);
    h->sp_ws = nullptr;
    h->sp_bytes = 0;
    e = hipMalloc(&h->sp_ws, need);
    if (e == hipSuccess) h->sp_bytes = need;
    return e;
}

// The handle's matrix workspace (APSP ping-pong partner, cycle-mean table),
// grown on demand.
hipError_t ensure_ws(btas_handle_t h, size_t need) {
    if (h->ws_bytes >= need) return hipSuccess;
    if (h->ws) {
        (void)hipStreamSynchronize(h->stream);
        (void)hipFree(h->ws);
        h->ws = nullptr;
        h->ws_bytes = 0;
    }
    const hipError_t e = hipMalloc(&h->ws, need);
    if (e == hipSuccess) h->ws_bytes = need;
    return e;
}

uint64_t flag_u64(btas_handle_t h, int slot) {
    uint64_t v;
    memcpy(&v, h->hflags + slot, sizeof v);
    return v;
}

// One squaring D -> E as a sparse product if the counts say it pays: 1 if it
// ran, 0 if the caller should run the dense step (D is too dense; later
// squarings are denser still), -1 on error (*st set).  The workspace holds
// the largest CSR the density limit admits, allocated on first use.
int sparse_step(btas_handle_t h, const char* fn, int dt, int n, const void* D, long ld, void* E,
                long lde, int* changed, int* wide_out, SparseMode mode, btas_status_t* st) {
    const size_t head = ((size_t)(2 * n + 2) * 4 + 255) & ~(size_t)255;  // rownnz | rowptr
    const size_t cap = (size_t)n * n / SPARSE_DENSITY_DIV;               // CSR entries
    hipError_t e = ensure_sparse_ws(h, head + cap * 8 + 16);
    if (e == hipErrorOutOfMemory) {  // no room for the CSR: the dense step needs none
        (void)hipGetLastError();
        return 0;
    }
    unsigned long long* counters = reinterpret_cast<unsigned long long*>(h->dflags + FLAG_SPARSE);
    int* rownnz = reinterpret_cast<int*>(h->sp_ws);
    int* rowptr = rownnz + n;
    int* cols = reinterpret_cast<int*>(static_cast<char*>(h->sp_ws) + head);
    void* vals = cols + cap;
    if (e == hipSuccess) e = btas::launch_clear_flags(h->dflags + FLAG_SPARSE, 4, h->stream);
    if (e == hipSuccess) e = btas::launch_sparse_count(dt, n, D, ld, rownnz, counters, h->stream);
    if (e != hipSuccess) {
        *st = device_fail(h, fn, e);
        return -1;
    }
    if ((*st = sync_flags(h, fn, FLAG_SPARSE + 4)) != BTAS_OK) return -1;
    if (flag_u64(h, FLAG_SPARSE) > cap) return 0;
    e = btas::launch_sparse_build(dt, n, D, ld, rownnz, rowptr, cols, vals, counters, h->stream);
    if (e != hipSuccess) {
        *st = device_fail(h, fn, e);
        return -1;
    }
    if ((*st = sync_flags(h, fn, FLAG_SPARSE + 4)) != BTAS_OK) return -1;
    const double terms = (double)flag_u64(h, FLAG_SPARSE + 2);
    const double nn = (double)n * n;
    if (mode == SparseMode::Auto && terms * SPARSE_TERM_COST + nn * SPARSE_ENTRY_COST > nn * n)
        return 0;
    e = btas::launch_sparse_square(dt, n, D, ld, E, lde, rowptr, cols, vals, changed, wide_out,
                                   h->stream);
    if (e != hipSuccess) {
        *st = device_fail(h, fn, e);
        return -1;
    }
    return 1;
}

// Successors from W's edge lists when W is sparse: |row i| terms per entry
// instead of n (the dense witness product's).  1 if done, 0 if W is too
// dense (or no workspace), -1 on error (*st set).
constexpr long SUCC_SPARSE_DIV = 32;  // sparse while W has <= n^2/32 edges

int sparse_successors(btas_handle_t h, const char* fn, int dt, int n, const void* W, long ldw,
                      const void* D, long ldd, int32_t* S, long lds, btas_status_t* st) {
    const size_t head = ((size_t)(2 * n + 2) * 4 + 255) & ~(size_t)255;
    const size_t cap = std::max<size_t>(1, (size_t)n * n / SUCC_SPARSE_DIV);
    hipError_t e = ensure_sparse_ws(h, head + cap * 8 + 16);
    if (e == hipErrorOutOfMemory) {
        (void)hipGetLastError();
        return 0;
    }
    unsigned long long* counters = reinterpret_cast<unsigned long long*>(h->dflags + FLAG_SPARSE);
    int* rownnz = reinterpret_cast<int*>(h->sp_ws);
    int* rowptr = rownnz + n;
    int* cols = reinterpret_cast<int*>(static_cast<char*>(h->sp_ws) + head);
    void* vals = cols + cap;
    if (e == hipSuccess) e = btas::launch_clear_flags(h->dflags + FLAG_SPARSE, 4, h->stream);
    if (e == hipSuccess) e = btas::launch_sparse_count(dt, n, W, ldw, rownnz, counters, h->stream, true);
    if (e != hipSuccess) {
        *st = device_fail(h, fn, e);
        return -1;
    }
    if ((*st = sync_flags(h, fn, FLAG_SPARSE + 4)) != BTAS_OK) return -1;
    if (flag_u64(h, FLAG_SPARSE) > cap) return 0;
    e = btas::launch_sparse_build(dt, n, W, ldw, rownnz, rowptr, cols, vals, counters, h->stream, true);
    if (e == hipSuccess)
        e = btas::launch_sparse_successors(dt, n, rowptr, cols, vals, D, ldd, S, lds, h->stream);
    if (e != hipSuccess) {
        *st = device_fail(h, fn, e);
        return -1;
    }
    return 1;
}

}  // namespace

extern "C" {

const char* btas_version(void) { return kVersion; }

const char* btas_status_string(btas_status_t s) {
    switch (s) {
        case BTAS_OK: return "BTAS_OK";
        case BTAS_ERR_INVALID_ARG: return "BTAS_ERR_INVALID_ARG";
        case BTAS_ERR_ALIAS: return "BTAS_ERR_ALIAS";
        case BTAS_ERR_DOMAIN: return "BTAS_ERR_DOMAIN";
        case BTAS_ERR_OOM: return "BTAS_ERR_OOM";
        case BTAS_ERR_DEVICE: return "BTAS_ERR_DEVICE";
        case BTAS_ERR_UNSUPPORTED: return "BTAS_ERR_UNSUPPORTED";
        case BTAS_WARN_NEG_CYCLE: return "BTAS_WARN_NEG_CYCLE";
        case BTAS_WARN_POS_CYCLE: return "BTAS_WARN_POS_CYCLE";
    }
    return "BTAS_UNKNOWN_STATUS";
}

const char* btas_last_error(btas_handle_t h) { return h ? h->last_error.c_str() : "null handle"; }

int btas_apsp_num_steps(int n) { return btas::apsp_steps(n); }

int btas_apsp_last_packed16(btas_handle_t h) { return h ? h->last_packed16 : 0; }

btas_status_t btas_create(btas_handle_t* out, int device) {
    if (!out) return BTAS_ERR_INVALID_ARG;
    *out = nullptr;
    int count = 0;
    if (hipGetDeviceCount(&count) != hipSuccess || device < 0 || device >= count)
        return BTAS_ERR_INVALID_ARG;
    DeviceGuard g(device);
    if (!g.ok) return BTAS_ERR_DEVICE;
    btas_ctx* h = new btas_ctx;
    h->device = device;
    const char* v = getenv("BTAS_VALIDATE");
    h->validate = v && v[0] == '1';
    // BTAS_TEST_SPIN_LIMIT bounds each device-wide barrier wait of the
    // single-launch solve (polls); a negative value makes every such wait
    // report a timeout at once, so tests can reach the error path with every
    // kernel still ending normally.
    if (const char* sl = getenv("BTAS_TEST_SPIN_LIMIT")) h->spin_limit = atoi(sl);
    if (hipMalloc(&h->dflags, kNumFlags * sizeof(int)) != hipSuccess ||
        hipHostMalloc((void**)&h->hflags, kNumFlags * sizeof(int), hipHostMallocDefault) != hipSuccess ||
        hipHostMalloc((void**)&h->hlatch, sizeof(int), hipHostMallocCoherent) != hipSuccess ||
        hipMalloc(&h->partials, (size_t)btas::dot_partials_needed(0) * 4) != hipSuccess) {
        if (h->dflags) (void)hipFree(h->dflags);
        if (h->hflags) (void)hipHostFree(h->hflags);
        if (h->hlatch) (void)hipHostFree(h->hlatch);
        if (h->partials) (void)hipFree(h->partials);
        delete h;
        return BTAS_ERR_OOM;
    }
    *h->hlatch = 0;
    h->scratch = scratch_for(device);
    if (hipMemset(h->dflags, 0, kNumFlags * sizeof(int)) != hipSuccess ||
        hipDeviceGetAttribute(&h->num_cus, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess ||
        h->num_cus < 1) {
        (void)hipFree(h->dflags);
        (void)hipHostFree(h->hflags);
        (void)hipHostFree(h->hlatch);
        (void)hipFree(h->partials);
        delete h;
        return BTAS_ERR_DEVICE;
    }
    *out = h;
    return BTAS_OK;
}

btas_status_t btas_destroy(btas_handle_t h) {
    if (!h) return BTAS_ERR_INVALID_ARG;
    DeviceGuard g(h->device);
    (void)hipStreamSynchronize(h->stream);
    h->batch_plan.reset();
    h->fw_batch_plan.reset();
    if (h->apsp_exec) (void)hipGraphExecDestroy(h->apsp_exec);
    if (h->apsp_graph) (void)hipGraphDestroy(h->apsp_graph);
    if (h->aux_stream) (void)hipStreamDestroy(h->aux_stream);
    if (h->fork_stream) (void)hipStreamDestroy(h->fork_stream);
    if (h->fork_event) (void)hipEventDestroy(h->fork_event);
    if (h->join_event) (void)hipEventDestroy(h->join_event);
    if (h->ws) (void)hipFree(h->ws);
    if (h->tagws) (void)hipFree(h->tagws);
    if (h->sp_ws) (void)hipFree(h->sp_ws);
    if (h->skws) (void)hipFree(h->skws);
    if (h->partials) (void)hipFree(h->partials);
    if (h->dflags) (void)hipFree(h->dflags);
    if (h->hflags) (void)hipHostFree(h->hflags);
    if (h->hlatch) (void)hipHostFree(h->hlatch);
    delete h;
    return BTAS_OK;
}

btas_status_t btas_set_stream(btas_handle_t h, void* stream) {
    if (!h) return BTAS_ERR_INVALID_ARG;
    h->stream = (hipStream_t)stream;
    return BTAS_OK;
}

btas_status_t btas_synchronize(btas_handle_t h) {
    if (!h) return BTAS_ERR_INVALID_ARG;
    DeviceGuard g(h->device);
    hipError_t e = hipStreamSynchronize(h->stream);
    if (e != hipSuccess) return device_fail(h, "btas_synchronize", e);
    return begin_call(h, "btas_synchronize");
}

// ------------------------------------------------------------- level 3 ---
btas_status_t btas_tropical_gemm(btas_handle_t h, btas_semiring_t sr, btas_dtype_t dt, int m,
                                 int n, int k, const void* A, int lda, const void* B, int ldb,
                                 void* C, int ldc) {
    const char* fn = "btas_tropical_gemm";
    btas_status_t st = check_common(h, fn, sr, dt);
    if (st != BTAS_OK) return st;
    if (m < 0) return fail(h, BTAS_ERR_INVALID_ARG, "%s: argument 4 (m=%d) < 0", fn, m);
    if (n < 0) return fail(h, BTAS_ERR_INVALID_ARG, "%s: argument 5 (n=%d) < 0", fn, n);
    if (k < 0) return fail(h, BTAS_ERR_INVALID_ARG, "%s: argument 6 (k=%d) < 0", fn, k);
    if (lda < (k > 1 ? k : 1))
        return fail(h, BTAS_ERR_INVALID_ARG, "%s: argument 8 (lda=%d) < max(1,k=%d)", fn, lda, k);
    if (ldb < (n > 1 ? n : 1))
        return fail(h, BTAS_ERR_INVALID_ARG, "%s: argument 10 (ldb=%d) < max(1,n=%d)", fn, ldb, n);
    if (ldc < (n > 1 ? n : 1))
        return fail(h, BTAS_ERR_INVALID_ARG, "%s: argument 12 (ldc=%d) < max(1,n=%d)", fn, ldc, n);
    if ((long)m * k > 0 && !A) return fail(h, BTAS_ERR_INVALID_ARG, "%s: argument 7 (A) is null", fn);
    if ((long)k * n > 0 && !B) return fail(h, BTAS_ERR_INVALID_ARG, "%s: argument 9 (B) is null", fn);
    if ((long)m * n > 0 && !C) return fail(h, BTAS_ERR_INVALID_ARG, "%s: argument 11 (C) is null", fn);
    const Span sc = mat_span(C, m, n, ldc);
    if (overlap(sc, mat_span(A, m, k, lda)) || overlap(sc, mat_span(B, k, n, ldb)))
        return fail(h, BTAS_ERR_ALIAS, "%s: C overlaps A or B", fn);
    if (m == 0 || n == 0 || k == 0) return BTAS_OK;
    DeviceGuard g(h->device);
    const void* ps[2] = {A, B};
    const long rows[2] = {m, k}, cols[2] = {k, n}, lds[2] = {lda, ldb};
    st = validate_operands(h, fn, sr, dt, ps, rows, cols, lds, 2);
    if (st != BTAS_OK) return st;
    int* wide = nullptr;
    hipError_t e = hipSuccess;
    if (dt == BTAS_INT32) {
        // Decide on the device whether the binary32-exact path applies.
        wide = h->dflags + FLAG_GEMM_WIDE;
        e = btas::launch_clear_flags(wide, 1, h->stream);
        if (e == hipSuccess) e = btas::launch_range_scan(sr, m, k, A, lda, wide, h->stream);
        if (e == hipSuccess) e = btas::launch_range_scan(sr, k, n, B, ldb, wide, h->stream);
        if (e != hipSuccess) return device_fail(h, fn, e);
    }
    if (ensure_splitk(h, btas::gemm_splitk_bytes(m, n, k)) != hipSuccess)
        return fail(h, BTAS_ERR_OOM, "%s: cannot allocate the split-K workspace", fn);
    btas::GemmArgs a{m, n, k, A, lda, B, ldb, C, ldc, C, ldc, nullptr, wide, nullptr,
                     h->skws, h->skws_bytes};
    e = btas::launch_gemm(sr, dt, a, -1, h->stream);
    return e == hipSuccess ? BTAS_OK : device_fail(h, fn, e);
}

// ------------------------------------------------------------- level 2 ---
btas_status_t btas_tropical_gemv(btas_handle_t h, btas_semiring_t sr, btas_dtype_t dt, int m,
                                 int n, const void* A, int lda, const void* x, int incx, void* y,
                                 int incy) {
    const char* fn = "btas_tropical_gemv";
    btas_status_t st = check_common(h, fn, sr, dt);
    if (st != BTAS_OK) return st;
    if (m < 0) return fail(h, BTAS_ERR_INVALID_ARG, "%s: argument 4 (m=%d) < 0", fn, m);
    if (n < 0) return fail(h, BTAS_ERR_INVALID_ARG, "%s: argument 5 (n=%d) < 0", fn, n);
    if (lda < (n > 1 ? n : 1))
        return fail(h, BTAS_ERR_INVALID_ARG, "%s: argument 7 (lda=%d) < max(1,n=%d)", fn, lda, n);
    if (incx < 1) return fail(h, BTAS_ERR_INVALID_ARG, "%s: argument 9 (incx=%d) < 1", fn, incx);
    if (incy < 1) return fail(h, BTAS_ERR_INVALID_ARG, "%s: argument 11 (incy=%d) < 1", fn, incy);
    if ((long)m * n > 0 && !A) return fail(h, BTAS_ERR_INVALID_ARG, "%s: argument 6 (A) is null", fn);
    if (n > 0 && m > 0 && !x) return fail(h, BTAS_ERR_INVALID_ARG, "%s: argument 8 (x) is null", fn);
    if (m > 0 && !y) return fail(h, BTAS_ERR_INVALID_ARG, "%s: argument 10 (y) is null", fn);
    const Span sy = vec_span(y, m, incy);
    if (overlap(sy, mat_span(A, m, n, lda)) || overlap(sy, vec_span(x, n, incx)))
        return fail(h, BTAS_ERR_ALIAS, "%s: y overlaps A or x", fn);
    if (m == 0 || n == 0) return BTAS_OK;
    DeviceGuard g(h->device);
    const void* ps[2] = {A, x};
    const long rows[2] = {m, n}, cols[2] = {n, 1}, lds[2] = {lda, incx};
    st = validate_operands(h, fn, sr, dt, ps, rows, cols, lds, 2);
    if (st != BTAS_OK) return st;
    hipError_t e = btas::launch_gemv(sr, dt, m, n, A, lda, x, incx, y, incy, h->stream);
    return e == hipSuccess ? BTAS_OK : device_fail(h, fn, e);
}

// ------------------------------------------------------------- level 1 ---
static btas_status_t vec_binary(btas_handle_t h, const char* fn, int op, btas_semiring_t sr,
                                btas_dtype_t dt, int n, const void* x, int incx, const void* y,
                                int incy, void* z, int incz) {
    btas_status_t st = check_common(h, fn, sr, dt);
    if (st != BTAS_OK) return st;
    if (n < 0) return fail(h, BTAS_ERR_INVALID_ARG, "%s: argument 4 (n=%d) < 0", fn, n);
    if (incx < 1) return fail(h, BTAS_ERR_INVALID_ARG, "%s: argument 6 (incx=%d) < 1", fn, incx);
    if (incy < 1) return fail(h, BTAS_ERR_INVALID_ARG, "%s: argument 8 (incy=%d) < 1", fn, incy);
    if (incz < 1) return fail(h, BTAS_ERR_INVALID_ARG, "%s: argument 10 (incz=%d) < 1", fn, incz);
    if (n > 0 && (!x || !y || !z)) return fail(h, BTAS_ERR_INVALID_ARG, "%s: null vector pointer", fn);
    const Span sz = vec_span(z, n, incz);
    const bool same_x = z == x && incz == incx, same_y = z == y && incz == incy;
    if ((!same_x && overlap(sz, vec_span(x, n, incx))) || (!same_y && overlap(sz, vec_span(y, n, incy))))
        return fail(h, BTAS_ERR_ALIAS, "%s: z partially overlaps x or y", fn);
    if (n == 0) return BTAS_OK;
    DeviceGuard g(h->device);
    if (op == 1) {
        const void* ps[2] = {x, y};
        const long rows[2] = {n, n}, cols[2] = {1, 1}, lds[2] = {incx, incy};
        st = validate_operands(h, fn, sr, dt, ps, rows, cols, lds, 2);
        if (st != BTAS_OK) return st;
    }
    hipError_t e = btas::launch_vec_binary(op, sr, dt, n, x, incx, y, incy, z, incz, h->stream);
    return e == hipSuccess ? BTAS_OK : device_fail(h, fn, e);
}

btas_status_t btas_tropical_vadd(btas_handle_t h, btas_semiring_t sr, btas_dtype_t dt, int n,
                                 const void* x, int incx, const void* y, int incy, void* z,
                                 int incz) {
    return vec_binary(h, "btas_tropical_vadd", 0, sr, dt, n, x, incx, y, incy, z, incz);
}

btas_status_t btas_tropical_vmul(btas_handle_t h, btas_semiring_t sr, btas_dtype_t dt, int n,
                                 const void* x, int incx, const void* y, int incy, void* z,
                                 int incz) {
    return vec_binary(h, "btas_tropical_vmul", 1, sr, dt, n, x, incx, y, incy, z, incz);
}

btas_status_t btas_tropical_dot(btas_handle_t h, btas_semiring_t sr, btas_dtype_t dt, int n,
                                const void* x, int incx, const void* y, int incy,
                                void* result_dev) {
    const char* fn = "btas_tropical_dot";
    btas_status_t st = check_common(h, fn, sr, dt);
    if (st != BTAS_OK) return st;
    if (n < 0) return fail(h, BTAS_ERR_INVALID_ARG, "%s: argument 4 (n=%d) < 0", fn, n);
    if (incx < 1) return fail(h, BTAS_ERR_INVALID_ARG, "%s: argument 6 (incx=%d) < 1", fn, incx);
    if (incy < 1) return fail(h, BTAS_ERR_INVALID_ARG, "%s: argument 8 (incy=%d) < 1", fn, incy);
    if (n > 0 && (!x || !y)) return fail(h, BTAS_ERR_INVALID_ARG, "%s: null vector pointer", fn);
    if (!result_dev) return fail(h, BTAS_ERR_INVALID_ARG, "%s: argument 9 (result) is null", fn);
    DeviceGuard g(h->device);
    const void* ps[2] = {x, y};
    const long rows[2] = {n, n}, cols[2] = {1, 1}, lds[2] = {incx, incy};
    st = validate_operands(h, fn, sr, dt, ps, rows, cols, lds, 2);
    if (st != BTAS_OK) return st;
    hipError_t e = btas::launch_dot(sr, dt, n, x, incx, y, incy, h->partials, result_dev, h->stream);
    return e == hipSuccess ? BTAS_OK : device_fail(h, fn, e);
}

btas_status_t btas_tropical_axpy(btas_handle_t h, btas_semiring_t sr, btas_dtype_t dt, int n,
                                 const void* alpha_host, const void* x, int incx, void* y,
                                 int incy) {
    const char* fn = "btas_tropical_axpy";
    btas_status_t st = check_common(h, fn, sr, dt);
    if (st != BTAS_OK) return st;
    if (n < 0) return fail(h, BTAS_ERR_INVALID_ARG, "%s: argument 4 (n=%d) < 0", fn, n);
    if (!alpha_host) return fail(h, BTAS_ERR_INVALID_ARG, "%s: argument 5 (alpha) is null", fn);
    if (incx < 1) return fail(h, BTAS_ERR_INVALID_ARG, "%s: argument 7 (incx=%d) < 1", fn, incx);
    if (incy < 1) return fail(h, BTAS_ERR_INVALID_ARG, "%s: argument 9 (incy=%d) < 1", fn, incy);
    if (n > 0 && (!x || !y)) return fail(h, BTAS_ERR_INVALID_ARG, "%s: null vector pointer", fn);
    if (overlap(vec_span(y, n, incy), vec_span(x, n, incx)))
        return fail(h, BTAS_ERR_ALIAS, "%s: y overlaps x", fn);
    uint32_t abits;
    std::memcpy(&abits, alpha_host, 4);
    if (h->validate) {
        // host-side check of the scalar operand
        bool ok;
        if (dt == BTAS_FLOAT32) {
            float a;
            std::memcpy(&a, &abits, 4);
            ok = a == a && !(sr == BTAS_MIN_PLUS && a == -__builtin_inff()) &&
                 !(sr == BTAS_MAX_PLUS && a == __builtin_inff());
        } else {
            const int32_t a = (int32_t)abits;
            const int32_t absent = sr == BTAS_MIN_PLUS ? BTAS_I32_INF : BTAS_I32_NEG_INF;
            ok = a == absent || (a >= -BTAS_I32_FINITE_MAX && a <= BTAS_I32_FINITE_MAX);
        }
        if (!ok) return fail(h, BTAS_ERR_DOMAIN, "%s: alpha is outside the semiring's domain", fn);
    }
    if (n == 0) return BTAS_OK;
    DeviceGuard g(h->device);
    const void* ps[1] = {x};
    const long rows[1] = {n}, cols[1] = {1}, lds[1] = {incx};
    st = validate_operands(h, fn, sr, dt, ps, rows, cols, lds, 1);
    if (st != BTAS_OK) return st;
    hipError_t e = btas::launch_axpy(sr, dt, n, abits, x, incx, y, incy, h->stream);
    return e == hipSuccess ? BTAS_OK : device_fail(h, fn, e);
}

// ----------------------------------------------------------------- APSP ---
namespace {

// A caller-provided workspace for the squaring (the no-allocation entry
// point): the ping-pong partner in [base, base + n*n*4), split-K partial
// products in the rest.
struct FixedWs {
    unsigned char* base;
    size_t bytes;
};

btas_status_t apsp_impl(btas_handle_t h, const char* fn, btas_dtype_t dt, int n, const void* W,
                        int ldw, void* D, int ldd, unsigned flags, int* steps_out,
                        const FixedWs* fixed) {
    if (!h) return BTAS_ERR_INVALID_ARG;
    if (btas_status_t l = begin_call(h, fn); l != BTAS_OK) return l;
    if (steps_out) *steps_out = 0;
    h->last_packed16 = 0;
    if (!dt_ok(dt)) return fail(h, BTAS_ERR_INVALID_ARG, "%s: argument 2 (dtype=%d) unknown", fn, (int)dt);
    if (n < 0) return fail(h, BTAS_ERR_INVALID_ARG, "%s: argument 3 (n=%d) < 0", fn, n);
    if (ldw < (n > 1 ? n : 1))
        return fail(h, BTAS_ERR_INVALID_ARG, "%s: argument 5 (ldw=%d) < max(1,n=%d)", fn, ldw, n);
    if (ldd < (n > 1 ? n : 1))
        return fail(h, BTAS_ERR_INVALID_ARG, "%s: argument 7 (ldd=%d) < max(1,n=%d)", fn, ldd, n);
    if (flags & ~(BTAS_APSP_EARLY_EXIT | BTAS_APSP_CHECK_NEG_CYCLE | BTAS_APSP_GRAPH |
                  BTAS_APSP_SINGLE_LAUNCH))
        return fail(h, BTAS_ERR_INVALID_ARG, "%s: argument 8 (flags=0x%x) has unknown bits", fn, flags);
    if ((flags & BTAS_APSP_EARLY_EXIT) && (flags & BTAS_APSP_GRAPH))
        return fail(h, BTAS_ERR_INVALID_ARG, "%s: EARLY_EXIT and GRAPH cannot be combined", fn);
    if ((flags & BTAS_APSP_SINGLE_LAUNCH) && (flags & BTAS_APSP_GRAPH))
        return fail(h, BTAS_ERR_INVALID_ARG, "%s: SINGLE_LAUNCH and GRAPH cannot be combined", fn);
    if (n > 0 && (!W || !D)) return fail(h, BTAS_ERR_INVALID_ARG, "%s: W or D is null", fn);
    if (fixed && (flags & BTAS_APSP_GRAPH))
        return fail(h, BTAS_ERR_INVALID_ARG, "%s: GRAPH needs allocations (graph capture); not "
                    "available here", fn);
    // The handle's (or the fixed) workspace: the n x n partner, and for the
    // single-launch solve of an int32 graph room for its packed 16-bit mode.
    const size_t need = n <= btas::RESIDENT_MAX_N ? btas::resident_ws_bytes(dt, n) : (size_t)n * n * 4;
    if (fixed && (need + 255) / 256 * 256 > fixed->bytes)
        return fail(h, BTAS_ERR_INVALID_ARG,
                    "%s: argument 3 (n=%d) exceeds the fixed workspace (%zu bytes: n <= %d)", fn,
                    n, fixed->bytes, btas::NOALLOC_MAX_N);
    const bool in_place = W == D && ldw == ldd;
    if (!in_place && overlap(mat_span(W, n, n, ldw), mat_span(D, n, n, ldd)))
        return fail(h, BTAS_ERR_ALIAS, "%s: D partially overlaps W", fn);
    if (n == 0) return BTAS_OK;
    DeviceGuard g(h->device);
    {
        const void* ps[1] = {W};
        const long rows[1] = {n}, cols[1] = {n}, lds[1] = {ldw};
        btas_status_t st = validate_operands(h, fn, BTAS_MIN_PLUS, dt, ps, rows, cols, lds, 1);
        if (st != BTAS_OK) return st;
    }
    const int T = btas_apsp_num_steps(n);
    void* ws = nullptr;
    void* skws = nullptr;
    size_t skws_bytes = 0;
    if (fixed) {
        // No allocation: the partner matrix and the split-K partials come from
        // the fixed workspace (a product whose partials do not fit runs
        // without split-K: same bits).
        const size_t part = (need + 255) & ~(size_t)255;  // fits: checked above
        ws = fixed->base;
        skws = fixed->base + part;
        skws_bytes = fixed->bytes - part;
    } else {
        if (T > 0 && ensure_ws(h, need) != hipSuccess)
            return fail(h, BTAS_ERR_OOM, "%s: cannot allocate the %zu-byte workspace", fn, need);
        ws = h->ws;
    }
    // Grow the handle's split-K workspace (not with a fixed workspace).
    auto prepare_splitk = [&]() -> bool {
        if (fixed) return true;
        if (ensure_splitk(h, btas::gemm_splitk_bytes(n, n, n)) != hipSuccess) return false;
        skws = h->skws;
        skws_bytes = h->skws_bytes;
        return true;
    };
    // Graphs of up to AUTO_SINGLE_LAUNCH_N vertices take the single-launch
    // solve also without the flag (it is faster there: one launch instead of
    // one or two per squaring) unless a captured graph was asked for or
    // BTAS_SINGLE_LAUNCH=0.  Above 256 that holds for the tagged mode only,
    // which needs the handle's tag buffer (not used with a fixed workspace).
    const char* sl_env = getenv("BTAS_SINGLE_LAUNCH");
    const int auto_max = fixed ? btas::AUTO_SINGLE_LAUNCH_BARRIER_N : btas::AUTO_SINGLE_LAUNCH_N;
    const bool auto_single = !(sl_env && sl_env[0] == '0') && n >= btas::AUTO_SINGLE_LAUNCH_MIN_N &&
                             n <= auto_max && !(flags & BTAS_APSP_GRAPH);
    bool resident =
        n <= btas::RESIDENT_MAX_N && ((flags & BTAS_APSP_SINGLE_LAUNCH) || auto_single);
    if (T > 0 && !resident && !prepare_splitk())
        return fail(h, BTAS_ERR_OOM, "%s: cannot allocate the split-K workspace", fn);
    const bool early = flags & BTAS_APSP_EARLY_EXIT;
    hipError_t e = hipSuccess;
    int steps = 0;
    if (resident) {
        // One cooperative launch: init, every squaring and (early exit) the
        // stop decision on the device; the host reads the step count only if
        // asked for it.
        // The barrier words carry the launch's epoch: they are cleared only
        // before the first launch and when the count restarts.
        // The tag buffer of the tagged mode (the handle's own, not the
        // caller's fixed workspace) follows the same rule.
        int* rf = h->dflags + FLAG_RESIDENT;
        bool fresh_tags = false;
        if (!fixed && !h->tagws) {
            if (hipMalloc(&h->tagws, btas::resident_tag_bytes()) != hipSuccess) {
                (void)hipGetLastError();
                h->tagws = nullptr;  // solved without the tagged mode
            } else {
                fresh_tags = true;
            }
        }
        if (fresh_tags || h->resident_epoch == 0 || h->resident_epoch >= (1u << 24) - 1) {
            e = btas::launch_clear_flags(rf, FLAG_RESIDENT_END - FLAG_RESIDENT, h->stream);
            if (e == hipSuccess && h->tagws)
                e = btas::launch_zero_words(h->tagws, btas::resident_tag_bytes() / 8, h->stream);
            if (e != hipSuccess) return device_fail(h, fn, e);
            h->resident_epoch = 0;
        }
        const unsigned epoch = ++h->resident_epoch;
        // BTAS_U16=1 lets int32 graphs that pass its gate run the packed
        // 16-bit mode (same bits; measured slower than the int32 squarings
        // at n=256, where panel-load and barrier latency, not bytes or
        // instructions, set the time).
        const char* u16_env = getenv("BTAS_U16");
        e = btas::launch_apsp_resident(dt, n, W, ldw, D, ldd, ws, fixed ? nullptr : h->tagws, T,
                                       early, rf, h->hlatch,
                                       h->num_cus, h->spin_limit, u16_env && u16_env[0] == '1',
                                       epoch, h->stream);
        if (e != hipSuccess && !(flags & BTAS_APSP_SINGLE_LAUNCH)) {
            // Chosen automatically and refused (its workgroups cannot all be
            // resident): one launch per squaring instead.
            (void)hipGetLastError();
            e = hipSuccess;
            resident = false;
            if (T > 0 && !prepare_splitk())
                return fail(h, BTAS_ERR_OOM, "%s: cannot allocate the split-K workspace", fn);
        } else {
            if (e != hipSuccess) return device_fail(h, fn, e);
            steps = T;
            if (steps_out) {
                btas_status_t st = sync_flags(h, fn, FLAG_RESIDENT + 2);
                if (st != BTAS_OK) return st;
                if (h->hflags[FLAG_RESIDENT] == (int)epoch) {  // a wait timed out: D is not valid
                    __atomic_store_n(h->hlatch, 0, __ATOMIC_RELEASE);  // reported here
                    return fail(h, BTAS_ERR_DEVICE, "%s: a wait on other workgroups timed out", fn);
                }
                steps = h->hflags[FLAG_RESIDENT + 1] & (btas::RESIDENT_PACKED16_BIT - 1);
                h->last_packed16 = (h->hflags[FLAG_RESIDENT + 1] & btas::RESIDENT_PACKED16_BIT) != 0;
            }
        }
    }
    if (resident) {
        // solved by the single launch above
    } else if (!early && (flags & BTAS_APSP_GRAPH)) {
        // One hipGraph per argument set: capture once on the auxiliary stream,
        // replay on the handle's stream.
        uint64_t key = 0x9E37ull;
        for (uint64_t v : {(uint64_t)dt, (uint64_t)n, (uint64_t)(uintptr_t)W, (uint64_t)ldw,
                           (uint64_t)(uintptr_t)D, (uint64_t)ldd, (uint64_t)(uintptr_t)ws,
                           (uint64_t)(uintptr_t)skws, (uint64_t)skws_bytes})
            key = (key ^ (v + 0x9E3779B97F4A7C15ull + (key << 6) + (key >> 2)));
        if (!h->apsp_exec || h->apsp_key != key) {
            if (h->apsp_exec) {
                e = hipStreamSynchronize(h->stream);
                (void)hipGraphExecDestroy(h->apsp_exec);
                (void)hipGraphDestroy(h->apsp_graph);
                h->apsp_exec = nullptr;
                h->apsp_graph = nullptr;
                if (e != hipSuccess) return device_fail(h, fn, e);
            }
            if (!h->aux_stream) {
                e = hipStreamCreateWithFlags(&h->aux_stream, hipStreamNonBlocking);
                if (e != hipSuccess) return device_fail(h, fn, e);
            }
            e = hipStreamBeginCapture(h->aux_stream, hipStreamCaptureModeThreadLocal);
            if (e != hipSuccess) return device_fail(h, fn, e);
            e = enqueue_fixed_apsp(h, dt, n, W, ldw, D, ldd, T, ws, skws, skws_bytes, h->aux_stream);
            hipGraph_t graph = nullptr;
            const hipError_t e2 = hipStreamEndCapture(h->aux_stream, &graph);
            if (e == hipSuccess) e = e2;
            if (e == hipSuccess) e = hipGraphInstantiate(&h->apsp_exec, graph, nullptr, nullptr, 0);
            if (e != hipSuccess) {
                if (graph) (void)hipGraphDestroy(graph);
                h->apsp_exec = nullptr;
                return device_fail(h, fn, e);
            }
            h->apsp_graph = graph;
            h->apsp_key = key;
        }
        e = hipGraphLaunch(h->apsp_exec, h->stream);
        if (e != hipSuccess) return device_fail(h, fn, e);
        steps = T;
    } else if (!early) {
        e = enqueue_fixed_apsp(h, dt, n, W, ldw, D, ldd, T, ws, skws, skws_bytes, h->stream);
        if (e != hipSuccess) return device_fail(h, fn, e);
        steps = T;
    } else {
        // Early exit: the same sequence, reading the change flag after each squaring.
        void* bufs[2] = {D, ws};
        long lds[2] = {ldd, n};
        int cur = (T % 2 == 0) ? 0 : 1;
        int* wide = dt == BTAS_INT32 ? h->dflags + FLAG_STEP_WIDE : nullptr;
        if (wide) e = btas::launch_clear_flags(wide, T + 1, h->stream);
        if (e == hipSuccess) e = btas::launch_apsp_init(dt, n, W, ldw, bufs[cur], lds[cur], wide, h->stream);
        if (e != hipSuccess) return device_fail(h, fn, e);
        const SparseMode smode = fixed ? SparseMode::Off : sparse_mode(n);
        bool sparse_phase = smode != SparseMode::Off;
        for (int t = 0; t < T; ++t) {
            const int nxt = cur ^ 1;
            int* changed = h->dflags + FLAG_CHANGED;
            e = btas::launch_clear_flags(changed, 1, h->stream);
            if (e != hipSuccess) return device_fail(h, fn, e);
            int ran_sparse = 0;
            if (sparse_phase) {
                btas_status_t st = BTAS_OK;
                ran_sparse = sparse_step(h, fn, dt, n, bufs[cur], lds[cur], bufs[nxt], lds[nxt], changed,
                                         wide ? wide + t + 1 : nullptr, smode, &st);
                if (ran_sparse < 0) return st;
                sparse_phase = ran_sparse == 1;
            }
            if (!ran_sparse) {
                btas::GemmArgs a{n, n, n, bufs[cur], lds[cur], bufs[cur], lds[cur], bufs[cur], lds[cur],
                                 bufs[nxt], lds[nxt], changed,
                                 wide ? wide + t : nullptr, wide ? wide + t + 1 : nullptr,
                                 skws, skws_bytes};
                e = btas::launch_gemm(BTAS_MIN_PLUS, dt, a, -1, h->stream);
                if (e != hipSuccess) return device_fail(h, fn, e);
            }
            ++steps;
            cur = nxt;
            btas_status_t st = sync_flags(h, fn, FLAG_CHANGED + 1);
            if (st != BTAS_OK) return st;
            if (h->hflags[FLAG_CHANGED] == 0) break;
        }
        if (cur != 0) {
            e = btas::launch_copy_matrix(n, n, bufs[cur], lds[cur], D, ldd, h->stream);
            if (e != hipSuccess) return device_fail(h, fn, e);
        }
    }
    btas_status_t result = BTAS_OK;
    if (flags & BTAS_APSP_CHECK_NEG_CYCLE) {
        int* flag = h->dflags + FLAG_CHECK;
        e = btas::launch_clear_flags(flag, 1, h->stream);
        if (e == hipSuccess) e = btas::launch_neg_diag_check(dt, n, D, ldd, flag, h->stream);
        if (e != hipSuccess) return device_fail(h, fn, e);
        btas_status_t st = sync_flags(h, fn, FLAG_CHECK + 1);
        if (st != BTAS_OK) return st;
        if (h->hflags[FLAG_CHECK]) result = fail(h, BTAS_WARN_NEG_CYCLE, "%s: negative cycle (some D_ii < 0)", fn);
    }
    if (steps_out) {
        e = hipStreamSynchronize(h->stream);
        if (e != hipSuccess) return device_fail(h, fn, e);
        *steps_out = steps;
    }
    return result;
}

}  // namespace

btas_status_t btas_apsp_squaring(btas_handle_t h, btas_dtype_t dt, int n, const void* W, int ldw,
                                 void* D, int ldd, unsigned flags, int* steps_out) {
    return apsp_impl(h, "btas_apsp_squaring", dt, n, W, ldw, D, ldd, flags, steps_out, nullptr);
}

btas_status_t btas_apsp_squaring_noalloc(btas_handle_t h, btas_dtype_t dt, int n, const void* W,
                                         int ldw, void* D, int ldd, unsigned flags,
                                         int* steps_out) {
    const char* fn = "btas_apsp_squaring_noalloc";
    if (!h) return BTAS_ERR_INVALID_ARG;
    if (!h->scratch)
        return fail(h, BTAS_ERR_DEVICE, "%s: the device address of the fixed workspace is unknown", fn);
    const FixedWs f{static_cast<unsigned char*>(h->scratch), btas::NOALLOC_SCRATCH_BYTES};
    return apsp_impl(h, fn, dt, n, W, ldw, D, ldd, flags, steps_out, &f);
}

// ------------------------------------------------------ Floyd-Warshall ---
btas_status_t btas_apsp_floyd_warshall(btas_handle_t h, btas_dtype_t dt, int n, const void* W,
                                       int ldw, void* D, int ldd, unsigned flags) {
    const char* fn = "btas_apsp_floyd_warshall";
    if (!h) return BTAS_ERR_INVALID_ARG;
    if (btas_status_t l = begin_call(h, fn); l != BTAS_OK) return l;
    if (!dt_ok(dt)) return fail(h, BTAS_ERR_INVALID_ARG, "%s: argument 2 (dtype=%d) unknown", fn, (int)dt);
    if (n < 0) return fail(h, BTAS_ERR_INVALID_ARG, "%s: argument 3 (n=%d) < 0", fn, n);
    if (ldw < (n > 1 ? n : 1))
        return fail(h, BTAS_ERR_INVALID_ARG, "%s: argument 5 (ldw=%d) < max(1,n=%d)", fn, ldw, n);
    if (ldd < (n > 1 ? n : 1))
        return fail(h, BTAS_ERR_INVALID_ARG, "%s: argument 7 (ldd=%d) < max(1,n=%d)", fn, ldd, n);
    if (flags & ~BTAS_APSP_CHECK_NEG_CYCLE)
        return fail(h, BTAS_ERR_INVALID_ARG, "%s: argument 8 (flags=0x%x): only CHECK_NEG_CYCLE", fn, flags);
    if (n > 0 && (!W || !D)) return fail(h, BTAS_ERR_INVALID_ARG, "%s: W or D is null", fn);
    const bool in_place = W == D && ldw == ldd;
    if (!in_place && overlap(mat_span(W, n, n, ldw), mat_span(D, n, n, ldd)))
        return fail(h, BTAS_ERR_ALIAS, "%s: D partially overlaps W", fn);
    if (n == 0) return BTAS_OK;
    DeviceGuard g(h->device);
    {
        const void* ps[1] = {W};
        const long rows[1] = {n}, cols[1] = {n}, lds[1] = {ldw};
        btas_status_t st = validate_operands(h, fn, BTAS_MIN_PLUS, dt, ps, rows, cols, lds, 1);
        if (st != BTAS_OK) return st;
    }
    hipError_t e = btas::launch_apsp_init(dt, n, W, ldw, D, ldd, nullptr, h->stream);
    if (e == hipSuccess) e = btas::launch_floyd_warshall(dt, n, D, ldd, h->stream);
    if (e != hipSuccess) return device_fail(h, fn, e);
    if (flags & BTAS_APSP_CHECK_NEG_CYCLE) {
        int* flag = h->dflags + FLAG_CHECK;
        e = btas::launch_clear_flags(flag, 1, h->stream);
        if (e == hipSuccess) e = btas::launch_neg_diag_check(dt, n, D, ldd, flag, h->stream);
        if (e != hipSuccess) return device_fail(h, fn, e);
        btas_status_t st = sync_flags(h, fn, FLAG_CHECK + 1);
        if (st != BTAS_OK) return st;
        if (h->hflags[FLAG_CHECK]) return fail(h, BTAS_WARN_NEG_CYCLE, "%s: negative cycle (some D_ii < 0)", fn);
    }
    return BTAS_OK;
}

// ------------------------------------------------------------ witnesses ---
btas_status_t btas_tropical_gemm_witness(btas_handle_t h, btas_semiring_t sr, btas_dtype_t dt,
                                         int m, int n, int k, const void* A, int lda,
                                         const void* B, int ldb, void* C, int ldc, int32_t* K,
                                         int ldk) {
    const char* fn = "btas_tropical_gemm_witness";
    btas_status_t st = check_common(h, fn, sr, dt);
    if (st != BTAS_OK) return st;
    if (m < 0) return fail(h, BTAS_ERR_INVALID_ARG, "%s: argument 4 (m=%d) < 0", fn, m);
    if (n < 0) return fail(h, BTAS_ERR_INVALID_ARG, "%s: argument 5 (n=%d) < 0", fn, n);
    if (k < 0) return fail(h, BTAS_ERR_INVALID_ARG, "%s: argument 6 (k=%d) < 0", fn, k);
    if (lda < (k > 1 ? k : 1))
        return fail(h, BTAS_ERR_INVALID_ARG, "%s: argument 8 (lda=%d) < max(1,k=%d)", fn, lda, k);
    if (ldb < (n > 1 ? n : 1))
        return fail(h, BTAS_ERR_INVALID_ARG, "%s: argument 10 (ldb=%d) < max(1,n=%d)", fn, ldb, n);
    if (ldc < (n > 1 ? n : 1))
        return fail(h, BTAS_ERR_INVALID_ARG, "%s: argument 12 (ldc=%d) < max(1,n=%d)", fn, ldc, n);
    if (ldk < (n > 1 ? n : 1))
        return fail(h, BTAS_ERR_INVALID_ARG, "%s: argument 14 (ldk=%d) < max(1,n=%d)", fn, ldk, n);
    if ((long)m * k > 0 && !A) return fail(h, BTAS_ERR_INVALID_ARG, "%s: argument 7 (A) is null", fn);
    if ((long)k * n > 0 && !B) return fail(h, BTAS_ERR_INVALID_ARG, "%s: argument 9 (B) is null", fn);
    if ((long)m * n > 0 && !C) return fail(h, BTAS_ERR_INVALID_ARG, "%s: argument 11 (C) is null", fn);
    if ((long)m * n > 0 && !K) return fail(h, BTAS_ERR_INVALID_ARG, "%s: argument 13 (K) is null", fn);
    const Span sc = mat_span(C, m, n, ldc), sk = mat_span(K, m, n, ldk);
    const Span sa = mat_span(A, m, k, lda), sb = mat_span(B, k, n, ldb);
    if (overlap(sc, sa) || overlap(sc, sb) || overlap(sk, sa) || overlap(sk, sb) || overlap(sk, sc))
        return fail(h, BTAS_ERR_ALIAS, "%s: C or K overlaps another operand", fn);
    if (m == 0 || n == 0 || k == 0) return BTAS_OK;
    DeviceGuard g(h->device);
    const void* ps[2] = {A, B};
    const long rows[2] = {m, k}, cols[2] = {k, n}, lds[2] = {lda, ldb};
    st = validate_operands(h, fn, sr, dt, ps, rows, cols, lds, 2);
    if (st != BTAS_OK) return st;
    hipError_t e = btas::launch_gemm_witness(sr, dt, m, n, k, A, lda, B, ldb, C, ldc, K, ldk,
                                             h->stream);
    return e == hipSuccess ? BTAS_OK : device_fail(h, fn, e);
}

btas_status_t btas_apsp_successors(btas_handle_t h, btas_dtype_t dt, int n, const void* W, int ldw,
                                   const void* D, int ldd, int32_t* S, int lds) {
    const char* fn = "btas_apsp_successors";
    if (!h) return BTAS_ERR_INVALID_ARG;
    if (btas_status_t l = begin_call(h, fn); l != BTAS_OK) return l;
    if (!dt_ok(dt)) return fail(h, BTAS_ERR_INVALID_ARG, "%s: argument 2 (dtype=%d) unknown", fn, (int)dt);
    if (n < 0) return fail(h, BTAS_ERR_INVALID_ARG, "%s: argument 3 (n=%d) < 0", fn, n);
    if (ldw < (n > 1 ? n : 1))
        return fail(h, BTAS_ERR_INVALID_ARG, "%s: argument 5 (ldw=%d) < max(1,n=%d)", fn, ldw, n);
    if (ldd < (n > 1 ? n : 1))
        return fail(h, BTAS_ERR_INVALID_ARG, "%s: argument 7 (ldd=%d) < max(1,n=%d)", fn, ldd, n);
    if (lds < (n > 1 ? n : 1))
        return fail(h, BTAS_ERR_INVALID_ARG, "%s: argument 9 (lds=%d) < max(1,n=%d)", fn, lds, n);
    if (n > 0 && (!W || !D || !S)) return fail(h, BTAS_ERR_INVALID_ARG, "%s: W, D or S is null", fn);
    const Span ss = mat_span(S, n, n, lds);
    if (overlap(ss, mat_span(W, n, n, ldw)) || overlap(ss, mat_span(D, n, n, ldd)))
        return fail(h, BTAS_ERR_ALIAS, "%s: S overlaps W or D", fn);
    if (n == 0) return BTAS_OK;
    DeviceGuard g(h->device);
    const void* ps[2] = {W, D};
    const long rows[2] = {n, n}, cols[2] = {n, n}, ldv[2] = {ldw, ldd};
    btas_status_t st = validate_operands(h, fn, BTAS_MIN_PLUS, dt, ps, rows, cols, ldv, 2);
    if (st != BTAS_OK) return st;
    const SparseMode mode = n <= SPARSE_MAX_N ? sparse_mode(n) : SparseMode::Off;
    const char* env = getenv("BTAS_SPARSE_STEPS");
    if (!(env && env[0] == '0') && (n >= 256 || mode == SparseMode::Force)) {
        const int r = sparse_successors(h, fn, dt, n, W, ldw, D, ldd, S, lds, &st);
        if (r < 0) return st;
        if (r == 1) return BTAS_OK;
    }
    hipError_t e = btas::launch_successors(dt, n, W, ldw, D, ldd, S, lds, h->stream);
    return e == hipSuccess ? BTAS_OK : device_fail(h, fn, e);
}

// ------------------------------------------------------------- closure ---
btas_status_t btas_tropical_closure(btas_handle_t h, btas_semiring_t sr, btas_dtype_t dt, int n,
                                    const void* W, int ldw, void* D, int ldd, unsigned flags,
                                    int* steps_out) {
    const char* fn = "btas_tropical_closure";
    if (!h) return BTAS_ERR_INVALID_ARG;
    if (btas_status_t l = begin_call(h, fn); l != BTAS_OK) return l;
    if (steps_out) *steps_out = 0;
    if (sr != BTAS_MIN_PLUS && sr != BTAS_MAX_PLUS)
        return fail(h, BTAS_ERR_INVALID_ARG, "%s: argument 2 (semiring=%d) unknown", fn, (int)sr);
    if (flags & ~(BTAS_APSP_EARLY_EXIT | BTAS_APSP_CHECK_NEG_CYCLE))
        return fail(h, BTAS_ERR_INVALID_ARG, "%s: argument 9 (flags=0x%x): EARLY_EXIT, CHECK_NEG_CYCLE",
                    fn, flags);
    if (sr == BTAS_MIN_PLUS) return btas_apsp_squaring(h, dt, n, W, ldw, D, ldd, flags, steps_out);
    if (!dt_ok(dt)) return fail(h, BTAS_ERR_INVALID_ARG, "%s: argument 3 (dtype=%d) unknown", fn, (int)dt);
    if (n < 0) return fail(h, BTAS_ERR_INVALID_ARG, "%s: argument 4 (n=%d) < 0", fn, n);
    if (ldw < (n > 1 ? n : 1))
        return fail(h, BTAS_ERR_INVALID_ARG, "%s: argument 6 (ldw=%d) < max(1,n=%d)", fn, ldw, n);
    if (ldd < (n > 1 ? n : 1))
        return fail(h, BTAS_ERR_INVALID_ARG, "%s: argument 8 (ldd=%d) < max(1,n=%d)", fn, ldd, n);
    if (n > 0 && (!W || !D)) return fail(h, BTAS_ERR_INVALID_ARG, "%s: W or D is null", fn);
    const bool in_place = W == D && ldw == ldd;
    if (!in_place && overlap(mat_span(W, n, n, ldw), mat_span(D, n, n, ldd)))
        return fail(h, BTAS_ERR_ALIAS, "%s: D partially overlaps W", fn);
    if (n == 0) return BTAS_OK;
    DeviceGuard g(h->device);
    {
        const void* ps[1] = {W};
        const long rows[1] = {n}, cols[1] = {n}, lds[1] = {ldw};
        btas_status_t st = validate_operands(h, fn, BTAS_MAX_PLUS, dt, ps, rows, cols, lds, 1);
        if (st != BTAS_OK) return st;
    }
    const int T = btas_apsp_num_steps(n);
    if (T > 0 && ensure_ws(h, (size_t)n * n * 4) != hipSuccess)
        return fail(h, BTAS_ERR_OOM, "%s: cannot allocate the %zu-byte workspace", fn, (size_t)n * n * 4);
    if (T > 0 && ensure_splitk(h, btas::gemm_splitk_bytes(n, n, n)) != hipSuccess)
        return fail(h, BTAS_ERR_OOM, "%s: cannot allocate the split-K workspace", fn);
    const bool early = flags & BTAS_APSP_EARLY_EXIT;
    void* bufs[2] = {D, h->ws};
    long lds[2] = {ldd, n};
    int cur = (T % 2 == 0) ? 0 : 1;
    int* wide = dt == BTAS_INT32 ? h->dflags + FLAG_STEP_WIDE : nullptr;
    hipError_t e = hipSuccess;
    if (wide) e = btas::launch_clear_flags(wide, T + 1, h->stream);
    if (e == hipSuccess)
        e = btas::launch_closure_init(BTAS_MAX_PLUS, dt, n, W, ldw, bufs[cur], lds[cur], wide, h->stream);
    if (e != hipSuccess) return device_fail(h, fn, e);
    int steps = 0;
    for (int t = 0; t < T; ++t) {
        const int nxt = cur ^ 1;
        int* changed = early ? h->dflags + FLAG_CHANGED : nullptr;
        if (changed) e = btas::launch_clear_flags(changed, 1, h->stream);
        btas::GemmArgs a{n, n, n, bufs[cur], lds[cur], bufs[cur], lds[cur], bufs[cur], lds[cur],
                         bufs[nxt], lds[nxt], changed,
                         wide ? wide + t : nullptr, wide ? wide + t + 1 : nullptr,
                         h->skws, h->skws_bytes};
        if (e == hipSuccess) e = btas::launch_gemm(BTAS_MAX_PLUS, dt, a, -1, h->stream);
        if (e != hipSuccess) return device_fail(h, fn, e);
        ++steps;
        cur = nxt;
        if (early) {
            btas_status_t st = sync_flags(h, fn, FLAG_CHANGED + 1);
            if (st != BTAS_OK) return st;
            if (h->hflags[FLAG_CHANGED] == 0) break;
        }
    }
    if (cur != 0) {
        e = btas::launch_copy_matrix(n, n, bufs[cur], lds[cur], D, ldd, h->stream);
        if (e != hipSuccess) return device_fail(h, fn, e);
    }
    if (steps_out) *steps_out = steps;
    if (flags & BTAS_APSP_CHECK_NEG_CYCLE) {
        int* flag = h->dflags + FLAG_CHECK;
        e = btas::launch_clear_flags(flag, 1, h->stream);
        if (e == hipSuccess) e = btas::launch_diag_check(BTAS_MAX_PLUS, dt, n, D, ldd, flag, h->stream);
        if (e != hipSuccess) return device_fail(h, fn, e);
        btas_status_t st = sync_flags(h, fn, FLAG_CHECK + 1);
        if (st != BTAS_OK) return st;
        if (h->hflags[FLAG_CHECK]) return fail(h, BTAS_WARN_POS_CYCLE, "%s: positive cycle (some D_ii > 0)", fn);
    }
    return BTAS_OK;
}

// ---------------------------------------------------------- cycle mean ---
btas_status_t btas_maxplus_cycle_mean(btas_handle_t h, btas_dtype_t dt, int n, const void* A, int lda,
                                      int64_t* num, int64_t* den, double* lambda) {
    const char* fn = "btas_maxplus_cycle_mean";
    if (!h) return BTAS_ERR_INVALID_ARG;
    if (btas_status_t l = begin_call(h, fn); l != BTAS_OK) return l;
    if (!dt_ok(dt)) return fail(h, BTAS_ERR_INVALID_ARG, "%s: argument 2 (dtype=%d) unknown", fn, (int)dt);
    if (n < 0) return fail(h, BTAS_ERR_INVALID_ARG, "%s: argument 3 (n=%d) < 0", fn, n);
    if (lda < (n > 1 ? n : 1))
        return fail(h, BTAS_ERR_INVALID_ARG, "%s: argument 5 (lda=%d) < max(1,n=%d)", fn, lda, n);
    if (n > 0 && !A) return fail(h, BTAS_ERR_INVALID_ARG, "%s: argument 4 (A) is null", fn);
    if (num) *num = 0;
    if (den) *den = 0;
    if (lambda) *lambda = -__builtin_inf();
    if (n == 0) return BTAS_OK;
    DeviceGuard g(h->device);
    {
        const void* ps[1] = {A};
        const long rows[1] = {n}, cols[1] = {n}, lds[1] = {lda};
        btas_status_t st = validate_operands(h, fn, BTAS_MAX_PLUS, dt, ps, rows, cols, lds, 1);
        if (st != BTAS_OK) return st;
    }
    hipError_t e = hipSuccess;
    if (dt == BTAS_INT32) {
        // walks of up to n edges must stay inside the int32 domain bound
        int* m = h->dflags + FLAG_CM_MAXABS;
        e = btas::launch_clear_flags(m, 1, h->stream);
        if (e == hipSuccess) e = btas::launch_cycle_mean_maxabs(n, A, lda, m, h->stream);
        if (e != hipSuccess) return device_fail(h, fn, e);
        btas_status_t st = sync_flags(h, fn, FLAG_CM_MAXABS + 1);
        if (st != BTAS_OK) return st;
        if ((long long)n * h->hflags[FLAG_CM_MAXABS] > (long long)BTAS_I32_FINITE_MAX)
            return fail(h, BTAS_ERR_DOMAIN, "%s: n * max|A| = %lld exceeds 2^29-1 (walk weights overflow)",
                        fn, (long long)n * h->hflags[FLAG_CM_MAXABS]);
    }
    const size_t need = btas::cycle_mean_ws_bytes(n);
    if (ensure_ws(h, need) != hipSuccess)
        return fail(h, BTAS_ERR_OOM, "%s: cannot allocate the %zu-byte workspace", fn, need);
    long long* result = reinterpret_cast<long long*>(h->dflags + FLAG_CM_RESULT);
    int uses_err = 0;
    e = btas::launch_cycle_mean(dt, n, A, lda, h->ws, result, h->num_cus, &uses_err, h->stream);
    if (e != hipSuccess) return device_fail(h, fn, e);
    btas_status_t st = sync_flags(h, fn, FLAG_CM_RESULT + 6);
    if (st != BTAS_OK) return st;
    if (uses_err) {
        int err = 0;
        e = hipMemcpy(&err, btas::cycle_mean_error_word(n, h->ws), sizeof err, hipMemcpyDeviceToHost);
        if (e != hipSuccess) return device_fail(h, fn, e);
        if (err) return fail(h, BTAS_ERR_DEVICE, "%s: device-wide barrier timed out", fn);
    }
    int64_t r[3];
    memcpy(r, h->hflags + FLAG_CM_RESULT, sizeof r);
    if (num) *num = r[0];
    if (den) *den = r[1];
    if (lambda) memcpy(lambda, &r[2], sizeof(double));
    return BTAS_OK;
}

}  // extern "C"
