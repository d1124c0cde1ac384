// Handle state and host helpers shared by the C-ABI translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdarg>
#include <cstdint>
#include <cstdio>
#include <map>
#include <memory>
#include <string>
#include <tuple>
#include <utility>

#include "btas.h"
#include "kernels.h"

namespace btas {
struct BatchPlan;  // batched_api.cpp
void destroy_batch_plan(BatchPlan* p);
struct BatchPlanDeleter {
    void operator()(BatchPlan* p) const { destroy_batch_plan(p); }
};
struct FwBatchPlan;  // batched_api.cpp
void destroy_fw_batch_plan(FwBatchPlan* p);
struct FwBatchPlanDeleter {
    void operator()(FwBatchPlan* p) const { destroy_fw_batch_plan(p); }
};
// Measured speed of one size bucket's squaring: for each tile family (0 =
// four-wave blocks, 1 = single waves, 2 = single-wave direct loads on padded
// buffers) the fastest shape and its seconds per useful term.
struct BucketTiming {
    int best[3];
    double spt[3];
};
}  // namespace btas

struct btas_ctx {
    int device = 0;
    hipStream_t stream = nullptr;        // borrowed
    hipStream_t aux_stream = nullptr;    // owned: graph capture and autotuning
    std::string last_error;
    bool validate = false;
    int num_cus = 0;                     // compute units of the device
    void* ws = nullptr;                  // APSP ping-pong partner matrix
    size_t ws_bytes = 0;
    void* partials = nullptr;            // dot reduction partials
    void* skws = nullptr;                // split-K partial products
    size_t skws_bytes = 0;
    int* dflags = nullptr;               // device flags [kNumFlags], see the FLAG_* slots
    int* hflags = nullptr;               // pinned host mirror
    // Pinned host word that a single-launch solve sets (from the device) when
    // one of its device-wide barrier waits hit its bound; reported and cleared
    // by the next call on the handle or by btas_synchronize.
    int* hlatch = nullptr;
    int spin_limit = 1 << 20;            // polls per device-wide barrier wait
    void* scratch = nullptr;             // this device's fixed no-allocation workspace
    int last_packed16 = 0;               // the last read single-launch solve ran 16-bit lanes
    unsigned resident_epoch = 0;         // tag of the last single-launch solve's barrier words
    // Single-launch solve's tag buffer (btas::resident_tag_bytes()): written
    // only by those launches, zeroed with the barrier words.
    void* tagws = nullptr;
    std::unique_ptr<btas::BatchPlan, btas::BatchPlanDeleter> batch_plan;  // last batched plan
    std::unique_ptr<btas::FwBatchPlan, btas::FwBatchPlanDeleter> fw_batch_plan;  // last batched FW plan
    std::map<std::pair<int, int>, int> tile_choice;  // (dtype, size bucket) -> shape of the last plan
    // (dtype, size bucket, log2 of the plan's launch size) -> autotune result
    std::map<std::tuple<int, int, int>, btas::BucketTiming> tile_timing;
    void* sp_ws = nullptr;               // sparse squarings: row counts, row pointers, CSR
    size_t sp_bytes = 0;
    hipStream_t fork_stream = nullptr;   // owned: second branch of a captured batched solve
    hipEvent_t fork_event = nullptr;     // fork / join of that branch
    hipEvent_t join_event = nullptr;
    hipGraph_t apsp_graph = nullptr;     // last captured single-solve graph (BTAS_APSP_GRAPH)
    hipGraphExec_t apsp_exec = nullptr;
    uint64_t apsp_key = 0;
};

namespace btas {

// Device flag slots of a handle.
constexpr int FLAG_CHANGED = 0;    // early exit: some output changed this step
constexpr int FLAG_CHECK = 1;      // domain scan / negative-cycle check
constexpr int FLAG_GEMM_WIDE = 2;  // int32 gemm operands exceed the binary32-exact range
constexpr int FLAG_STEP_WIDE = 8;  // APSP: slot 8 + t describes D_t (t = 0..T <= 31)
constexpr int FLAG_SPARSE = 136;   // sparse squarings: two 64-bit counters (finite entries, terms)
constexpr int FLAG_CM_MAXABS = 140;  // cycle mean: max |A| of int32 entries
constexpr int FLAG_CM_RESULT = 144;  // cycle mean: num, den (int64), lambda bits (binary64)
// Single-launch solve: +0 error, +1 steps, then its barrier's arrival words
// (two sets of RESIDENT_MAX_GRID, one per barrier parity).
constexpr int FLAG_RESIDENT = 192;
constexpr int FLAG_RESIDENT_END = FLAG_RESIDENT + 2 + 2 * RESIDENT_MAX_GRID;
constexpr int kNumFlags = FLAG_RESIDENT_END;
static_assert(FLAG_STEP_WIDE + 32 <= FLAG_SPARSE && FLAG_SPARSE % 2 == 0 && FLAG_SPARSE + 4 <= FLAG_CM_MAXABS &&
                  FLAG_CM_MAXABS < FLAG_CM_RESULT && FLAG_CM_RESULT % 2 == 0 &&
                  FLAG_CM_RESULT + 6 <= FLAG_RESIDENT,
              "flag slots overlap");

struct DeviceGuard {
    int prev = -1;
    bool ok = false;
    explicit DeviceGuard(int dev) {
        if (hipGetDevice(&prev) != hipSuccess) prev = -1;
        ok = hipSetDevice(dev) == hipSuccess;
    }
    ~DeviceGuard() {
        if (prev >= 0) (void)hipSetDevice(prev);
    }
};

inline btas_status_t fail(btas_handle_t h, btas_status_t st, const char* fmt, ...) {
    if (h) {
        char buf[512];
        va_list ap;
        va_start(ap, fmt);
        vsnprintf(buf, sizeof buf, fmt, ap);
        va_end(ap);
        h->last_error = buf;
    }
    return st;
}

inline btas_status_t device_fail(btas_handle_t h, const char* where, hipError_t e) {
    return fail(h, BTAS_ERR_DEVICE, "%s: HIP error %d (%s)", where, (int)e, hipGetErrorString(e));
}

// Start of every entry point on a handle: clears the last error and reports
// (once) a barrier timeout latched by an earlier single-launch solve whose
// caller did not synchronise on it.  The word is written by the device only
// on that error path and is visible here once that kernel has ended.
inline btas_status_t begin_call(btas_handle_t h, const char* fn) {
    h->last_error.clear();
    if (h->hlatch && __atomic_load_n(h->hlatch, __ATOMIC_ACQUIRE) != 0) {
        __atomic_store_n(h->hlatch, 0, __ATOMIC_RELEASE);
        return fail(h, BTAS_ERR_DEVICE,
                    "%s: an earlier single-launch APSP solve on this handle timed out "
                    "waiting on other workgroups; its D is not valid", fn);
    }
    return BTAS_OK;
}

// Byte span [lo, hi) touched by a row-major rows x cols matrix with leading
// dimension ld (4-byte elements); empty when rows or cols is 0.
struct Span {
    uintptr_t lo = 0, hi = 0;
    bool empty() const { return hi <= lo; }
};
inline Span mat_span(const void* p, long rows, long cols, long ld) {
    Span s;
    if (rows <= 0 || cols <= 0 || p == nullptr) return s;
    s.lo = (uintptr_t)p;
    s.hi = s.lo + (uintptr_t)(((rows - 1) * ld + cols) * 4);
    return s;
}
inline Span vec_span(const void* p, long n, long inc) {
    Span s;
    if (n <= 0 || p == nullptr) return s;
    s.lo = (uintptr_t)p;
    s.hi = s.lo + (uintptr_t)(((n - 1) * inc + 1) * 4);
    return s;
}
inline bool overlap(const Span& a, const Span& b) {
    return !a.empty() && !b.empty() && a.lo < b.hi && b.lo < a.hi;
}

// Grow the split-K workspace to `need` bytes (0: nothing to do).  The old
// buffer may still be read by queued work, so the stream is drained first.
inline hipError_t ensure_splitk(btas_handle_t h, size_t need) {
    if (need <= h->skws_bytes) return hipSuccess;
    if (h->skws) {
        hipError_t e = hipStreamSynchronize(h->stream);
        if (e != hipSuccess) return e;
        (void)hipFree(h->skws);
        h->skws = nullptr;
        h->skws_bytes = 0;
    }
    hipError_t e = hipMalloc(&h->skws, need);
    if (e == hipSuccess) h->skws_bytes = need;
    return e;
}

inline int apsp_steps(int n) {
    if (n <= 2) return 0;
    int t = 0;
    long reach = 1;
    while (reach < (long)n - 1) {
        reach *= 2;
        ++t;
    }
    return t;
}

}  // namespace btas
