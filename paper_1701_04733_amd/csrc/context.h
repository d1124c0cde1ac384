// Handle state and host helpers shared by the C-ABI translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdarg>
#include <cstdint>
#include <cstdio>
#include <map>
#include <memory>
#include <string>
#include <utility>

#include "btas.h"

namespace btas {
struct BatchPlan;  // batched_api.cpp
void destroy_batch_plan(BatchPlan* p);
struct BatchPlanDeleter {
    void operator()(BatchPlan* p) const { destroy_batch_plan(p); }
};
}  // namespace btas

struct btas_ctx {
    int device = 0;
    hipStream_t stream = nullptr;        // borrowed
    hipStream_t aux_stream = nullptr;    // owned: graph capture and autotuning
    std::string last_error;
    bool validate = false;
    void* ws = nullptr;                  // APSP ping-pong partner matrix
    size_t ws_bytes = 0;
    void* partials = nullptr;            // dot reduction partials
    int* dflags = nullptr;               // device flags [kNumFlags], see the FLAG_* slots
    int* hflags = nullptr;               // pinned host mirror
    std::unique_ptr<btas::BatchPlan, btas::BatchPlanDeleter> batch_plan;  // last batched plan
    std::map<std::pair<int, int>, int> tile_choice;  // (dtype, size bucket) -> tile shape
};

namespace btas {

// Device flag slots of a handle.
constexpr int FLAG_CHANGED = 0;    // early exit: some output changed this step
constexpr int FLAG_CHECK = 1;      // domain scan / negative-cycle check
constexpr int FLAG_GEMM_WIDE = 2;  // int32 gemm operands exceed the binary32-exact range
constexpr int FLAG_STEP_WIDE = 8;  // APSP: slot 8 + t describes D_t (t = 0..T <= 32)
constexpr int kNumFlags = 64;

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
