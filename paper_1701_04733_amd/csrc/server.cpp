// Serving engine for APSP requests: admission by a device-memory budget,
// device-resident distance matrices, and continuous batching at squaring
// granularity (Sec. III squarings of many requests share each launch).
//
// One engine thread owns a non-blocking stream and loops:
//   1. admit pending requests in arrival order while the memory pool has room
//      for their two padded n x n buffers and their COO edges; upload the edges
//      and densify I (+) W on the device;
//   2. build one work list: for every active request, the next tiles of its
//      current squaring, at most `quantum` terms' worth per request (a large
//      request's squaring is spread over several launches, so small requests
//      never wait for a whole large squaring: round-robin processor sharing);
//   3. launch the grouped step kernel once for the whole list, wait for it;
//   4. advance requests whose squaring completed; finish those that ran T(n)
//      squarings (or, with early exit, one that changed nothing); signal
//      waiters.
// In FIFO mode the engine instead runs one request at a time with the plain
// single-solve path (one GEMM launch per squaring): the baseline that the
// continuous mode is compared against on the same request trace.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <string>
#include <chrono>
#include <condition_variable>
#include <cstdlib>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "batched.h"
#include "btas.h"
#include "gemm_tile.h"
#include "kernels.h"
#include "range_alloc.h"

namespace btas {
namespace {

size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

int steps_for(int n) {
    if (n <= 2) return 0;
    int t = 0;
    long reach = 1;
    while (reach < (long)n - 1) {
        reach *= 2;
        ++t;
    }
    return t;
}

// The memory pool: one device allocation carved by a RangeAllocator.
class DevicePool {
   public:
    bool init(size_t bytes) {
        ranges_.reset(bytes);
        if (hipMalloc(&base_, ranges_.size()) != hipSuccess) {
            base_ = nullptr;
            return false;
        }
        return true;
    }
    ~DevicePool() {
        if (base_) (void)hipFree(base_);
    }
    // Shared by the engine lanes: each call takes the pool's own lock (always
    // after a lane's lock, never the other way round).
    size_t alloc(size_t bytes) {
        std::lock_guard<std::mutex> g(m_);
        return ranges_.alloc(bytes);
    }
    void release(size_t off, size_t bytes) {
        std::lock_guard<std::mutex> g(m_);
        ranges_.release(off, bytes);
    }
    char* at(size_t off) const { return (char*)base_ + off; }
    size_t size() const { return ranges_.size(); }
    size_t used() const {
        std::lock_guard<std::mutex> g(m_);
        return ranges_.used();
    }
    size_t peak() const {
        std::lock_guard<std::mutex> g(m_);
        return ranges_.peak();
    }

   private:
    void* base_ = nullptr;
    RangeAllocator ranges_;
    mutable std::mutex m_;
};

enum ReqState { PENDING = 0, ACTIVE = 1, DONE = 2, FAILED = 3 };

struct Request {
    int64_t id = 0;
    int n = 0, T = 0, ld = 0, nnz = 0, ntiles = 0;
    std::vector<TileRef> tiles;  // output tiles of one squaring
    bool early = false;
    int maxabs = 0;
    std::vector<int32_t> rows, cols;
    std::vector<uint32_t> w;
    double arrival = 0, admitted = -1, done = -1;
    int state = PENDING;
    size_t off = SIZE_MAX, bytes = 0;   // matrices
    size_t coo_off = SIZE_MAX, coo_bytes = 0;
    void* buf[2] = {nullptr, nullptr};
    int planned = 0;      // squarings whose tiles have all been enqueued
    int next_tile = 0;    // first tile of squaring planned+1 not yet enqueued
    int done_steps = 0;   // squarings known complete
    int changed_acc = 0;  // some entry changed in the squaring in flight (early exit)
    int refs = 0;         // launches in flight that name this request
    bool released = false;  // the client released it while refs > 0: free at refs == 0
};

// Host-pinned and device copies of one launch's descriptors.
struct Staging {
    BatchGraph* h_graphs = nullptr;
    BatchItem* h_items = nullptr;
    int* h_maxabs = nullptr;
    int* h_changed = nullptr;
    BatchGraph* d_graphs = nullptr;
    BatchItem* d_items = nullptr;
    int* d_maxabs = nullptr;
    int* d_changed = nullptr;
    size_t cap_graphs = 0, cap_items = 0;

    void free_graphs() {
        for (void** p : {(void**)&h_graphs, (void**)&h_maxabs, (void**)&h_changed})
            if (*p) (void)hipHostFree(*p), *p = nullptr;
        for (void** p : {(void**)&d_graphs, (void**)&d_maxabs, (void**)&d_changed})
            if (*p) (void)hipFree(*p), *p = nullptr;
        cap_graphs = 0;
    }
    void free_items() {
        if (h_items) (void)hipHostFree(h_items), h_items = nullptr;
        if (d_items) (void)hipFree(d_items), d_items = nullptr;
        cap_items = 0;
    }
    // Only called when no launch that uses this staging set is in flight.
    bool reserve(size_t ng, size_t ni) {
        if (ng > cap_graphs) {
            const size_t c = std::max(ng, cap_graphs * 2 + 64);
            free_graphs();
            if (hipHostMalloc((void**)&h_graphs, c * sizeof(BatchGraph), 0) != hipSuccess ||
                hipHostMalloc((void**)&h_maxabs, c * sizeof(int), 0) != hipSuccess ||
                hipHostMalloc((void**)&h_changed, c * sizeof(int), 0) != hipSuccess ||
                hipMalloc((void**)&d_graphs, c * sizeof(BatchGraph)) != hipSuccess ||
                hipMalloc((void**)&d_maxabs, c * sizeof(int)) != hipSuccess ||
                hipMalloc((void**)&d_changed, c * sizeof(int)) != hipSuccess)
                return false;
            cap_graphs = c;
        }
        if (ni > cap_items) {
            const size_t c = std::max(ni, cap_items * 2 + 1024);
            free_items();
            if (hipHostMalloc((void**)&h_items, c * sizeof(BatchItem), 0) != hipSuccess ||
                hipMalloc((void**)&d_items, c * sizeof(BatchItem)) != hipSuccess)
                return false;
            cap_items = c;
        }
        return true;
    }
};

// One enqueued unit of device work and what its completion means.
struct Launch {
    int slot = -1;                       // staging set used (-1: none)
    hipEvent_t ev = nullptr;
    std::vector<Request*> graphs;        // graph index -> request
    std::vector<char> ends_step;         // launch holds the last tiles of that squaring
    std::vector<Request*> densified;     // admitted just before this launch
    std::vector<Request*> whole;         // FIFO mode: solved entirely by this launch
};

}  // namespace

struct Server {
    int device = 0;
    int dt = BTAS_FLOAT32;
    int mode = 0;
    double quantum = 6e10;
    double launch_terms = 0;             // > 0: a launch holds at most about this much work,
                                         // split evenly over the requests it advances
    hipStream_t stream = nullptr;
    DevicePool* pool = nullptr;          // shared with the other lane
    Server* peer = nullptr;              // the other lane (continuous mode), or null
    std::chrono::steady_clock::time_point t0 = std::chrono::steady_clock::now();

    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<Request*> pending;
    std::vector<Request*> active;        // admitted, not finished, in admission order
    std::unordered_map<int64_t, std::unique_ptr<Request>> all;
    int64_t next_id = 1;
    bool stop = false;
    bool admission_blocked = false;      // the head of `pending` did not fit the pool
    std::string error;
    std::thread engine;

    static constexpr int kDepth = 2;     // launches in flight
    // Below this many tiles a grouped launch cannot fill the GPU; requests at
    // the start of a squaring then get the single-GEMM path instead (split-K
    // for small n, XCD-swizzled large tiles for big n).
    static constexpr int kMinGroupedItems = 256;
    void* splitk_ws = nullptr;           // split-K partials of the single-GEMM path
    size_t splitk_bytes = 0;
    int* d_zero = nullptr;               // a device 0: "operands fit the binary32 path"
    Staging staging[kDepth];
    std::deque<Launch> inflight;
    std::vector<hipEvent_t> free_events;
    // statistics
    std::atomic<long> launches{0}, iterations{0};
    double busy_s = 0;

    double now() const {
        return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    }

    // Memory went back to the shared pool: let the other lane retry its
    // admission.  Called without holding this lane's lock.
    void wake_peer() {
        if (!peer) return;
        {
            std::lock_guard<std::mutex> g(peer->mu);
            peer->admission_blocked = false;
        }
        peer->cv_work.notify_all();
    }

    void free_staging() {
        if (splitk_ws) (void)hipFree(splitk_ws), splitk_ws = nullptr;
        if (d_zero) (void)hipFree(d_zero), d_zero = nullptr;
        for (Staging& st : staging) {
            st.free_graphs();
            st.free_items();
        }
        for (hipEvent_t e : free_events) (void)hipEventDestroy(e);
        free_events.clear();
    }

    hipEvent_t get_event() {
        if (!free_events.empty()) {
            hipEvent_t e = free_events.back();
            free_events.pop_back();
            return e;
        }
        hipEvent_t e = nullptr;
        if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) return nullptr;
        return e;
    }

    // Caller holds mu.  Admit pending requests in arrival order while the pool
    // has room.  FIFO mode admits one request only when nothing else is on the
    // device.
    void admit_locked(std::vector<Request*>& admitted) {
        admission_blocked = false;
        while (!pending.empty()) {
            if (mode == BTAS_SERVE_FIFO && (!active.empty() || !inflight.empty() || !admitted.empty()))
                break;
            Request* r = pending.front();
            const size_t half = align_up((size_t)r->n * r->ld * 4, 256);
            const size_t off = pool->alloc(2 * half);
            if (off == SIZE_MAX) {
                admission_blocked = true;
                break;
            }
            const size_t coo = align_up((size_t)r->nnz * 4, 256) * 3;
            const size_t coff = r->nnz > 0 ? pool->alloc(coo) : SIZE_MAX;
            if (r->nnz > 0 && coff == SIZE_MAX) {
                pool->release(off, 2 * half);
                admission_blocked = true;
                break;
            }
            r->off = off;
            r->bytes = 2 * half;
            r->coo_off = coff;
            r->coo_bytes = coo;
            r->buf[0] = pool->at(off);
            r->buf[1] = pool->at(off + half);
            r->state = ACTIVE;
            r->admitted = now();
            pending.pop_front();
            active.push_back(r);
            admitted.push_back(r);
        }
    }

    // Upload edges and densify on the engine stream (engine thread only).
    hipError_t densify(Request* r) {
        if (r->nnz > 0) {
            const size_t seg = align_up((size_t)r->nnz * 4, 256);
            char* base = pool->at(r->coo_off);
            hipError_t e = hipMemcpyAsync(base, r->rows.data(), r->nnz * 4, hipMemcpyHostToDevice, stream);
            if (e == hipSuccess) e = hipMemcpyAsync(base + seg, r->cols.data(), r->nnz * 4, hipMemcpyHostToDevice, stream);
            if (e == hipSuccess) e = hipMemcpyAsync(base + 2 * seg, r->w.data(), r->nnz * 4, hipMemcpyHostToDevice, stream);
            if (e != hipSuccess) return e;
            return launch_densify(dt, r->buf[0], r->n, r->ld, r->nnz, (const int32_t*)base,
                                  (const int32_t*)(base + seg), base + 2 * seg, stream);
        }
        return launch_densify(dt, r->buf[0], r->n, r->ld, 0, nullptr, nullptr, nullptr, stream);
    }

    // Early-exit requests are planned speculatively: the next squaring is
    // enqueued before the flag of the previous one is known.  When that flag
    // says the previous squaring changed nothing, D_s is a fixpoint, so the
    // speculative squaring s + 1 writes into the other buffer exactly the
    // values of D_s (and never touches buf[s & 1], which holds the result);
    // the request finishes with s steps, as with a wait per squaring, but
    // without leaving the launches in between.
    bool plannable(const Request* r) const { return r->planned < r->T; }

    // Fill a launch with, for every active request that can advance, the next
    // tiles of its next squaring (at most `quantum` terms of work each).
    // Planning assumes that every enqueued launch completes, which stream
    // order guarantees; only early-exit requests wait for their flag.
    hipError_t plan_and_enqueue(Launch& L, const std::vector<Request*>& order) {
        Staging& st = staging[L.slot];
        size_t ng = 0, ni = 0;
        for (Request* r : order)
            if (plannable(r)) {
                ++ng;
                ni += (size_t)(r->ntiles - r->next_tile);
            }
        if (!st.reserve(ng + 1, ni + 1)) return hipErrorOutOfMemory;
        // Few tiles in total: requests at a squaring boundary take the
        // single-GEMM path, one launch per request.
        const bool few = ni < (size_t)kMinGroupedItems;
        const double q_each = launch_terms > 0 && ng > 0 ? std::min(quantum, launch_terms / (double)ng) : quantum;
        int nitems = 0;
        std::vector<Request*> single;
        for (Request* r : order) {
            if (!plannable(r)) continue;
            const int gi = (int)L.graphs.size();
            st.h_graphs[gi] = {{r->buf[0], r->buf[1]}, r->n, r->ld, r->T, 0};
            st.h_maxabs[gi] = r->maxabs;
            st.h_changed[gi] = 0;
            if (few && r->next_tile == 0) {
                single.push_back(r);
                r->next_tile = r->ntiles;
            } else {
                double work = 0;  // terms scheduled for this request in this launch
                while (r->next_tile < r->ntiles && (work == 0 || work < q_each)) {
                    const TileRef& t = r->tiles[r->next_tile++];
                    st.h_items[nitems++] = {gi, t.m0, t.n0, t.kind, r->planned + 1, 0};
                    work += (t.kind == BATCH_TILE_128 ? 16384.0 : 4096.0) * r->n;
                }
            }
            const bool ends = r->next_tile == r->ntiles;
            L.graphs.push_back(r);
            L.ends_step.push_back(ends);
        }
        const int g = (int)L.graphs.size();
        if (g == 0) return hipSuccess;
        hipError_t e = hipMemcpyAsync(st.d_changed, st.h_changed, g * sizeof(int), hipMemcpyHostToDevice, stream);
        if (e == hipSuccess && nitems > 0) {
            e = hipMemcpyAsync(st.d_graphs, st.h_graphs, g * sizeof(BatchGraph), hipMemcpyHostToDevice, stream);
            if (e == hipSuccess) e = hipMemcpyAsync(st.d_maxabs, st.h_maxabs, g * sizeof(int), hipMemcpyHostToDevice, stream);
            if (e == hipSuccess) e = hipMemcpyAsync(st.d_items, st.h_items, nitems * sizeof(BatchItem), hipMemcpyHostToDevice, stream);
            if (e == hipSuccess)
                e = launch_grouped_step(dt, st.d_graphs, st.d_items, nitems,
                                        dt == BTAS_INT32 ? st.d_maxabs : nullptr, st.d_changed, stream);
            launches++;
        }
        for (size_t i = 0; e == hipSuccess && i < L.graphs.size(); ++i) {
            Request* r = L.graphs[i];
            if (std::find(single.begin(), single.end(), r) == single.end()) continue;
            const int s = r->planned + 1;  // squaring s reads buf[(s-1)&1], writes buf[s&1]
            void* src = r->buf[(s - 1) & 1];
            void* dst = r->buf[s & 1];
            // int32 operands within 2^T * max|w| <= FP32_EXACT_MAX stay on the binary32 path
            const bool narrow = dt == BTAS_INT32 &&
                                (long)r->maxabs <= ((long)FP32_EXACT_MAX >> (r->T < 31 ? r->T : 31));
            GemmArgs a{r->n, r->n, r->n, src, r->ld, src, r->ld, src, r->ld, dst, r->ld,
                       st.d_changed + i, narrow ? d_zero : nullptr, nullptr, splitk_ws, splitk_bytes};
            e = launch_gemm(BTAS_MIN_PLUS, dt, a, -1, stream);
            launches++;
        }
        for (size_t i = 0; i < L.graphs.size(); ++i)
            if (L.ends_step[i]) {
                Request* r = L.graphs[i];
                r->planned += 1;
                r->next_tile = 0;
            }
        if (e == hipSuccess) e = hipMemcpyAsync(st.h_changed, st.d_changed, g * sizeof(int), hipMemcpyDeviceToHost, stream);
        return e;
    }

    // FIFO mode: the plain path, every squaring one GEMM launch.
    hipError_t enqueue_whole(Request* r) {
        hipError_t e = hipSuccess;
        int cur = 0;
        for (int t = 0; t < r->T && e == hipSuccess; ++t) {
            GemmArgs a{r->n, r->n, r->n, r->buf[cur], r->ld, r->buf[cur], r->ld,
                       r->buf[cur], r->ld, r->buf[cur ^ 1], r->ld, nullptr, nullptr, nullptr};
            e = launch_gemm(BTAS_MIN_PLUS, dt, a, -1, stream);
            cur ^= 1;
            launches++;
        }
        r->planned = r->T;
        return e;
    }

    void finish_locked(Request* r, double t, int steps) {
        r->state = DONE;
        r->done = t;
        r->T = steps;  // squarings executed; the result is in buf[steps & 1]
        active.erase(std::remove(active.begin(), active.end(), r), active.end());
    }

    // The distinct requests a launch names.
    static std::vector<Request*> launch_requests(const Launch& L) {
        std::vector<Request*> v(L.graphs);
        v.insert(v.end(), L.densified.begin(), L.densified.end());
        v.insert(v.end(), L.whole.begin(), L.whole.end());
        std::sort(v.begin(), v.end());
        v.erase(std::unique(v.begin(), v.end()), v.end());
        return v;
    }

    // Wait for the oldest launch and apply what its completion means.
    hipError_t retire_oldest() {
        Launch L = std::move(inflight.front());
        inflight.pop_front();
        hipError_t e = hipEventSynchronize(L.ev);
        const double t = now();
        free_events.push_back(L.ev);
        bool freed = false;
        {
            std::lock_guard<std::mutex> g(mu);
            if (e != hipSuccess) return e;
            for (Request* r : L.densified) {
                if (r->coo_off != SIZE_MAX) {
                    pool->release(r->coo_off, r->coo_bytes);
                    r->coo_off = SIZE_MAX;
                    freed = true;
                }
                if (r->T == 0) finish_locked(r, t, 0);
            }
            for (Request* r : L.whole) finish_locked(r, t, r->T);
            const int* chg = L.slot >= 0 ? staging[L.slot].h_changed : nullptr;
            for (size_t i = 0; i < L.graphs.size(); ++i) {
                Request* r = L.graphs[i];
                if (r->state != ACTIVE) continue;  // finished earlier: speculative work
                if (r->early) r->changed_acc |= chg[i];
                if (!L.ends_step[i]) continue;
                r->done_steps += 1;
                bool stop_early = false;
                if (r->early) {
                    stop_early = r->changed_acc == 0;
                    r->changed_acc = 0;
                }
                if (r->done_steps >= r->T || stop_early) finish_locked(r, t, r->done_steps);
            }
            // Drop this launch's references; a request the client released
            // while launches still named it is freed now.
            for (Request* r : launch_requests(L))
                if (--r->refs == 0 && r->released) {
                    if (r->off != SIZE_MAX) pool->release(r->off, r->bytes);
                    r->off = SIZE_MAX;
                    freed = true;
                    all.erase(r->id);
                }
            if (freed) admission_blocked = false;  // retry the head of the queue
            cv_done.notify_all();
            cv_work.notify_all();
        }
        if (freed) wake_peer();
        return hipSuccess;
    }

    void run() {
        (void)hipSetDevice(device);
        while (true) {
            std::vector<Request*> admitted, order;
            {
                std::unique_lock<std::mutex> lk(mu);
                auto has_plannable = [&] {
                    if (mode == BTAS_SERVE_FIFO) return false;
                    for (Request* r : active)
                        if (plannable(r)) return true;
                    return false;
                };
                cv_work.wait(lk, [&] {
                    return stop || !inflight.empty() || has_plannable() ||
                           (!pending.empty() && !admission_blocked);
                });
                if (stop) break;
                admit_locked(admitted);
                order = active;
            }
            const double it_start = now();
            hipError_t e = hipSuccess;
            for (Request* r : admitted)
                if (e == hipSuccess) e = densify(r);
            Launch L;
            L.densified = admitted;
            bool any = !admitted.empty();
            if (e == hipSuccess && mode == BTAS_SERVE_CONTINUOUS) {
                // A staging set is free once the launch that used it retired.
                if (inflight.size() >= (size_t)kDepth) e = retire_oldest();
                if (e == hipSuccess) {
                    L.slot = (int)(launches.load() % kDepth);
                    for (const Launch& o : inflight)
                        if (o.slot == L.slot) L.slot ^= 1;
                    e = plan_and_enqueue(L, order);
                    any = any || !L.graphs.empty();
                }
            } else if (e == hipSuccess && mode == BTAS_SERVE_FIFO) {
                for (Request* r : admitted)
                    if (e == hipSuccess && r->T > 0) {
                        e = enqueue_whole(r);
                        L.whole.push_back(r);
                    }
            }
            if (e == hipSuccess && any) {
                L.ev = get_event();
                if (L.ev == nullptr) e = hipErrorOutOfMemory;
                else e = hipEventRecord(L.ev, stream);
                if (e == hipSuccess) {
                    std::lock_guard<std::mutex> g(mu);
                    for (Request* r : launch_requests(L)) ++r->refs;
                    inflight.push_back(std::move(L));
                }
            }
            // Keep at most kDepth launches in flight; when nothing new can be
            // planned, wait for the oldest so that its requests advance.
            bool more = false;
            if (e == hipSuccess && !inflight.empty()) {
                std::lock_guard<std::mutex> g(mu);
                if (mode == BTAS_SERVE_CONTINUOUS)
                    for (Request* r : active)
                        if (plannable(r)) more = true;
            }
            if (e == hipSuccess && !inflight.empty() && (!more || inflight.size() >= (size_t)kDepth))
                e = retire_oldest();
            busy_s += now() - it_start;
            iterations++;
            if (e != hipSuccess) {
                (void)hipStreamSynchronize(stream);
                inflight.clear();
                std::lock_guard<std::mutex> g(mu);
                fail_all_locked(std::string("engine: HIP error ") + hipGetErrorString(e));
                break;
            }
        }
        // Drain before the stream and pool go away.
        while (!inflight.empty()) (void)retire_oldest();
    }

    void fail_all_locked(const std::string& msg) {
        error = msg;
        for (Request* r : active) r->state = FAILED;
        for (Request* r : pending) r->state = FAILED;
        active.clear();
        pending.clear();
        cv_done.notify_all();
    }
};

}  // namespace btas

using btas::Server;

// Continuous mode runs two lanes, each an engine thread with its own stream:
// requests of at most small_n vertices go to the small lane, the others to
// the large one.  Both share one memory pool (admission stays bounded by the
// budget) and one clock; a small request's squarings then run in short
// launches beside the large requests' instead of waiting for them.  A
// request id carries its lane in bit 0.
struct btas_server {
    btas::DevicePool pool;
    Server lanes[2];
    int nlanes = 1;
    int small_n = 0;
};

namespace {

Server* lane_of(btas_server_t srv, int64_t id, int64_t* local) {
    const int l = (int)(id & 1);
    if (id < 0 || l >= srv->nlanes) return nullptr;
    *local = id >> 1;
    return &srv->lanes[l];
}

void stop_lanes(btas_server_t srv) {
    for (int l = 0; l < srv->nlanes; ++l) {
        Server& s = srv->lanes[l];
        {
            std::lock_guard<std::mutex> g(s.mu);
            s.stop = true;
        }
        s.cv_work.notify_all();
    }
    for (int l = 0; l < srv->nlanes; ++l)
        if (srv->lanes[l].engine.joinable()) srv->lanes[l].engine.join();
    for (int l = 0; l < srv->nlanes; ++l) {
        Server& s = srv->lanes[l];
        (void)hipSetDevice(s.device);
        if (s.stream) {
            (void)hipStreamSynchronize(s.stream);
            (void)hipStreamDestroy(s.stream);
            s.stream = nullptr;
        }
        s.free_staging();
    }
}

}  // namespace

extern "C" {

btas_status_t btas_server_create(btas_server_t* out, int device, btas_dtype_t dt,
                                 size_t budget_bytes, int mode, double quantum_terms) {
    if (!out) return BTAS_ERR_INVALID_ARG;
    *out = nullptr;
    if (dt != BTAS_INT32 && dt != BTAS_FLOAT32) return BTAS_ERR_INVALID_ARG;
    if (mode != BTAS_SERVE_CONTINUOUS && mode != BTAS_SERVE_FIFO) return BTAS_ERR_INVALID_ARG;
    if (budget_bytes < 4096) return BTAS_ERR_INVALID_ARG;
    int count = 0;
    if (hipGetDeviceCount(&count) != hipSuccess || device < 0 || device >= count)
        return BTAS_ERR_INVALID_ARG;
    if (hipSetDevice(device) != hipSuccess) return BTAS_ERR_DEVICE;
    std::unique_ptr<btas_server> srv(new btas_server);
    if (!srv->pool.init(budget_bytes)) return BTAS_ERR_OOM;
    // The small lane (continuous mode only): graphs of up to 1024 vertices
    // by default (one squaring <= 2.1e9 ops); BTAS_SERVE_SMALL_N overrides,
    // 0 keeps a single lane.
    int small_n = 1024;
    if (const char* env = getenv("BTAS_SERVE_SMALL_N")) small_n = atoi(env);
    srv->small_n = mode == BTAS_SERVE_CONTINUOUS && small_n > 0 ? small_n : 0;
    srv->nlanes = srv->small_n > 0 ? 2 : 1;
    hipError_t e = hipSuccess;
    for (int l = 0; l < srv->nlanes; ++l) {
        Server& s = srv->lanes[l];
        s.device = device;
        s.dt = dt;
        s.mode = mode;
        if (quantum_terms > 0) s.quantum = quantum_terms;
        s.pool = &srv->pool;
        s.t0 = srv->lanes[0].t0;
        if (srv->nlanes == 2) s.peer = &srv->lanes[1 - l];
        if (const char* env = getenv("BTAS_SERVE_LAUNCH_TERMS"); env && l == 0 && srv->nlanes == 2)
            s.launch_terms = atof(env);
        e = hipStreamCreateWithFlags(&s.stream, hipStreamNonBlocking);
        if (e != hipSuccess) break;
        // Split-K workspace for the single-GEMM path (only products with fewer
        // than 256 output tiles split, i.e. n < 512: at most a few MiB).
        s.splitk_bytes = 16u << 20;
        if ((e = hipMalloc(&s.splitk_ws, s.splitk_bytes)) != hipSuccess) break;
        if ((e = hipMalloc((void**)&s.d_zero, 4)) != hipSuccess) break;
        if ((e = hipMemset(s.d_zero, 0, 4)) != hipSuccess) break;
    }
    if (e != hipSuccess) {
        stop_lanes(srv.get());
        return e == hipErrorOutOfMemory ? BTAS_ERR_OOM : BTAS_ERR_DEVICE;
    }
    for (int l = 0; l < srv->nlanes; ++l) {
        Server* p = &srv->lanes[l];
        p->engine = std::thread([p] { p->run(); });
    }
    *out = srv.release();
    return BTAS_OK;
}

btas_status_t btas_server_destroy(btas_server_t srv) {
    if (!srv) return BTAS_ERR_INVALID_ARG;
    stop_lanes(srv);
    delete srv;
    return BTAS_OK;
}

double btas_server_now(btas_server_t srv) { return srv ? srv->lanes[0].now() : -1.0; }

btas_status_t btas_server_submit(btas_server_t srv, int n, int nnz, const int32_t* rows,
                                 const int32_t* cols, const void* w, unsigned flags,
                                 double arrival, int64_t* id_out) {
    if (!srv || n < 0 || nnz < 0 || (nnz > 0 && (!rows || !cols || !w)) || !id_out)
        return BTAS_ERR_INVALID_ARG;
    if (flags & ~(unsigned)BTAS_APSP_EARLY_EXIT) return BTAS_ERR_INVALID_ARG;
    const int lane = srv->nlanes == 2 && n <= srv->small_n ? 1 : 0;
    Server& s = srv->lanes[lane];
    try {
    std::unique_ptr<btas::Request> r(new btas::Request);
    r->n = n;
    r->T = btas::steps_for(n);
    r->ld = (int)btas::align_up(std::max(n, 1), 4);
    r->nnz = nnz;
    r->early = flags & BTAS_APSP_EARLY_EXIT;
    r->rows.assign(rows, rows + nnz);
    r->cols.assign(cols, cols + nnz);
    r->w.resize(nnz);
    if (nnz) std::memcpy(r->w.data(), w, (size_t)nnz * 4);
    for (int e = 0; e < nnz; ++e)  // the densify kernel writes D[rows[e]][cols[e]]
        if (rows[e] < 0 || rows[e] >= n || cols[e] < 0 || cols[e] >= n) return BTAS_ERR_INVALID_ARG;
    int mx = 0;
    if (s.dt == BTAS_INT32) {
        for (int e = 0; e < nnz; ++e) {
            const int32_t v = (int32_t)r->w[e];
            if (v == BTAS_I32_INF) continue;
            if (v < -BTAS_I32_FINITE_MAX || v > BTAS_I32_FINITE_MAX) return BTAS_ERR_DOMAIN;
            mx = std::max(mx, v < 0 ? -v : v);
        }
    } else {
        for (int e = 0; e < nnz; ++e) {
            float v;
            std::memcpy(&v, &r->w[e], 4);
            if (v != v || v == -__builtin_inff()) return BTAS_ERR_DOMAIN;
        }
    }
    r->maxabs = mx;
    // Tile plan: padded-area model (64x64 tiles charged 15% more per element).
    r->tiles = btas::tile_plan(n, btas::model_shape(n));
    r->ntiles = (int)r->tiles.size();
    const size_t need = 2 * btas::align_up((size_t)n * r->ld * 4, 256) +
                        3 * btas::align_up((size_t)nnz * 4, 256);
    if (need > s.pool->size()) return BTAS_ERR_OOM;
    {
        std::lock_guard<std::mutex> g(s.mu);
        if (!s.error.empty()) return BTAS_ERR_DEVICE;
        r->id = s.next_id++;
        r->arrival = arrival >= 0 ? arrival : s.now();
        *id_out = r->id * 2 + lane;
        s.admission_blocked = false;
        s.pending.push_back(r.get());
        s.all[r->id] = std::move(r);
    }
    s.cv_work.notify_all();
    return BTAS_OK;
    } catch (...) {
        return BTAS_ERR_OOM;
    }
}

btas_status_t btas_server_wait(btas_server_t srv, int64_t id, double timeout_s, int* done) {
    if (!srv) return BTAS_ERR_INVALID_ARG;
    int64_t local = 0;
    Server* sp = lane_of(srv, id, &local);
    if (!sp) return BTAS_ERR_INVALID_ARG;
    Server& s = *sp;
    std::unique_lock<std::mutex> lk(s.mu);
    auto it = s.all.find(local);
    if (it == s.all.end() || it->second->released) return BTAS_ERR_INVALID_ARG;
    btas::Request* r = it->second.get();
    auto ready = [&] { return r->state == btas::DONE || r->state == btas::FAILED; };
    if (timeout_s < 0) s.cv_done.wait(lk, ready);
    else s.cv_done.wait_for(lk, std::chrono::duration<double>(timeout_s), ready);
    if (done) *done = r->state == btas::DONE;
    return r->state == btas::FAILED ? BTAS_ERR_DEVICE : BTAS_OK;
}

btas_status_t btas_server_result(btas_server_t srv, int64_t id, const void** D_dev, int* ldd,
                                 int* steps) {
    if (!srv) return BTAS_ERR_INVALID_ARG;
    int64_t local = 0;
    Server* sp = lane_of(srv, id, &local);
    if (!sp) return BTAS_ERR_INVALID_ARG;
    Server& s = *sp;
    std::lock_guard<std::mutex> g(s.mu);
    auto it = s.all.find(local);
    if (it == s.all.end() || it->second->released) return BTAS_ERR_INVALID_ARG;
    btas::Request* r = it->second.get();
    if (r->state != btas::DONE) return BTAS_ERR_INVALID_ARG;
    if (D_dev) *D_dev = r->buf[r->T & 1];
    if (ldd) *ldd = r->ld;
    if (steps) *steps = r->T;
    return BTAS_OK;
}

btas_status_t btas_server_copy_result(btas_server_t srv, int64_t id, void* D, int ldd) {
    if (!srv || !D) return BTAS_ERR_INVALID_ARG;
    int64_t local = 0;
    Server* sp = lane_of(srv, id, &local);
    if (!sp) return BTAS_ERR_INVALID_ARG;
    Server& s = *sp;
    const void* src;
    int n, ld;
    {
        std::lock_guard<std::mutex> g(s.mu);
        auto it = s.all.find(local);
        if (it == s.all.end() || it->second->released || it->second->state != btas::DONE)
            return BTAS_ERR_INVALID_ARG;
        btas::Request* r = it->second.get();
        src = r->buf[r->T & 1];
        n = r->n;
        ld = r->ld;
    }
    if (n == 0) return BTAS_OK;
    if (ldd < n) return BTAS_ERR_INVALID_ARG;
    (void)hipSetDevice(s.device);
    hipError_t e = hipMemcpy2D(D, (size_t)ldd * 4, src, (size_t)ld * 4, (size_t)n * 4, n,
                               hipMemcpyDeviceToDevice);
    return e == hipSuccess ? BTAS_OK : BTAS_ERR_DEVICE;
}

btas_status_t btas_server_times(btas_server_t srv, int64_t id, double* arrival, double* admitted,
                                double* done) {
    if (!srv) return BTAS_ERR_INVALID_ARG;
    int64_t local = 0;
    Server* sp = lane_of(srv, id, &local);
    if (!sp) return BTAS_ERR_INVALID_ARG;
    Server& s = *sp;
    std::lock_guard<std::mutex> g(s.mu);
    auto it = s.all.find(local);
    if (it == s.all.end() || it->second->released) return BTAS_ERR_INVALID_ARG;
    btas::Request* r = it->second.get();
    if (arrival) *arrival = r->arrival;
    if (admitted) *admitted = r->admitted;
    if (done) *done = r->done;
    return BTAS_OK;
}

btas_status_t btas_server_release(btas_server_t srv, int64_t id) {
    if (!srv) return BTAS_ERR_INVALID_ARG;
    int64_t local = 0;
    Server* sp = lane_of(srv, id, &local);
    if (!sp) return BTAS_ERR_INVALID_ARG;
    Server& s = *sp;
    {
        std::lock_guard<std::mutex> g(s.mu);
        auto it = s.all.find(local);
        if (it == s.all.end() || it->second->released) return BTAS_ERR_INVALID_ARG;
        btas::Request* r = it->second.get();
        if (r->state != btas::DONE && r->state != btas::FAILED) return BTAS_ERR_INVALID_ARG;
        if (r->refs > 0) {
            // a speculative squaring still runs in its buffers: the engine
            // frees them when that launch retires
            r->released = true;
            return BTAS_OK;
        }
        if (r->off != SIZE_MAX) s.pool->release(r->off, r->bytes);
        s.all.erase(it);
        s.admission_blocked = false;
    }
    s.cv_work.notify_all();
    s.wake_peer();
    return BTAS_OK;
}

btas_status_t btas_server_stats(btas_server_t srv, btas_server_stats_t* out) {
    if (!srv || !out) return BTAS_ERR_INVALID_ARG;
    *out = btas_server_stats_t{};
    bool ok = true;
    for (int l = 0; l < srv->nlanes; ++l) {
        Server& s = srv->lanes[l];
        std::lock_guard<std::mutex> g(s.mu);
        out->iterations += s.iterations.load();
        out->launches += s.launches.load();
        out->busy_seconds += s.busy_s;
        out->active += (int)s.active.size();
        out->pending += (int)s.pending.size();
        ok = ok && s.error.empty();
    }
    out->pool_bytes = srv->pool.size();
    out->pool_used_bytes = srv->pool.used();
    out->pool_peak_bytes = srv->pool.peak();
    return ok ? BTAS_OK : BTAS_ERR_DEVICE;
}

}  // extern "C"
