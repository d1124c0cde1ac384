// btas_apsp_squaring_batched: many independent APSP solves in one hipGraph.
//
// Plan (built once per distinct argument set, cached on the handle):
//  * every graph gets two padded internal buffers; D_0 = I (+) W is written
//    into the first, T(n) squarings alternate between them, the last one is
//    copied to the caller's D;
//  * graphs are ordered by decreasing T(n), then n, so the work list of
//    squaring t is a prefix of the graph order and its largest tiles come
//    first (longest-processing-time-first within each launch);
//  * each size bucket (half-octaves of n) uses the tile shape (128x128 or
//    64x64 output tiles) that the autotuner measured fastest for that bucket
//    on this device, timed on the plan's own buffers and work lists;
//  * init, every squaring launch and the copy-out are captured into one
//    hipGraph on the handle's auxiliary stream and replayed on the caller's
//    stream, so a batched solve is a single graph launch with no host
//    round trip between squarings.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <numeric>
#include <vector>

#include "batched.h"
#include "context.h"
#include "kernels.h"

namespace btas {

struct BatchPlan {
    uint64_t key = 0;
    int dt = 0;
    int count = 0;
    void* ws = nullptr;
    BatchGraph* d_graphs = nullptr;
    BatchItem* d_items = nullptr;
    BatchCopy* d_init = nullptr;
    BatchCopy* d_out = nullptr;
    int* d_maxabs = nullptr;
    int* d_block_job = nullptr;           // copy-pass workgroup -> graph job
    int init_blocks = 0, njobs = 0;
    std::vector<int> step_off, step_cnt;  // launch t (1-based) covers [off, off+cnt)
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    double terms = 0;                     // sum over graphs of T(n) * n^3
    int family = 0;                       // squaring kernel: 0 block, 1 wave, 2 direct
    int* d_changed = nullptr;             // early exit: changed[s * ngraphs + g] for squaring s
    BatchSmall* d_small = nullptr;        // graphs solved whole in LDS, one workgroup each
    int nsmall = 0;
    bool early = false;
    int nflags = 0;                       // early exit: entries of d_changed
    bool direct = false;                  // no captured graph: launched in order on every call
};

void destroy_batch_plan(BatchPlan* p) {
    if (!p) return;
    if (p->exec) (void)hipGraphExecDestroy(p->exec);
    if (p->graph) (void)hipGraphDestroy(p->graph);
    for (void* q : {(void*)p->d_graphs, (void*)p->d_items, (void*)p->d_init, (void*)p->d_out,
                    (void*)p->d_maxabs, (void*)p->d_block_job, (void*)p->d_changed,
                    (void*)p->d_small, p->ws})
        if (q) (void)hipFree(q);
    delete p;
}

namespace {

uint64_t mix(uint64_t h, uint64_t v) {
    h ^= v + 0x9E3779B97F4A7C15ull + (h << 6) + (h >> 2);
    return h;
}

int size_bucket(int n) {
    // half-octave buckets: 2*floor(log2 n) + (upper half of the octave)
    if (n <= 1) return 0;
    int lg = 31 - __builtin_clz((unsigned)n);
    const int half = (n - (1 << lg)) * 2 >= (1 << lg) ? 1 : 0;
    return 2 * lg + half;
}

size_t round_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

struct HostGraph {
    int idx;  // caller's index
    int n, T, ld;
};

void append_items(std::vector<BatchItem>& items, int graph_slot, int n, int shape, int step) {
    for (const TileRef& t : tile_plan(n, shape))
        items.push_back({graph_slot, t.m0, t.n0, t.kind, step, 0});
}

// An empty table still gets a small allocation (kernels take its address)
// but nothing is copied into it.
btas_status_t upload(btas_handle_t h, const char* fn, void** dst, const void* src, size_t bytes) {
    if (hipMalloc(dst, bytes > 0 ? bytes : 16) != hipSuccess)
        return fail(h, BTAS_ERR_OOM, "%s: cannot allocate %zu bytes of descriptors", fn, bytes);
    if (bytes == 0) return BTAS_OK;
    hipError_t e = hipMemcpy(*dst, src, bytes, hipMemcpyHostToDevice);
    return e == hipSuccess ? BTAS_OK : device_fail(h, fn, e);
}

// BTAS_BATCHED_TILE=128|64|mixed|w64|wmix forces a shape; -1 if unset.
int forced_shape() {
    const char* f = getenv("BTAS_BATCHED_TILE");
    if (!f || !*f) return -1;
    const char* names[NUM_SHAPES] = {"128", "64", "mixed", "w64", "wmix", "w64d"};
    for (int s = 0; s < NUM_SHAPES; ++s)
        if (std::strcmp(f, names[s]) == 0) return s;
    return -1;
}

// Time one squaring of a size bucket with every candidate shape, on the
// plan's (not yet initialised) buffers: the kernels' speed does not depend on
// the values, and the binary32 path is the one taken for in-range int32 data.
// The bucket's work list is repeated until the launch holds about as much
// work as the plan's own squaring launches (`target_terms`, capped at a
// millisecond of work), so a bucket that shares big launches is measured at
// the throughput it gets there, and a plan too small to fill the device is
// measured at its latency.  Repeated items write identical values.
btas_status_t time_bucket(btas_handle_t h, const char* fn, int dt, BatchPlan* p,
                          const std::vector<HostGraph>& hg, const std::vector<int>& slots,
                          double target_terms, BucketTiming* out) {
    hipError_t e = launch_clear_ints(p->d_maxabs, std::max((int)hg.size(), 1), h->aux_stream);
    if (e != hipSuccess) return device_fail(h, fn, e);
    double useful = 0;
    for (int g : slots) useful += (double)hg[g].n * hg[g].n * hg[g].n;
    std::vector<int> all_n(hg.size());
    for (size_t g = 0; g < hg.size(); ++g) all_n[g] = hg[g].n;
    double spt[NUM_SHAPES];
    for (int cand = 0; cand < NUM_SHAPES; ++cand) {
        std::vector<BatchItem> one;
        double padded = 0;
        for (int g : slots) {
            const size_t before = one.size();
            append_items(one, g, hg[g].n, cand, 1);
            for (size_t i = before; i < one.size(); ++i) padded += tile_area(one[i].kind) * hg[g].n;
        }
        int reps = 1;
        while (reps < 256 && padded * 2 * reps <= target_terms) reps *= 2;
        std::vector<BatchItem> its;
        its.reserve(one.size() * reps);
        for (int r = 0; r < reps; ++r) its.insert(its.end(), one.begin(), one.end());
        its = order_for_xcds(its, all_n);
        BatchItem* d_its = nullptr;
        btas_status_t st = upload(h, fn, (void**)&d_its, its.data(), sizeof(BatchItem) * its.size());
        if (st != BTAS_OK) return st;
        hipEvent_t e0, e1;
        (void)hipEventCreate(&e0);
        (void)hipEventCreate(&e1);
        float best = 1e30f;
        for (int rep_i = 0; rep_i < 3 && e == hipSuccess; ++rep_i) {
            (void)hipEventRecord(e0, h->aux_stream);
            e = launch_grouped_step(dt, p->d_graphs, d_its, (int)its.size(), p->d_maxabs, nullptr,
                                    h->aux_stream, shape_family(cand), dt == BTAS_INT32);
            (void)hipEventRecord(e1, h->aux_stream);
            if (e == hipSuccess) e = hipEventSynchronize(e1);
            float t = 0;
            (void)hipEventElapsedTime(&t, e0, e1);
            if (rep_i > 0) best = std::min(best, t);  // the first run warms up
        }
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        (void)hipFree(d_its);
        if (e != hipSuccess) return device_fail(h, fn, e);
        spt[cand] = best * 1e-3 / (useful * reps);
    }
    out->best[0] = SHAPE_128;
    out->best[1] = SHAPE_W64;
    out->best[2] = SHAPE_W64D;
    for (int cand = 0; cand < NUM_SHAPES; ++cand) {
        const int f = shape_family(cand);
        if (spt[cand] < spt[out->best[f]]) out->best[f] = cand;
    }
    for (int f = 0; f < NUM_FAMILIES; ++f) out->spt[f] = spt[out->best[f]];
    if (const char* lg = getenv("BTAS_LOG"); lg && lg[0] == '1')
        fprintf(stderr, "[btas] autotune dt=%d n<=%d graphs=%zu Tterm/s: 128 %.1f, 64 %.1f, mixed %.1f, "
                "w64 %.1f, wmix %.1f, w64d %.1f -> block %d, wave %d\n", dt, hg[slots.front()].n,
                slots.size(), 1e-12 / spt[0], 1e-12 / spt[1], 1e-12 / spt[2], 1e-12 / spt[3],
                1e-12 / spt[4], 1e-12 / spt[5], out->best[0], out->best[1]);
    return BTAS_OK;
}

// The launch sequence of a plan on stream s: (int32) max |w| per graph,
// then D_0 = I (+) W into the internal buffers, the squaring launches and the
// copy-out; with fork, the small graphs' whole solves on a second stream
// forked from s and joined back to it (so that, captured, they form a branch
// of the graph), else on s first.
hipError_t enqueue_batch(btas_handle_t h, const BatchPlan* p, hipStream_t s, bool fork) {
    hipError_t e = hipSuccess;
    const int ng = p->njobs, blocks = p->init_blocks;
    if (p->nsmall > 0) {
        if (fork) {
            e = hipEventRecord(h->fork_event, s);
            if (e == hipSuccess) e = hipStreamWaitEvent(h->fork_stream, h->fork_event, 0);
            if (e == hipSuccess)
                e = launch_batched_lds_solve(p->dt, p->d_small, p->nsmall, p->early, h->fork_stream);
            if (e == hipSuccess) e = hipEventRecord(h->join_event, h->fork_stream);
        } else {
            e = launch_batched_lds_solve(p->dt, p->d_small, p->nsmall, p->early, s);
        }
    }
    // int32: max |w| per graph first, so that graphs in the binary32-exact
    // range are stored (and squared) as binary32 with no per-element
    // conversions in the squarings.
    const bool i32 = p->dt == BTAS_INT32;
    if (e == hipSuccess && i32) e = launch_clear_ints(p->d_maxabs, std::max(ng, 1), s);
    if (e == hipSuccess && i32)
        e = launch_grouped_maxabs(p->d_graphs, p->d_init, ng, blocks, p->d_maxabs, s, p->d_block_job);
    if (e == hipSuccess)
        e = launch_grouped_init(p->dt, p->d_graphs, p->d_init, ng, blocks, i32 ? p->d_maxabs : nullptr,
                                s, i32, p->d_block_job);
    // early exit: per squaring and graph, whether it changed D; an item
    // whose graph did not change at the previous squaring is skipped
    if (e == hipSuccess && p->nflags > 0) e = launch_clear_ints(p->d_changed, p->nflags, s);
    for (size_t t = 0; t < p->step_off.size() && e == hipSuccess; ++t)
        e = launch_grouped_step(p->dt, p->d_graphs, p->d_items + p->step_off[t], p->step_cnt[t],
                                i32 ? p->d_maxabs : nullptr, p->d_changed, s, p->family, i32,
                                p->nflags > 0 ? ng : 0);
    if (e == hipSuccess)
        e = launch_grouped_copy_out(p->d_graphs, p->d_out, ng, blocks, s, i32 ? p->d_maxabs : nullptr,
                                    p->d_block_job);
    if (e == hipSuccess && fork && p->nsmall > 0) e = hipStreamWaitEvent(s, h->join_event, 0);
    return e;
}

// Run a built plan on the handle's stream: replay its captured graph, or
// (BTAS_BATCH_GRAPH=0 when it was built) issue its launches in order.
hipError_t run_batch(btas_handle_t h, const BatchPlan* p) {
    return p->direct ? enqueue_batch(h, p, h->stream, false) : hipGraphLaunch(p->exec, h->stream);
}

}  // namespace
}  // namespace btas

using namespace btas;

extern "C" btas_status_t btas_apsp_squaring_batched(btas_handle_t h, btas_dtype_t dt, int count,
                                                    const int* n, const void* const* W,
                                                    const int* ldw, void* const* D,
                                                    const int* ldd, unsigned flags) {
    const char* fn = "btas_apsp_squaring_batched";
    if (!h) return BTAS_ERR_INVALID_ARG;
    if (btas_status_t l = begin_call(h, fn); l != BTAS_OK) return l;
    if (dt != BTAS_INT32 && dt != BTAS_FLOAT32)
        return fail(h, BTAS_ERR_INVALID_ARG, "%s: argument 2 (dtype=%d) unknown", fn, (int)dt);
    if (count < 0) return fail(h, BTAS_ERR_INVALID_ARG, "%s: argument 3 (count=%d) < 0", fn, count);
    if (flags & ~BTAS_APSP_EARLY_EXIT)
        return fail(h, BTAS_ERR_UNSUPPORTED, "%s: flags=0x%x; only BTAS_APSP_EARLY_EXIT", fn, flags);
    const bool early = flags & BTAS_APSP_EARLY_EXIT;
    if (count == 0) return BTAS_OK;
    if (!n || !W || !ldw || !D || !ldd)
        return fail(h, BTAS_ERR_INVALID_ARG, "%s: a host array argument is null", fn);
    uint64_t key = mix(0x42ull, (uint64_t)dt);
    key = mix(key, early ? 1u : 0u);
    key = mix(key, (uint64_t)count);
    for (int i = 0; i < count; ++i) {
        key = mix(key, (uint64_t)n[i]);
        key = mix(key, ((uint64_t)(uint32_t)ldw[i] << 32) | (uint32_t)ldd[i]);
        key = mix(key, (uint64_t)(uintptr_t)W[i]);
        key = mix(key, (uint64_t)(uintptr_t)D[i]);
    }
    if (h->batch_plan && h->batch_plan->key == key) {
        // the arguments of the current plan (every argument is in the key),
        // checked when it was built: replay it
        DeviceGuard g(h->device);
        const hipError_t e = run_batch(h, h->batch_plan.get());
        return e == hipSuccess ? BTAS_OK : device_fail(h, fn, e);
    }
    std::vector<Span> dspans;
    for (int i = 0; i < count; ++i) {
        if (n[i] < 0) return fail(h, BTAS_ERR_INVALID_ARG, "%s: n[%d]=%d < 0", fn, i, n[i]);
        if (ldw[i] < std::max(1, n[i]))
            return fail(h, BTAS_ERR_INVALID_ARG, "%s: ldw[%d]=%d < max(1,n)", fn, i, ldw[i]);
        if (ldd[i] < std::max(1, n[i]))
            return fail(h, BTAS_ERR_INVALID_ARG, "%s: ldd[%d]=%d < max(1,n)", fn, i, ldd[i]);
        if (n[i] > 0 && (!W[i] || !D[i]))
            return fail(h, BTAS_ERR_INVALID_ARG, "%s: W[%d] or D[%d] is null", fn, i, i);
        if (n[i] > 0) dspans.push_back(mat_span(D[i], n[i], n[i], ldd[i]));
    }
    // Outputs must not overlap each other (each W is read before any D is written).
    std::sort(dspans.begin(), dspans.end(), [](const Span& a, const Span& b) { return a.lo < b.lo; });
    for (size_t i = 1; i < dspans.size(); ++i)
        if (dspans[i].lo < dspans[i - 1].hi)
            return fail(h, BTAS_ERR_ALIAS, "%s: two output matrices overlap", fn);

    // One or two graphs small enough for the automatic single-launch solve:
    // that solve per graph is faster than a batched plan's dozen launches
    // (n=256: 79 us against 233 us) and gives the same bits (early exit
    // included); no plan is built.
    {
        const char* sl_env = getenv("BTAS_SINGLE_LAUNCH");
        bool direct = count <= BATCH_DIRECT_MAX_COUNT && !(sl_env && sl_env[0] == '0');
        for (int i = 0; i < count && direct; ++i) direct = n[i] <= AUTO_SINGLE_LAUNCH_N;
        // Solved one after the other, so an earlier output must not overlap
        // a later input (the batched contract reads every W first).
        for (int i = 0; i < count && direct; ++i)
            for (int j = i + 1; j < count && direct; ++j)
                if (n[i] > 0 && n[j] > 0)
                    direct = !overlap(mat_span(D[i], n[i], n[i], ldd[i]), mat_span(W[j], n[j], n[j], ldw[j]));
        if (direct) {
            for (int i = 0; i < count; ++i) {
                if (n[i] == 0) continue;
                const btas_status_t st =
                    btas_apsp_squaring(h, dt, n[i], W[i], ldw[i], D[i], ldd[i], flags, nullptr);
                if (st != BTAS_OK) return st;
            }
            return BTAS_OK;
        }
    }

    DeviceGuard guard(h->device);

    hipError_t e = hipSuccess;
    if (!h->aux_stream) {
        e = hipStreamCreateWithFlags(&h->aux_stream, hipStreamNonBlocking);
        if (e != hipSuccess) return device_fail(h, fn, e);
    }

    BatchPlan* plan = h->batch_plan.get();
    if (!plan || plan->key != key) {
        if (plan) {
            // The previous plan's graph may still run on the caller's stream.
            e = hipStreamSynchronize(h->stream);
            if (e != hipSuccess) return device_fail(h, fn, e);
        }
        h->batch_plan.reset();
        std::unique_ptr<BatchPlan, BatchPlanDeleter> p(new BatchPlan);
        p->key = key;
        p->dt = dt;
        p->count = count;
        // With BTAS_BATCH_LDS=1, graphs of at most BATCH_LDS_MAX_N vertices
        // are solved whole in LDS by one workgroup each, on a branch of the
        // captured graph (same bits; measured slower on the 4096-graph
        // workload: those 1024-thread workgroups, bound by LDS bandwidth,
        // take compute units from the squaring launches, which handle the
        // small graphs' few tiles cheaply).  The rest, ordered by decreasing
        // T, then decreasing n; n == 0 dropped.
        const char* lds_env = getenv("BTAS_BATCH_LDS");
        const bool lds_small = lds_env && lds_env[0] == '1';
        std::vector<HostGraph> hg;
        std::vector<BatchSmall> small;
        for (int i = 0; i < count; ++i) {
            if (n[i] <= 0) continue;
            if (lds_small && n[i] <= BATCH_LDS_MAX_N) {
                small.push_back({n[i], apsp_steps(n[i]), (long)ldw[i], (long)ldd[i], W[i], D[i]});
                p->terms += (double)apsp_steps(n[i]) * n[i] * (double)n[i] * n[i];
            } else {
                hg.push_back({i, n[i], apsp_steps(n[i]), padded_edge(n[i])});
            }
        }
        // larger graphs first: their workgroups start before the short ones
        std::stable_sort(small.begin(), small.end(),
                         [](const BatchSmall& a, const BatchSmall& b) { return a.n > b.n; });
        p->nsmall = (int)small.size();
        std::stable_sort(hg.begin(), hg.end(), [](const HostGraph& a, const HostGraph& b) {
            return a.T != b.T ? a.T > b.T : a.n > b.n;
        });
        const int ng = (int)hg.size();
        // Workspace: two 256-byte aligned np x np buffers per graph (np = n
        // rounded up to 64, the padding filled with the absent value at init),
        // so that every shape, including the direct one, can run on them.
        std::vector<size_t> off(ng);
        size_t total = 0;
        for (int g = 0; g < ng; ++g) {
            off[g] = total;
            total += 2 * round_up((size_t)hg[g].ld * hg[g].ld * 4, 256);
        }
        if (total > 0 && hipMalloc(&p->ws, total) != hipSuccess)
            return fail(h, BTAS_ERR_OOM, "%s: cannot allocate the %zu-byte batch workspace", fn, total);
        std::vector<BatchGraph> graphs(ng);
        for (int g = 0; g < ng; ++g) {
            const size_t half = round_up((size_t)hg[g].ld * hg[g].ld * 4, 256);
            char* base = (char*)p->ws + off[g];
            graphs[g] = {{base, base + half}, hg[g].n, hg[g].ld, hg[g].T, 0, hg[g].ld};
            p->terms += (double)hg[g].T * hg[g].n * (double)hg[g].n * hg[g].n;
        }
        btas_status_t st = upload(h, fn, (void**)&p->d_graphs, graphs.data(), sizeof(BatchGraph) * ng);
        if (st != BTAS_OK) return st;
        if (hipMalloc((void**)&p->d_maxabs, sizeof(int) * std::max(ng, 1)) != hipSuccess)
            return fail(h, BTAS_ERR_OOM, "%s: cannot allocate flags", fn);

        // Tile shape per size bucket: forced, modelled, or measured.
        std::map<int, std::vector<int>> buckets;  // bucket -> graph slots
        for (int g = 0; g < ng; ++g)
            if (hg[g].T > 0) buckets[size_bucket(hg[g].n)].push_back(g);
        std::map<int, int> kind_of_bucket;
        int family = 2;
        const int forced = forced_shape();
        const char* tune_env = getenv("BTAS_AUTOTUNE");
        const bool tune = !(tune_env && tune_env[0] == '0');
        if (forced >= 0) {
            family = shape_family(forced);
            for (auto& kv : buckets) kind_of_bucket[kv.first] = forced;
        } else if (!tune) {
            for (auto& kv : buckets) kind_of_bucket[kv.first] = SHAPE_W64D;
        } else {
            // Measure the buckets this handle has not timed yet, then take the
            // family with the smaller predicted time for the whole plan.
            double cost[NUM_FAMILIES] = {0, 0, 0};
            double step1 = 0;  // useful terms of the first squaring launch
            for (int g = 0; g < ng; ++g)
                if (hg[g].T > 0) step1 += (double)hg[g].n * hg[g].n * hg[g].n;
            const double target = std::min(step1, 2e10);
            const int scale = (int)std::floor(std::log2(std::max(target, 1.0)));
            for (auto& kv : buckets) {
                const auto key = std::make_tuple((int)dt, kv.first, scale);
                auto it = h->tile_timing.find(key);
                if (it == h->tile_timing.end()) {
                    BucketTiming bt;
                    st = time_bucket(h, fn, dt, p.get(), hg, kv.second, target, &bt);
                    if (st != BTAS_OK) return st;
                    it = h->tile_timing.emplace(key, bt).first;
                }
                double terms = 0;
                for (int g : kv.second) terms += (double)hg[g].T * hg[g].n * (double)hg[g].n * hg[g].n;
                for (int f = 0; f < NUM_FAMILIES; ++f) cost[f] += terms * it->second.spt[f];
            }
            family = 0;
            for (int f = 1; f < NUM_FAMILIES; ++f)
                if (cost[f] < cost[family]) family = f;
            for (auto& kv : buckets)
                kind_of_bucket[kv.first] =
                    h->tile_timing[std::make_tuple((int)dt, kv.first, scale)].best[family];
            if (const char* lg = getenv("BTAS_LOG"); lg && lg[0] == '1')
                fprintf(stderr, "[btas] batched plan: predicted %.3f ms with block tiles, %.3f ms with "
                        "wave tiles, %.3f ms with direct tiles -> family %d\n", cost[0] * 1e3,
                        cost[1] * 1e3, cost[2] * 1e3, family);
        }
        p->family = family;
        for (auto& kv : kind_of_bucket) h->tile_choice[{(int)dt, kv.first}] = kv.second;

        // Work lists: launch t holds the tiles of every graph with T >= t.
        std::vector<BatchItem> items;
        std::vector<int> graph_n(ng);
        for (int g = 0; g < ng; ++g) graph_n[g] = hg[g].n;
        const char* xo = getenv("BTAS_XCD_ORDER");
        const bool xcd_order = !(xo && xo[0] == '0');
        const int Tmax = ng > 0 ? hg[0].T : 0;
        for (int t = 1; t <= Tmax; ++t) {
            std::vector<BatchItem> step;
            for (int g = 0; g < ng && hg[g].T >= t; ++g)
                append_items(step, g, hg[g].n, kind_of_bucket[size_bucket(hg[g].n)], t);
            if (xcd_order) step = order_for_xcds(step, graph_n);
            p->step_off.push_back((int)items.size());
            items.insert(items.end(), step.begin(), step.end());
            p->step_cnt.push_back((int)step.size());
        }
        st = upload(h, fn, (void**)&p->d_items, items.data(), sizeof(BatchItem) * items.size());
        if (st != BTAS_OK) return st;
        const int nflags = early ? ng * (Tmax + 1) : 0;
        if (nflags > 0 && hipMalloc((void**)&p->d_changed, sizeof(int) * nflags) != hipSuccess)
            return fail(h, BTAS_ERR_OOM, "%s: cannot allocate the change flags", fn);
        // Copy jobs (caller order is irrelevant: one job per graph).
        std::vector<BatchCopy> init(ng), out(ng);
        int blocks = 0;
        for (int g = 0; g < ng; ++g) {
            const int nb = copy_blocks_for(hg[g].n);
            init[g] = {g, blocks, nb, 0, (long)ldw[hg[g].idx], W[hg[g].idx]};
            out[g] = {g, blocks, nb, 0, (long)ldd[hg[g].idx], D[hg[g].idx]};
            blocks += nb;
        }
        p->init_blocks = blocks;
        p->njobs = ng;
        std::vector<int> block_job(std::max(blocks, 1));
        for (int g = 0; g < ng; ++g)
            for (int b = 0; b < init[g].nblocks; ++b) block_job[init[g].first_block + b] = g;
        st = upload(h, fn, (void**)&p->d_block_job, block_job.data(), sizeof(int) * block_job.size());
        if (st != BTAS_OK) return st;
        st = upload(h, fn, (void**)&p->d_init, init.data(), sizeof(BatchCopy) * ng);
        if (st == BTAS_OK) st = upload(h, fn, (void**)&p->d_out, out.data(), sizeof(BatchCopy) * ng);
        if (st == BTAS_OK && p->nsmall > 0)
            st = upload(h, fn, (void**)&p->d_small, small.data(), sizeof(BatchSmall) * p->nsmall);
        if (st != BTAS_OK) return st;
        if (p->nsmall > 0 && !h->fork_stream) {
            e = hipStreamCreateWithFlags(&h->fork_stream, hipStreamNonBlocking);
            if (e == hipSuccess) e = hipEventCreateWithFlags(&h->fork_event, hipEventDisableTiming);
            if (e == hipSuccess) e = hipEventCreateWithFlags(&h->join_event, hipEventDisableTiming);
            if (e != hipSuccess) return device_fail(h, fn, e);
        }

        p->early = early;
        p->nflags = nflags;
        // Capture the whole solve (the small graphs' solves as a branch of
        // the captured graph), unless BTAS_BATCH_GRAPH=0 asks for the same
        // launches issued in order on every call (for tools that cannot
        // follow graph launches, such as counter collection).
        const char* graph_env = getenv("BTAS_BATCH_GRAPH");
        p->direct = graph_env && graph_env[0] == '0';
        if (!p->direct) {
            e = hipStreamBeginCapture(h->aux_stream, hipStreamCaptureModeThreadLocal);
            if (e != hipSuccess) return device_fail(h, fn, e);
            e = enqueue_batch(h, p.get(), h->aux_stream, true);
            hipGraph_t graph = nullptr;
            hipError_t e2 = hipStreamEndCapture(h->aux_stream, &graph);
            if (e != hipSuccess || e2 != hipSuccess) {
                if (graph) (void)hipGraphDestroy(graph);
                return device_fail(h, fn, e != hipSuccess ? e : e2);
            }
            p->graph = graph;
            e = hipGraphInstantiate(&p->exec, graph, nullptr, nullptr, 0);
            if (e != hipSuccess) return device_fail(h, fn, e);
        }
        h->batch_plan = std::move(p);
        plan = h->batch_plan.get();
    }
    e = run_batch(h, plan);
    return e == hipSuccess ? BTAS_OK : device_fail(h, fn, e);
}

extern "C" btas_status_t btas_batched_plan_info(btas_handle_t h, int* num_launches,
                                                double* total_terms) {
    if (!h) return BTAS_ERR_INVALID_ARG;
    const BatchPlan* p = h->batch_plan.get();
    if (!p) return fail(h, BTAS_ERR_INVALID_ARG, "btas_batched_plan_info: no batched plan yet");
    if (num_launches)
        *num_launches = (int)p->step_cnt.size() + (p->dt == BTAS_INT32 ? 4 : 2) + (p->nsmall > 0 ? 1 : 0);
    if (total_terms) *total_terms = p->terms;
    return BTAS_OK;
}

extern "C" int btas_batched_tile_choice(btas_handle_t h, btas_dtype_t dt, int n) {
    if (!h) return -1;
    auto it = h->tile_choice.find({(int)dt, size_bucket(n)});
    return it == h->tile_choice.end() ? -1 : it->second;
}

// ------------------------------------------------- batched Floyd-Warshall ---
namespace btas {

struct FwBatchPlan {
    uint64_t key = 0;
    int dt = 0;
    FwGraph* d_graphs = nullptr;
    FwItem* d_items = nullptr;
    struct Launch {
        int phase, kb, off, cnt;
    };
    std::vector<Launch> launches;
    bool vec = false;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

void destroy_fw_batch_plan(FwBatchPlan* p) {
    if (!p) return;
    if (p->exec) (void)hipGraphExecDestroy(p->exec);
    if (p->graph) (void)hipGraphDestroy(p->graph);
    if (p->d_graphs) (void)hipFree(p->d_graphs);
    if (p->d_items) (void)hipFree(p->d_items);
    delete p;
}

}  // namespace btas

extern "C" btas_status_t btas_apsp_floyd_warshall_batched(btas_handle_t h, btas_dtype_t dt, int count,
                                                         const int* n, const void* const* W,
                                                         const int* ldw, void* const* D,
                                                         const int* ldd, unsigned flags) {
    const char* fn = "btas_apsp_floyd_warshall_batched";
    if (!h) return BTAS_ERR_INVALID_ARG;
    if (btas_status_t l = begin_call(h, fn); l != BTAS_OK) return l;
    if (dt != BTAS_INT32 && dt != BTAS_FLOAT32)
        return fail(h, BTAS_ERR_INVALID_ARG, "%s: argument 2 (dtype=%d) unknown", fn, (int)dt);
    if (count < 0) return fail(h, BTAS_ERR_INVALID_ARG, "%s: argument 3 (count=%d) < 0", fn, count);
    if (flags != 0) return fail(h, BTAS_ERR_UNSUPPORTED, "%s: flags=0x%x; none are defined", fn, flags);
    if (count == 0) return BTAS_OK;
    if (!n || !W || !ldw || !D || !ldd)
        return fail(h, BTAS_ERR_INVALID_ARG, "%s: a host array argument is null", fn);
    uint64_t key = mix(0x46ull, (uint64_t)dt);
    key = mix(key, (uint64_t)count);
    for (int i = 0; i < count; ++i) {
        key = mix(key, (uint64_t)n[i]);
        key = mix(key, ((uint64_t)(uint32_t)ldw[i] << 32) | (uint32_t)ldd[i]);
        key = mix(key, (uint64_t)(uintptr_t)W[i]);
        key = mix(key, (uint64_t)(uintptr_t)D[i]);
    }
    if (h->fw_batch_plan && h->fw_batch_plan->key == key) {  // validated when it was built
        DeviceGuard g(h->device);
        const hipError_t e = hipGraphLaunch(h->fw_batch_plan->exec, h->stream);
        return e == hipSuccess ? BTAS_OK : device_fail(h, fn, e);
    }
    // D[i] may be W[i] with the same leading dimension (in place); no output
    // may touch another graph's input or output, nor its own input otherwise
    // (the first launch reads every W while it writes every D).
    struct Tagged {
        Span s;
        int graph;
        bool out;
    };
    std::vector<Tagged> spans;
    for (int i = 0; i < count; ++i) {
        if (n[i] < 0) return fail(h, BTAS_ERR_INVALID_ARG, "%s: n[%d]=%d < 0", fn, i, n[i]);
        if (ldw[i] < std::max(1, n[i]))
            return fail(h, BTAS_ERR_INVALID_ARG, "%s: ldw[%d]=%d < max(1,n)", fn, i, ldw[i]);
        if (ldd[i] < std::max(1, n[i]))
            return fail(h, BTAS_ERR_INVALID_ARG, "%s: ldd[%d]=%d < max(1,n)", fn, i, ldd[i]);
        if (n[i] == 0) continue;
        if (!W[i] || !D[i]) return fail(h, BTAS_ERR_INVALID_ARG, "%s: W[%d] or D[%d] is null", fn, i, i);
        const bool in_place = W[i] == D[i] && ldw[i] == ldd[i];
        spans.push_back({mat_span(D[i], n[i], n[i], ldd[i]), i, true});
        if (!in_place) spans.push_back({mat_span(W[i], n[i], n[i], ldw[i]), i, false});
    }
    std::sort(spans.begin(), spans.end(), [](const Tagged& a, const Tagged& b) { return a.s.lo < b.s.lo; });
    for (size_t i = 0; i < spans.size(); ++i)  // every overlapping pair that involves an output
        for (size_t j = i + 1; j < spans.size() && spans[j].s.lo < spans[i].s.hi; ++j)
            if (spans[i].out || spans[j].out)
                return fail(h, BTAS_ERR_ALIAS, "%s: an output overlaps another matrix (graphs %d, %d)", fn,
                            spans[i].graph, spans[j].graph);

    DeviceGuard guard(h->device);
    hipError_t e = hipSuccess;
    if (!h->aux_stream) {
        e = hipStreamCreateWithFlags(&h->aux_stream, hipStreamNonBlocking);
        if (e != hipSuccess) return device_fail(h, fn, e);
    }
    FwBatchPlan* plan = h->fw_batch_plan.get();
    if (!plan || plan->key != key) {
        if (plan) {
            e = hipStreamSynchronize(h->stream);
            if (e != hipSuccess) return device_fail(h, fn, e);
        }
        h->fw_batch_plan.reset();
        std::unique_ptr<FwBatchPlan, FwBatchPlanDeleter> p(new FwBatchPlan);
        p->key = key;
        p->dt = dt;
        const int B = fw_block_size();
        std::vector<FwGraph> graphs;
        bool vec = true;
        int nbmax = 0;
        for (int i = 0; i < count; ++i) {
            if (n[i] == 0) continue;
            const int nb = (n[i] + B - 1) / B;
            graphs.push_back({W[i], (long)ldw[i], D[i], (long)ldd[i], n[i], nb});
            vec = vec && ldd[i] % 4 == 0 && (uintptr_t)D[i] % 16 == 0;
            nbmax = std::max(nbmax, nb);
        }
        p->vec = vec;
        // Work lists: init; then per pair of pivot blocks (kb, kb+1) every
        // graph that has both runs the single-graph pair schedule (phases 1-2
        // of kb, kb's strip update of row/column kb+1, phases 1-2 of kb+1,
        // the k=128 update of the tiles outside both, kb+1's deferred strip
        // update of row/column kb); a graph whose last block is kb runs the
        // three plain phases.  Graphs are independent, so each launch takes
        // one step of every graph that has it.
        std::vector<FwItem> items;
        auto add_launch = [&](int phase, int kb, const std::vector<FwItem>& its) {
            if (its.empty()) return;
            p->launches.push_back({phase, kb, (int)items.size(), (int)its.size()});
            items.insert(items.end(), its.begin(), its.end());
        };
        std::vector<FwItem> its;
        for (int g = 0; g < (int)graphs.size(); ++g)
            for (int r = 0; r < graphs[g].nb; ++r) its.push_back({g, r});
        add_launch(FWB_INIT, 0, its);
        for (int kb = 0; kb < nbmax; kb += 2) {
            std::vector<FwItem> p1a, p2a, next, last, p1b, p2b, pair, prev;
            for (int g = 0; g < (int)graphs.size(); ++g) {
                const int nb = graphs[g].nb;
                if (nb <= kb) continue;
                p1a.push_back({g, 0});
                for (int b = 0; b < 2 * (nb - 1); ++b) p2a.push_back({g, b});
                if (nb == kb + 1) {  // last block, unpaired
                    for (int t = 0; t < (nb - 1) * (nb - 1); ++t) last.push_back({g, t});
                    continue;
                }
                for (int t = 0; t < 2 * nb - 3; ++t) next.push_back({g, t});
                p1b.push_back({g, 0});
                for (int b = 0; b < 2 * (nb - 1); ++b) p2b.push_back({g, b});
                const int nb2 = (graphs[g].n + 2 * B - 1) / (2 * B);
                for (int t = 0; t < (nb2 - 1) * (nb2 - 1); ++t) pair.push_back({g, t});
                for (int t = 0; t < 2 * nb - 3; ++t) prev.push_back({g, t});
            }
            add_launch(FWB_PHASE1, kb, p1a);
            add_launch(FWB_PHASE2, kb, p2a);
            add_launch(FWB_PHASE3, kb, last);
            add_launch(FWB_STRIP_NEXT, kb, next);
            add_launch(FWB_PHASE1, kb + 1, p1b);
            add_launch(FWB_PHASE2, kb + 1, p2b);
            add_launch(FWB_PAIR, kb, pair);
            add_launch(FWB_STRIP_PREV, kb + 1, prev);
        }
        btas_status_t st = upload(h, fn, (void**)&p->d_graphs, graphs.data(), sizeof(FwGraph) * graphs.size());
        if (st == BTAS_OK) st = upload(h, fn, (void**)&p->d_items, items.data(), sizeof(FwItem) * items.size());
        if (st != BTAS_OK) return st;
        e = hipStreamBeginCapture(h->aux_stream, hipStreamCaptureModeThreadLocal);
        if (e != hipSuccess) return device_fail(h, fn, e);
        for (const auto& L : p->launches) {
            e = launch_fw_batched(dt, L.phase, p->d_graphs, p->d_items + L.off, L.cnt, L.kb, p->vec,
                                  h->aux_stream);
            if (e != hipSuccess) break;
        }
        hipGraph_t graph = nullptr;
        const hipError_t e2 = hipStreamEndCapture(h->aux_stream, &graph);
        if (e != hipSuccess || e2 != hipSuccess) {
            if (graph) (void)hipGraphDestroy(graph);
            return device_fail(h, fn, e != hipSuccess ? e : e2);
        }
        p->graph = graph;
        e = hipGraphInstantiate(&p->exec, graph, nullptr, nullptr, 0);
        if (e != hipSuccess) return device_fail(h, fn, e);
        h->fw_batch_plan = std::move(p);
        plan = h->fw_batch_plan.get();
    }
    e = hipGraphLaunch(plan->exec, h->stream);
    return e == hipSuccess ? BTAS_OK : device_fail(h, fn, e);
}
