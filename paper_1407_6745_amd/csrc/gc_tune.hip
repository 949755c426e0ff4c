// gc_tune.hip - autotuning.  The knobs of gc_tuning (degree-bin thresholds,
// lanes per vertex, workgroups per CU, graph order of the batch, ...) only
// change how the work is scheduled, never a color: the autotuner times the
// method under candidate settings on the caller's own input, checks that
// every candidate produced the same colors (a 64-bit checksum of the
// (vertex, color) pairs and of the per-graph statistics), and keeps the
// fastest in the context.
#include "gc_internal.h"

#include <vector>

__global__ void k_checksum(int64_t n, const int32_t *__restrict__ a, unsigned long long *out) {
    unsigned long long acc = 0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        acc += gc_mix64(((uint64_t)i << 32) ^ (uint32_t)a[i]);
    acc = wave_sum_u64(acc);
    if (__lane_id() == 0 && acc) atomicAdd(out, acc);
}

// Sum over i of mix64(i << 32 ^ a[i]) for the two arrays (either may be empty).
static gc_status checksum2(gc_ctx *ctx, const int32_t *a, int64_t na, const int32_t *b, int64_t nb, hipStream_t s,
                           uint64_t *out) {
    GC_HIP(hipMemsetAsync(ctx->scal + S_SUM, 0, 8, s));
    if (na > 0) {
        k_checksum<<<gc_grid(ctx, na, 256), 256, 0, s>>>(na, a, ctx->scal + S_SUM);
        GC_LAUNCHED();
    }
    if (nb > 0) {
        k_checksum<<<gc_grid(ctx, nb, 256), 256, 0, s>>>(nb, b, ctx->scal + S_SUM);
        GC_LAUNCHED();
    }
    gc_status st = gc_sync_scalars(ctx, s);
    if (st) return st;
    *out = ctx->hscal[S_SUM];
    return GC_OK;
}

namespace {

// Event pair timing one run of a callable on the stream.
struct Timer {
    hipEvent_t e0 = nullptr, e1 = nullptr;
    ~Timer() {
        if (e0) (void)hipEventDestroy(e0);
        if (e1) (void)hipEventDestroy(e1);
    }
};

}  // namespace

// Applies t (validated) and runs `run`; *ms = elapsed, *sum = checksum of the outputs.
template <class Run>
static gc_status try_tuning(gc_ctx *ctx, const gc_tuning &t, hipStream_t s, Timer &tm, Run &&run, const int32_t *a,
                            int64_t na, const int32_t *b, int64_t nb, double *ms, uint64_t *sum) {
    gc_status st = gc_ctx_set_tuning(ctx, &t);
    if (st) return st;
    GC_HIP(hipEventRecord(tm.e0, s));
    st = run();
    if (st) return st;
    GC_HIP(hipEventRecord(tm.e1, s));
    GC_HIP(hipEventSynchronize(tm.e1));
    float f = 0.f;
    GC_HIP(hipEventElapsedTime(&f, tm.e0, tm.e1));
    *ms = f;
    return checksum2(ctx, a, na, b, nb, s, sum);
}

static gc_status gc_autotune_impl(gc_ctx *ctx, const gc_csr *g, int32_t select, int32_t X, int32_t perm, int32_t passes,
                                 uint64_t seed, int32_t *colors, gc_tuning *best, double *best_ms, void *stream) {
    gc_status status = gc_check_graph_args(ctx, g);
    if (status) return status;
    if (passes < 0) return gc_fail(ctx, GC_ERR_ARG, "passes must be >= 0");
    if (g->n > 0 && !colors) return gc_fail(ctx, GC_ERR_ARG, "colors is NULL");
    hipStream_t s = (hipStream_t)stream;
    GC_HIP(hipSetDevice(ctx->device));
    const gc_tuning start = ctx->tune;
    Timer tm;
    GC_HIP(hipEventCreate(&tm.e0));
    GC_HIP(hipEventCreate(&tm.e1));
    auto run = [&]() -> gc_status {
        gc_status st = gc_init_color(ctx, g, select, X, seed, 0, 0, colors, nullptr, s);
        for (int32_t p = 0; p < passes && st == GC_OK; p++)
            st = gc_recolor(ctx, g, perm, seed, p, colors, colors, nullptr, s);
        return st;
    };
    // warm-up (first-use allocations, residency probes) and the reference colors
    double ms = 0;
    uint64_t ref = 0, sum = 0;
    status = try_tuning(ctx, start, s, tm, run, colors, g->n, nullptr, 0, &ms, &ref);
    if (status) { ctx->tune = start; return status; }
    gc_tuning cur = start;
    double cur_ms = 1e30;
    for (int rep = 0; rep < 2; rep++) {
        status = try_tuning(ctx, cur, s, tm, run, colors, g->n, nullptr, 0, &ms, &sum);
        if (status) { ctx->tune = start; return status; }
        cur_ms = ms < cur_ms ? ms : cur_ms;
    }
    // one knob at a time, each over its candidates, the others fixed at the best so far
    struct Knob {
        int32_t gc_tuning::*field;
        std::vector<int32_t> values;
    };
    const Knob knobs[] = {
        {&gc_tuning::deg_wave, {32, 64, 128, 256, 1024}},
        {&gc_tuning::group, {2, 4, 8, 16, 32}},
        {&gc_tuning::walk_group, {0, 4, 8, 16}},
        {&gc_tuning::deg_split, {1024, 4096, 16384}},
        {&gc_tuning::grid_per_cu, {4, 8, 16}},
    };
    for (const Knob &k : knobs) {
        for (int32_t v : k.values) {
            if (cur.*(k.field) == v) continue;
            gc_tuning t = cur;
            t.*(k.field) = v;
            double best_here = 1e30;
            for (int rep = 0; rep < 2; rep++) {
                status = try_tuning(ctx, t, s, tm, run, colors, g->n, nullptr, 0, &ms, &sum);
                if (status) { ctx->tune = start; return status; }
                if (sum != ref) {
                    ctx->tune = start;
                    return gc_fail(ctx, GC_ERR_DEVICE, "autotune: a tuning changed the colors (knob value %d)", v);
                }
                best_here = ms < best_here ? ms : best_here;
            }
            if (best_here < cur_ms) {
                cur_ms = best_here;
                cur = t;
            }
        }
    }
    ctx->tune = cur;
    if (best) *best = cur;
    if (best_ms) *best_ms = cur_ms;
    return GC_OK;
}

static gc_status gc_autotune_batch_impl(gc_ctx *ctx, const gc_batch_csr *b, int32_t select, int32_t X, int32_t perm,
                                       int32_t passes, uint64_t base_seed, int32_t max_rounds,
                                       int32_t max_vertices_per_graph, int32_t *colors, gc_graph_stats *per_graph,
                                       gc_tuning *best, double *best_ms, void *stream) {
    if (!ctx) return GC_ERR_ARG;
    if (!b) return gc_fail(ctx, GC_ERR_ARG, "batch is NULL");
    if (b->num_graphs <= 0) return gc_fail(ctx, GC_ERR_ARG, "autotune needs at least one graph");
    if (!b->vtx_off) return gc_fail(ctx, GC_ERR_ARG, "NULL batch array");
    hipStream_t s = (hipStream_t)stream;
    GC_HIP(hipSetDevice(ctx->device));
    int64_t total_v = 0;
    GC_HIP(hipMemcpyAsync(&total_v, b->vtx_off + b->num_graphs, 8, hipMemcpyDeviceToHost, s));
    GC_HIP(hipStreamSynchronize(s));
    const gc_tuning start = ctx->tune;
    Timer tm;
    GC_HIP(hipEventCreate(&tm.e0));
    GC_HIP(hipEventCreate(&tm.e1));
    auto run = [&]() -> gc_status {
        return gc_batch_color(ctx, b, select, X, perm, passes, base_seed, max_rounds, max_vertices_per_graph, colors,
                              per_graph, s);
    };
    const int32_t *pg = (const int32_t *)per_graph;
    const int64_t npg = per_graph ? 4LL * b->num_graphs : 0;
    double ms = 0;
    uint64_t ref = 0, sum = 0;
    gc_status status = try_tuning(ctx, start, s, tm, run, colors, total_v, pg, npg, &ms, &ref);  // warm-up
    if (status) { ctx->tune = start; return status; }
    gc_tuning cur = start;
    double cur_ms = 1e30;
    for (int32_t order = 0; order <= 1; order++) {
        for (int32_t wg = 1; wg <= 5; wg++) {
            gc_tuning t = start;
            t.batch_order = order;
            t.batch_wg_per_cu = wg;
            status = try_tuning(ctx, t, s, tm, run, colors, total_v, pg, npg, &ms, &sum);
            if (status) { ctx->tune = start; return status; }
            if (sum != ref) {
                ctx->tune = start;
                return gc_fail(ctx, GC_ERR_DEVICE, "autotune: order %d with %d workgroups per CU changed the colors",
                               order, wg);
            }
            if (ms < cur_ms) {
                cur_ms = ms;
                cur = t;
            }
        }
    }
    ctx->tune = cur;
    if (best) *best = cur;
    if (best_ms) *best_ms = cur_ms;
    return GC_OK;
}

// Public entry points: the implementations above, with any sticky device
// failure harvested on the way reported in the returned status.
extern "C" gc_status gc_autotune(gc_ctx *ctx, const gc_csr *g, int32_t select, int32_t X, int32_t perm, int32_t passes,
                                 uint64_t seed, int32_t *colors, gc_tuning *best, double *best_ms, void *stream) {
    return gc_report(ctx, gc_autotune_impl(ctx, g, select, X, perm, passes, seed, colors, best, best_ms, stream));
}

extern "C" gc_status gc_autotune_batch(gc_ctx *ctx, const gc_batch_csr *b, int32_t select, int32_t X, int32_t perm,
                                       int32_t passes, uint64_t base_seed, int32_t max_rounds,
                                       int32_t max_vertices_per_graph, int32_t *colors, gc_graph_stats *per_graph,
                                       gc_tuning *best, double *best_ms, void *stream) {
    return gc_report(ctx, gc_autotune_batch_impl(ctx, b, select, X, perm, passes, base_seed, max_rounds, max_vertices_per_graph, colors, per_graph, best, best_ms, stream));
}
