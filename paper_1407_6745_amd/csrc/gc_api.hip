// gc_api.hip - context management, status strings, and the checking /
// counting entry points of the C ABI (validate, count colors, CSR check).
#include "gc_internal.h"

#include <algorithm>
#include <mutex>
#include <vector>

#include <stdlib.h>
#include <string.h>

extern "C" const char *gc_status_string(gc_status s) {
    switch (s) {
        case GC_OK: return "ok";
        case GC_ERR_ARG: return "invalid argument";
        case GC_ERR_GRAPH: return "graph breaks a CSR precondition";
        case GC_ERR_COLORING: return "input coloring out of range";
        case GC_ERR_OOM: return "out of memory";
        case GC_ERR_DEVICE: return "HIP device error";
        case GC_ERR_NOT_CONVERGED: return "max_rounds reached before every vertex was colored";
    }
    return "unknown status";
}

gc_status gc_fail(gc_ctx *ctx, gc_status s, const char *fmt, ...) {
    if (ctx) {
        va_list ap;
        va_start(ap, fmt);
        vsnprintf(ctx->err, sizeof(ctx->err), fmt, ap);
        va_end(ap);
    }
    return s;
}

extern "C" const char *gc_ctx_last_error(const gc_ctx *ctx) { return ctx ? ctx->err : "no context"; }

int gc_grid(const gc_ctx *ctx, int64_t work, int block) {
    int64_t want = (work + block - 1) / block;
    int64_t cap = (int64_t)ctx->num_cu * (ctx->tune.grid_per_cu > 0 ? ctx->tune.grid_per_cu : 8);
    if (want > cap) want = cap;
    if (want < 1) want = 1;
    return (int)want;
}

gc_status gc_check_graph_args(gc_ctx *ctx, const gc_csr *g) {
    if (!ctx) return GC_ERR_ARG;
    if (!g) return gc_fail(ctx, GC_ERR_ARG, "graph is NULL");
    if (g->n < 0 || g->nnz < 0) return gc_fail(ctx, GC_ERR_ARG, "negative size");
    if (g->n > ctx->max_n) return gc_fail(ctx, GC_ERR_ARG, "n = %d above the context capacity %lld", g->n, (long long)ctx->max_n);
    if (g->nnz >= 2147483647LL) return gc_fail(ctx, GC_ERR_ARG, "nnz must be < 2^31");
    if (g->n > 0 && !g->row_ptr) return gc_fail(ctx, GC_ERR_ARG, "row_ptr is NULL");
    if (g->nnz > 0 && !g->col_idx) return gc_fail(ctx, GC_ERR_ARG, "col_idx is NULL");
    return GC_OK;
}

static void free_all(gc_ctx *c) {
    void *ptrs[] = {c->wl[0], c->wl[1], c->wl[2], c->wl[3], c->list, c->rows, c->hist, c->rank, c->pi, c->off, c->cursor,
                    c->keys, c->bitmap, c->round_stats, c->scal, c->bws, c->coff, c->segnz, c->histw, c->hist_s,
                    c->hist_sc, c->sbase, c->hsub, c->hub_bits, c->hub_cnt, c->hub_v, c->hub_first, c->shadow,
                    c->d2mask, c->border, c->longidx, c->fm, c->act, c->alen, c->hcopy, c->trace, c->sync};
    for (void *p : ptrs)
        if (p) (void)hipFree(p);
    if (c->hscal) (void)hipHostFree(c->hscal);
}

extern "C" gc_status gc_ctx_create(int device, int64_t max_n, int64_t max_nnz, gc_ctx **out) {
    if (!out) return GC_ERR_ARG;
    *out = nullptr;
    if (max_n < 0 || max_n > 2147483647LL - 4096 || max_nnz < 0) return GC_ERR_ARG;
    gc_ctx *ctx = (gc_ctx *)calloc(1, sizeof(gc_ctx));
    if (!ctx) return GC_ERR_OOM;
    ctx->device = device;
    ctx->max_n = max_n;
    ctx->max_nnz = max_nnz;
    ctx->ccap = (int32_t)(max_n + GC_MAX_X + 64);
    ctx->tune.block = 256;
    ctx->tune.deg_wave = 64;
    ctx->tune.group = 4;
    ctx->tune.grid_per_cu = 8;
    ctx->tune.walk_mode = 0;
    ctx->tune.xcd_chunks = -1;
    ctx->tune.deg_split = 4096;
    ctx->tune.split_len = 1024;
    ctx->tune.hub_words = GC_HUB_WORDS;
    ctx->tune.walk_group = 0;
    ctx->tune.d2_star = 0;
    ctx->tune.walk_flags = 0;
    ctx->tune.compact_init = -1;
    hipError_t e = hipSetDevice(device);
    if (e != hipSuccess) { free(ctx); return GC_ERR_DEVICE; }
    hipDeviceProp_t prop;
    e = hipGetDeviceProperties(&prop, device);
    if (e != hipSuccess) { free(ctx); return GC_ERR_DEVICE; }
    ctx->num_cu = prop.multiProcessorCount;
    ctx->dev_cu = prop.multiProcessorCount;
    size_t N = (size_t)max_n + 64;
    size_t CC = (size_t)ctx->ccap + 64;
    ctx->bitmap_bits = (int64_t)((CC + 63) / 64 * 64);
    struct { void **p; size_t bytes; } allocs[] = {
        {(void **)&ctx->wl[0], N * 4},       {(void **)&ctx->wl[1], N * 4},
        {(void **)&ctx->wl[2], N * 4},       {(void **)&ctx->wl[3], N * 4},
        {(void **)&ctx->list, (N + CC * 64) * 4},
        {(void **)&ctx->rows, (N + 64) * 8},
        {(void **)&ctx->hist, CC * 4},       {(void **)&ctx->rank, CC * 4},
        {(void **)&ctx->pi, CC * 4},         {(void **)&ctx->off, (3 * CC + 4) * 4},
        {(void **)&ctx->coff, (3 * CC + 4) * 4},
        {(void **)&ctx->segnz, (3 * CC + 4) * 4},
        {(void **)&ctx->histw, CC * 4},      {(void **)&ctx->hist_s, CC * 4},
        {(void **)&ctx->hist_sc, CC * 4},    {(void **)&ctx->sbase, (CC + 2) * 4},
        {(void **)&ctx->hcopy, (size_t)GC_HCOPY_INTS * 4},
        {(void **)&ctx->hsub, N * 4},        {(void **)&ctx->shadow, N * 2 + 256},
        {(void **)&ctx->cursor, (3 * CC + 4) * 4}, {(void **)&ctx->keys, CC * 8},
        {(void **)&ctx->bitmap, (size_t)ctx->bitmap_bits / 8},
        {(void **)&ctx->round_stats, 2 * N * 8},
        {(void **)&ctx->scal, S_COUNT * 8},
        {(void **)&ctx->sync, GC_SYNC_BYTES},
    };
    for (auto &a : allocs) {
        if (hipMalloc(a.p, a.bytes) != hipSuccess) { free_all(ctx); free(ctx); return GC_ERR_OOM; }
    }
    if (hipHostMalloc((void **)&ctx->hscal, S_COUNT * 8, hipHostMallocDefault) != hipSuccess) {
        free_all(ctx); free(ctx); return GC_ERR_OOM;
    }
    // buffers that must be zero between calls
    if (hipMemset(ctx->hist, 0, CC * 4) != hipSuccess || hipMemset(ctx->histw, 0, CC * 4) != hipSuccess ||
        hipMemset(ctx->hist_s, 0, CC * 4) != hipSuccess || hipMemset(ctx->hist_sc, 0, CC * 4) != hipSuccess ||
        hipMemset(ctx->hcopy, 0, (size_t)GC_HCOPY_INTS * 4) != hipSuccess || hipMemset(ctx->bitmap, 0, (size_t)ctx->bitmap_bits / 8) != hipSuccess ||
        hipMemset(ctx->scal, 0, S_COUNT * 8) != hipSuccess || hipDeviceSynchronize() != hipSuccess) {
        free_all(ctx); free(ctx); return GC_ERR_DEVICE;
    }
    *out = ctx;
    return GC_OK;
}

// ---------------------------------------------------------------------------
// kernel timing
// ---------------------------------------------------------------------------

#define TIMER_PAIRS 4096

struct gc_timer {
    unsigned mask;  // kernel kinds timed (bit k: kind k)
    hipEvent_t ev[2 * TIMER_PAIRS];
    int kind[TIMER_PAIRS];
    int pending;
    int open;  // index of the pair whose begin event was recorded last, or -1
    int64_t launches[GC_KERNEL_KINDS];
    double ms[GC_KERNEL_KINDS];
};

static void timer_flush(gc_timer *t) {
    for (int i = 0; i < t->pending; i++) {
        float ms = 0.f;
        if (hipEventSynchronize(t->ev[2 * i + 1]) == hipSuccess &&
            hipEventElapsedTime(&ms, t->ev[2 * i], t->ev[2 * i + 1]) == hipSuccess) {
            t->ms[t->kind[i]] += ms;
            t->launches[t->kind[i]]++;
        }
    }
    t->pending = 0;
}

static void timer_free(gc_timer *t) {
    if (!t) return;
    for (int i = 0; i < 2 * TIMER_PAIRS; i++)
        if (t->ev[i]) (void)hipEventDestroy(t->ev[i]);
    free(t);
}

void gc_time_begin(gc_ctx *ctx, int kind, hipStream_t s) {
    gc_timer *t = ctx->timer;
    if (!t || !((t->mask >> kind) & 1u)) return;
    if (t->pending == TIMER_PAIRS) timer_flush(t);
    t->kind[t->pending] = kind;
    (void)hipEventRecord(t->ev[2 * t->pending], s);
    t->open = t->pending;
}

void gc_time_end(gc_ctx *ctx, int kind, hipStream_t s) {
    gc_timer *t = ctx->timer;
    if (!t || t->open < 0 || t->kind[t->open] != kind) return;
    (void)hipEventRecord(t->ev[2 * t->open + 1], s);
    t->pending = t->open + 1;
    t->open = -1;
}

extern "C" gc_status gc_ctx_set_timing(gc_ctx *ctx, int enable) {
    if (!ctx) return GC_ERR_ARG;
    GC_HIP(hipSetDevice(ctx->device));
    if (ctx->timer) {
        (void)hipDeviceSynchronize();
        timer_free(ctx->timer);
        ctx->timer = nullptr;
    }
    if (!enable) return GC_OK;
    gc_timer *t = (gc_timer *)calloc(1, sizeof(gc_timer));
    if (!t) return gc_fail(ctx, GC_ERR_OOM, "timer");
    for (int i = 0; i < 2 * TIMER_PAIRS; i++) {
        if (hipEventCreate(&t->ev[i]) != hipSuccess) {
            timer_free(t);
            return gc_fail(ctx, GC_ERR_DEVICE, "hipEventCreate failed");
        }
    }
    t->open = -1;
    t->mask = enable < 0 ? ~0u : (unsigned)enable;
    ctx->timer = t;
    return GC_OK;
}

extern "C" gc_status gc_ctx_get_timing(gc_ctx *ctx, int64_t *launches, double *ms, int cap) {
    if (!ctx || cap < 0 || (cap > 0 && (!launches || !ms))) return GC_ERR_ARG;
    GC_HIP(hipSetDevice(ctx->device));
    for (int i = 0; i < cap && i < GC_KERNEL_KINDS; i++) { launches[i] = 0; ms[i] = 0.0; }
    if (!ctx->timer) return GC_OK;
    GC_HIP(hipDeviceSynchronize());
    timer_flush(ctx->timer);
    for (int i = 0; i < cap && i < GC_KERNEL_KINDS; i++) {
        launches[i] = ctx->timer->launches[i];
        ms[i] = ctx->timer->ms[i];
    }
    return GC_OK;
}

extern "C" void gc_ctx_destroy(gc_ctx *ctx) {
    if (!ctx) return;
    (void)hipSetDevice(ctx->device);
    (void)hipDeviceSynchronize();
    timer_free(ctx->timer);
    free_all(ctx);
    free(ctx);
}

extern "C" gc_status gc_ctx_get_tuning(const gc_ctx *ctx, gc_tuning *t) {
    if (!ctx || !t) return GC_ERR_ARG;
    *t = ctx->tune;
    return GC_OK;
}

extern "C" gc_status gc_ctx_set_tuning(gc_ctx *ctx, const gc_tuning *t) {
    if (!ctx || !t) return GC_ERR_ARG;
    if (t->block < 64 || t->block > 1024 || t->block % 64) return gc_fail(ctx, GC_ERR_ARG, "block must be a multiple of 64 in [64, 1024]");
    if (t->group < 1 || t->group > 64 || (t->group & (t->group - 1))) return gc_fail(ctx, GC_ERR_ARG, "group must be a power of two in [1, 64]");
    if (t->deg_wave < 0) return gc_fail(ctx, GC_ERR_ARG, "deg_wave must be >= 0");
    if (t->walk_mode < 0 || t->walk_mode > 1) return gc_fail(ctx, GC_ERR_ARG, "walk_mode must be 0 or 1");
    if (t->xcd_chunks < -1) return gc_fail(ctx, GC_ERR_ARG, "xcd_chunks must be >= -1");
    if (t->check_resident < 0 || t->check_resident > 1) return gc_fail(ctx, GC_ERR_ARG, "check_resident must be 0 or 1");
    if (t->deg_split < 0) return gc_fail(ctx, GC_ERR_ARG, "deg_split must be >= 0");
    if (t->split_len < 64) return gc_fail(ctx, GC_ERR_ARG, "split_len must be >= 64");
    if (t->hub_words < 1 || t->hub_words > GC_HUB_WORDS)
        return gc_fail(ctx, GC_ERR_ARG, "hub_words must be in [1, %d]", GC_HUB_WORDS);
    if (t->grid_per_cu < 1 || t->grid_per_cu > 64) return gc_fail(ctx, GC_ERR_ARG, "grid_per_cu must be in [1, 64]");
    if (t->walk_group < 0 || t->walk_group > 64 || (t->walk_group & (t->walk_group - 1)))
        return gc_fail(ctx, GC_ERR_ARG, "walk_group must be 0 or a power of two in [1, 64]");
    if (t->d2_star < -1 || t->d2_star > 1) return gc_fail(ctx, GC_ERR_ARG, "d2_star must be -1, 0 or 1");
    if (t->batch_wg_per_cu < 0 || t->batch_wg_per_cu > 5)
        return gc_fail(ctx, GC_ERR_ARG, "batch_wg_per_cu must be in [0, 5]");
    if (t->batch_order < 0 || t->batch_order > 1) return gc_fail(ctx, GC_ERR_ARG, "batch_order must be 0 or 1");
    if (t->spin_limit < 0) return gc_fail(ctx, GC_ERR_ARG, "spin_limit must be >= 0");
    if (t->check_input < 0 || t->check_input > 1) return gc_fail(ctx, GC_ERR_ARG, "check_input must be 0 or 1");
    if (t->trace < 0 || t->trace > 1) return gc_fail(ctx, GC_ERR_ARG, "trace must be 0 or 1");
    if (t->tail_max < -1) return gc_fail(ctx, GC_ERR_ARG, "tail_max must be >= -1");
    if (t->walk_flags < 0 || t->walk_flags > 7) return gc_fail(ctx, GC_ERR_ARG, "walk_flags must be in [0, 7]");
    if (t->cu_count < 0) return gc_fail(ctx, GC_ERR_ARG, "cu_count must be >= 0");
    if (t->compact_init < -1 || t->compact_init > 1) return gc_fail(ctx, GC_ERR_ARG, "compact_init must be -1, 0 or 1");
    if (t->compact_sat < 0 || t->compact_sat > 32767) return gc_fail(ctx, GC_ERR_ARG, "compact_sat must be in [0, 32767]");
    const int cus = t->cu_count > 0 && t->cu_count < ctx->dev_cu ? t->cu_count : ctx->dev_cu;
    if (cus != ctx->num_cu) {
        // launch sizes follow the compute units; the persistent walk's grid is measured again
        ctx->num_cu = cus;
        for (int &b : ctx->walk_blocks_v) b = 0;
    }
    ctx->tune = *t;
    return GC_OK;
}

extern "C" gc_status gc_ctx_get_info(gc_ctx *ctx, int64_t *info, int cap) {
    if (!ctx || cap < 0 || (cap > 0 && !info)) return GC_ERR_ARG;
    const int64_t v[5] = {ctx->num_cu, ctx->walk_blocks, ctx->num_cu ? ctx->walk_blocks / ctx->num_cu : 0,
                          ctx->deg_known ? ctx->deg_max : -1, ctx->deg_known ? ctx->deg_far_n : -1};
    for (int i = 0; i < cap && i < 5; i++) info[i] = v[i];
    return GC_OK;
}

gc_status gc_sync_scalars(gc_ctx *ctx, hipStream_t s) {
    GC_HIP(hipMemcpyAsync(ctx->hscal, ctx->scal, S_COUNT * 8, hipMemcpyDeviceToHost, s));
    GC_HIP(hipStreamSynchronize(s));
    if (ctx->hscal[S_STICKY]) {
        ctx->sticky |= ctx->hscal[S_STICKY];
        ctx->hscal[S_STICKY] = 0;
        GC_HIP(hipMemsetAsync(ctx->scal + S_STICKY, 0, 8, s));
    }
    return GC_OK;
}

gc_status gc_report(gc_ctx *ctx, gc_status st) {
    if (st != GC_OK || !ctx || !ctx->sticky) return st;
    const unsigned long long b = ctx->sticky;
    ctx->sticky = 0;
    return gc_fail(ctx, GC_ERR_DEVICE, "earlier asynchronous work on this context failed on the device:%s%s",
                   (b & 2) ? " a class-walk dependency wait gave up (colors of that pass are wrong)" : "",
                   (b & 4) ? " class-walk workgroups were not all resident" : "");
}

gc_status gc_check_input_coloring(gc_ctx *ctx, const gc_csr *g, const int32_t *colors, void *stream, int dist) {
    if (!ctx->tune.check_input || g->n == 0) return GC_OK;
    int64_t conflicts = 0, uncolored = 0;
    gc_status st = dist == 2 ? gc_validate_d2_impl(ctx, g, colors, &conflicts, &uncolored, stream)
                             : gc_validate_impl(ctx, g, colors, &conflicts, &uncolored, stream);
    if (st) return st;
    if (conflicts || uncolored)
        return gc_fail(ctx, GC_ERR_COLORING, "input is not a proper %scoloring: %lld conflicting %s, %lld vertices <= 0",
                       dist == 2 ? "distance-2 " : "", (long long)conflicts, dist == 2 ? "pairs" : "edges",
                       (long long)uncolored);
    return GC_OK;
}

extern "C" gc_status gc_ctx_get_trace(gc_ctx *ctx, int64_t *out, int64_t cap, int64_t *count, void *stream) {
    if (!ctx || cap < 0 || (cap > 0 && !out)) return GC_ERR_ARG;
    if (count) *count = 0;
    if (!ctx->trace) return gc_fail(ctx, GC_ERR_ARG, "no traced walk on this context (set the trace knob)");
    hipStream_t s = (hipStream_t)stream;
    GC_HIP(hipSetDevice(ctx->device));
    gc_status st = gc_sync_scalars(ctx, s);  // S_K: classes of the last pass
    if (st) return gc_report(ctx, st);
    const int64_t k = (int64_t)ctx->hscal[S_K];
    const int64_t words = 2 + 2 * k;
    std::vector<unsigned long long> raw((size_t)words);
    GC_HIP(hipMemcpyAsync(raw.data(), ctx->trace, (size_t)words * 8, hipMemcpyDeviceToHost, s));
    GC_HIP(hipStreamSynchronize(s));
    int rate_khz = 0;
    GC_HIP(hipDeviceGetAttribute(&rate_khz, hipDeviceAttributeWallClockRate, ctx->device));
    if (rate_khz <= 0) return gc_fail(ctx, GC_ERR_DEVICE, "wall clock rate unknown");
    const double ns_per_tick = 1e6 / (double)rate_khz;
    const unsigned long long t0 = raw[0];
    for (int64_t i = 0; i < words && i < cap; i++)
        out[i] = (i == 0) ? 0 : (raw[i] >= t0 ? (int64_t)((double)(raw[i] - t0) * ns_per_tick) : -1);
    if (count) *count = words;
    return gc_report(ctx, GC_OK);
}

extern "C" gc_status gc_ctx_status(gc_ctx *ctx, void *stream) {
    if (!ctx) return GC_ERR_ARG;
    GC_HIP(hipSetDevice(ctx->device));
    return gc_report(ctx, gc_sync_scalars(ctx, (hipStream_t)stream));
}

// ---------------------------------------------------------------------------
// validate: conflicting edges and uncolored vertices
// ---------------------------------------------------------------------------

// Validation in windows of 64 consecutive vertices: a wavefront loads their
// rows' bounds and colors, one vertex a lane, and spreads the rows' entries
// over its 64 lanes in flat order (a lane finds the row of its entry by a
// binary search over the rows' prefix sums, read across lanes), so that every
// lane stays busy whatever the degree mix.  A window with more than VAL_WIN
// entries goes, as (window, chunk) pairs of VAL_WIN entries, to a list that
// k_validate_long scans one wavefront per chunk: the work of a wavefront is
// then bounded by VAL_WIN entries however the long rows cluster (a skewed
// graph with its hubs at low ids has windows of 78,000 entries).  Counts
// entries (u, w) with u < w and equal positive colors, and vertices with a
// color <= 0.
#define VAL_WIN 4096
#define VAL_U 4

struct ValWindow {
    int32_t e0, excl, cv, total;
};

// Bounds, colors and prefix sums of the window's rows (lane = vertex
// base + lane); an uncolored vertex contributes no entries, since it has no
// conflicting edge.  unc counts the uncolored vertices when asked.
__device__ inline ValWindow val_window(const int32_t *__restrict__ rp, int64_t nnz, int32_t n,
                                       const int32_t *__restrict__ C, int64_t base, int lane,
                                       unsigned long long *unc) {
    ValWindow w = {0, 0, 0, 0};
    const int64_t v = base + lane;
    int32_t e1 = 0;
    if (v < n) {
        row_range(rp, (int32_t)v, nnz, w.e0, e1);
        w.cv = C[v];
        if (unc && w.cv <= 0) (*unc)++;
    }
    const int32_t len = w.cv > 0 ? e1 - w.e0 : 0;
    int32_t incl = len;
    for (int o = 1; o < 64; o <<= 1) {
        const int32_t y = __shfl_up(incl, o);
        if (lane >= o) incl += y;
    }
    w.excl = incl - len;
    w.total = __shfl(incl, 63);
    return w;
}

// Entries [t0, t1) of a window in flat order, VAL_U per lane a step; the
// next step's neighbor ids are loaded before this step's color gathers, so
// the two round trips overlap.
// IT: type of the positions in a window (int64_t only for graphs with nearly
// 2^31 entries, where t + 64 * VAL_U could wrap in 32 bits).
template <typename IT>
__device__ inline unsigned long long val_scan(const int32_t *__restrict__ col, const int32_t *__restrict__ C, int32_t n,
                                              int64_t base, const ValWindow &win, int32_t t0, int32_t t1, int lane) {
    unsigned long long conf = 0;
    int32_t w[VAL_U], c[VAL_U], uu[VAL_U];
    auto fetch = [&](IT ts) {
#pragma unroll
        for (int k = 0; k < VAL_U; k++) {
            const IT t = ts + 64 * k + lane;
            int32_t lo = 0, hi = 63;  // last lane whose rows start at or before t
#pragma unroll
            for (int step = 0; step < 6; step++) {
                const int32_t mid = (lo + hi + 1) >> 1;
                if (__shfl(win.excl, mid) <= t) lo = mid;
                else hi = mid - 1;
            }
            const int32_t a = __shfl(win.e0, lo), x = __shfl(win.excl, lo);
            c[k] = __shfl(win.cv, lo);
            uu[k] = (int32_t)base + lo;
            w[k] = t < t1 ? col[a + (t - x)] : -1;
        }
    };
    if (t0 < t1) fetch(t0);
    for (IT ts = t0; ts < t1; ts += 64 * VAL_U) {
        int32_t wn[VAL_U], cn[VAL_U], un[VAL_U];
#pragma unroll
        for (int k = 0; k < VAL_U; k++) {
            wn[k] = w[k];
            cn[k] = c[k];
            un[k] = uu[k];
        }
        if (ts + 64 * VAL_U < t1) fetch(ts + 64 * VAL_U);
        // each edge is checked from its smaller end only: half the color gathers
        int32_t cw[VAL_U];
#pragma unroll
        for (int k = 0; k < VAL_U; k++) {
            const bool need = (uint32_t)wn[k] < (uint32_t)n && wn[k] > un[k];
            cw[k] = need ? C[wn[k]] : 0;
        }
#pragma unroll
        for (int k = 0; k < VAL_U; k++)
            if (cw[k] == cn[k] && (uint32_t)wn[k] < (uint32_t)n && wn[k] > un[k]) conf++;
    }
    return conf;
}

template <typename IT>
__global__ void __launch_bounds__(256) k_validate(const int32_t *__restrict__ rp, const int32_t *__restrict__ col,
                                                  int64_t nnz, int32_t n, const int32_t *__restrict__ C,
                                                  int32_t *__restrict__ long_win, int32_t *__restrict__ long_chunk,
                                                  int64_t long_cap, unsigned long long *scal) {
    const int wpb = blockDim.x / 64;
    const int wib = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int lane = __lane_id();
    unsigned long long conf = 0, unc = 0;
    for (int64_t base = ((int64_t)blockIdx.x * wpb + wib) * 64; base < n; base += (int64_t)gridDim.x * wpb * 64) {
        const ValWindow win = val_window(rp, nnz, n, C, base, lane, &unc);
        if (win.total > VAL_WIN && long_cap > 0) {
            const int32_t nch = (win.total + VAL_WIN - 1) / VAL_WIN;
            unsigned long long p0 = 0;
            if (lane == 0) p0 = atomicAdd(&scal[S_VLONG], (unsigned long long)nch);
            const int64_t p = (int64_t)(((unsigned long long)__builtin_amdgcn_readfirstlane((uint32_t)(p0 >> 32)) << 32) |
                                        (uint32_t)__builtin_amdgcn_readfirstlane((uint32_t)p0));
            if (p + nch <= long_cap) {
                for (int32_t j = lane; j < nch; j += 64) {
                    long_win[p + j] = (int32_t)base;
                    long_chunk[p + j] = j;
                }
                continue;
            }
            // list full: the window stays here; the reserved slots that do
            // exist are marked empty
            for (int64_t j = p + lane; j < p + nch && j < long_cap; j += 64) long_win[j] = -1;
        }
        conf += val_scan<IT>(col, C, n, base, win, 0, win.total, lane);
    }
    __shared__ unsigned long long lds[16];
    conf = block_sum_u64(conf, lds);
    unc = block_sum_u64(unc, lds);
    if (threadIdx.x == 0) {
        if (conf) atomicAdd(&scal[S_CONFLICTS], conf);
        if (unc) atomicAdd(&scal[S_UNCOLORED], unc);
    }
}

// The heavy windows' chunks listed by k_validate: one wavefront per chunk.
template <typename IT>
__global__ void __launch_bounds__(256) k_validate_long(const int32_t *__restrict__ rp, const int32_t *__restrict__ col,
                                                       int64_t nnz, int32_t n, const int32_t *__restrict__ C,
                                                       const int32_t *__restrict__ long_win,
                                                       const int32_t *__restrict__ long_chunk, int64_t long_cap,
                                                       unsigned long long *scal) {
    const int wpb = blockDim.x / 64;
    const int wib = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int lane = __lane_id();
    int64_t cnt = (int64_t)scal[S_VLONG];
    if (cnt > long_cap) cnt = long_cap;  // reservations past the list were scanned by k_validate
    unsigned long long conf = 0;
    for (int64_t i = (int64_t)blockIdx.x * wpb + wib; i < cnt; i += (int64_t)gridDim.x * wpb) {
        const int32_t base = __builtin_amdgcn_readfirstlane(long_win[i]);
        if (base < 0) continue;
        const int32_t j = __builtin_amdgcn_readfirstlane(long_chunk[i]);
        const ValWindow win = val_window(rp, nnz, n, C, base, lane, nullptr);
        const int32_t t0 = j * VAL_WIN, t1 = win.total - t0 > VAL_WIN ? t0 + VAL_WIN : win.total;
        conf += val_scan<IT>(col, C, n, base, win, t0, t1, lane);
    }
    __shared__ unsigned long long lds[16];
    conf = block_sum_u64(conf, lds);
    if (threadIdx.x == 0 && conf) atomicAdd(&scal[S_CONFLICTS], conf);
}

gc_status gc_validate_impl(gc_ctx *ctx, const gc_csr *g, const int32_t *colors, int64_t *conflict_edges,
                                 int64_t *uncolored, void *stream) {
    gc_status st = gc_check_graph_args(ctx, g);
    if (st) return st;
    if (g->n > 0 && !colors) return gc_fail(ctx, GC_ERR_ARG, "colors is NULL");
    hipStream_t s = (hipStream_t)stream;
    GC_HIP(hipSetDevice(ctx->device));
    // Windows of more than VAL_WIN entries exist only when 64 rows can hold
    // them; otherwise the long-window launch is left out, and the list is
    // given no room, so that a window heavier than the cached longest row
    // promised (a graph changed in place) is still scanned where it is.
    int32_t maxdeg = 0;
    st = gc_graph_max_degree(ctx, g, s, &maxdeg);
    if (st) return st;
    const bool heavy = (int64_t)maxdeg * 64 > VAL_WIN;
    GC_HIP(hipMemsetAsync(ctx->scal + S_CONFLICTS, 0, 2 * 8, s));
    if (heavy) GC_HIP(hipMemsetAsync(ctx->scal + S_VLONG, 0, 8, s));
    if (g->n > 0) {
        const int block = 256;
        const int64_t waves = ((int64_t)g->n + 63) / 64;
        const int64_t cap = (int64_t)ctx->num_cu * 16;
        const int grid = (int)std::min<int64_t>((waves + 3) / 4, cap);
        // the long-row chunk list lives in two initial-coloring worklists (free here)
        // positions within a window in 64 bits only where 32 could wrap
        const bool wide = g->nnz > (int64_t)INT32_MAX - 65536;
        auto kv = wide ? k_validate<int64_t> : k_validate<int32_t>;
        auto kl = wide ? k_validate_long<int64_t> : k_validate_long<int32_t>;
        GC_TIMED(GC_K_OTHER, s, kv<<<grid, block, 0, s>>>(g->row_ptr, g->col_idx, g->nnz, g->n, colors, ctx->wl[1],
                                                           ctx->wl[2], heavy ? ctx->max_n : 0, ctx->scal));
        GC_LAUNCHED();
        if (heavy) {
            GC_TIMED(GC_K_OTHER, s, kl<<<ctx->num_cu * 4, block, 0, s>>>(g->row_ptr, g->col_idx, g->nnz, g->n, colors,
                                                                          ctx->wl[1], ctx->wl[2], ctx->max_n,
                                                                          ctx->scal));
            GC_LAUNCHED();
        }
    }
    st = gc_sync_scalars(ctx, s);
    if (st) return st;
    if (conflict_edges) *conflict_edges = (int64_t)ctx->hscal[S_CONFLICTS];
    if (uncolored) *uncolored = (int64_t)ctx->hscal[S_UNCOLORED];
    return GC_OK;
}

// ---------------------------------------------------------------------------
// count colors: max / min reduction, then a bitmap of present colors
// (workgroup-private in LDS for small colors) and a popcount
// ---------------------------------------------------------------------------

__global__ void k_minmax(int32_t n, const int32_t *__restrict__ C, unsigned long long *scal) {
    int32_t mx = 0, mn = 0x7fffffff;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        int32_t c = C[i];
        mx = max(mx, c);
        mn = min(mn, c);
    }
    __shared__ int32_t lds[16];
    mx = block_max_i32(mx, lds);
    mn = block_min_i32(mn, lds);
    if (threadIdx.x == 0) {
        atomicMax((int *)&scal[S_MAXC], mx);
        atomicMin((int *)&scal[S_MINC], mn);
    }
}

#define BITMAP_LDS_WORDS 2048  // colors 1..65536 tracked in LDS

__global__ void k_bitmap(int32_t n, const int32_t *__restrict__ C, uint32_t *bitmap, int64_t bitmap_bits) {
    __shared__ uint32_t lb[BITMAP_LDS_WORDS];
    for (int i = threadIdx.x; i < BITMAP_LDS_WORDS; i += blockDim.x) lb[i] = 0;
    __syncthreads();
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        int32_t c = C[i];
        if (c <= 0) continue;
        uint32_t b = (uint32_t)c - 1u;
        if (b < BITMAP_LDS_WORDS * 32u) {
            if (!(lb[b >> 5] & (1u << (b & 31)))) atomicOr(&lb[b >> 5], 1u << (b & 31));  // set bits are only read
        } else if ((int64_t)b < bitmap_bits) {
            atomicOr(&bitmap[b >> 5], 1u << (b & 31));
        }
    }
    __syncthreads();
    for (int i = threadIdx.x; i < BITMAP_LDS_WORDS; i += blockDim.x) {
        uint32_t w = lb[i];
        if (w && (int64_t)i * 32 < bitmap_bits) atomicOr(&bitmap[i], w);
    }
}

// popcount of bitmap words covering colors 1..maxc, clearing them for the next call
__global__ void k_popcount_clear(uint32_t *bitmap, int64_t bitmap_bits, unsigned long long *scal) {
    int64_t maxc = (int64_t)(int32_t)scal[S_MAXC];
    if (maxc > bitmap_bits) maxc = bitmap_bits;
    int64_t words = (maxc + 31) / 32;
    unsigned long long cnt = 0;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < words; i += stride) {
        uint32_t w = bitmap[i];
        if (w) {
            cnt += __popc(w);
            bitmap[i] = 0;
        }
    }
    __shared__ unsigned long long lds[16];
    cnt = block_sum_u64(cnt, lds);
    if (threadIdx.x == 0 && cnt) atomicAdd(&scal[S_NUMC], cnt);
}

__global__ void k_init_minmax(unsigned long long *scal) {
    if (threadIdx.x == 0) {
        scal[S_MAXC] = 0;
        scal[S_MINC] = 0x7fffffff;
        scal[S_NUMC] = 0;
    }
}

// Queues the count of distinct colors / max / min into ctx->scal (no sync).
// Colors above the bitmap capacity are not counted as distinct (the caller
// handles that case); the bitmap is left all zero.
gc_status gc_count_device(gc_ctx *ctx, int32_t n, const int32_t *colors, hipStream_t s, bool reset_minmax) {
    if (reset_minmax) {
        GC_TIMED(GC_K_COUNT, s, k_init_minmax<<<1, 64, 0, s>>>(ctx->scal));
        GC_LAUNCHED();
    }
    if (n <= 0) return GC_OK;
    int block = 256;
    const int rgrid = gc_grid(ctx, n, block) < 2 * ctx->num_cu ? gc_grid(ctx, n, block) : 2 * ctx->num_cu;
    GC_TIMED(GC_K_COUNT, s, k_minmax<<<rgrid, block, 0, s>>>(n, colors, ctx->scal));
    GC_LAUNCHED();
    GC_TIMED(GC_K_COUNT, s, k_bitmap<<<rgrid, block, 0, s>>>(n, colors, ctx->bitmap, ctx->bitmap_bits));
    GC_LAUNCHED();
    GC_TIMED(GC_K_COUNT, s, k_popcount_clear<<<gc_grid(ctx, ctx->bitmap_bits / 32, block), block, 0, s>>>(ctx->bitmap, ctx->bitmap_bits, ctx->scal));
    GC_LAUNCHED();
    return GC_OK;
}

static gc_status gc_count_colors_impl(gc_ctx *ctx, int32_t n, const int32_t *colors, int32_t *num_colors,
                                     int32_t *max_color, void *stream) {
    if (!ctx) return GC_ERR_ARG;
    if (n < 0 || n > ctx->max_n) return gc_fail(ctx, GC_ERR_ARG, "n out of range");
    if (n > 0 && !colors) return gc_fail(ctx, GC_ERR_ARG, "colors is NULL");
    hipStream_t s = (hipStream_t)stream;
    GC_HIP(hipSetDevice(ctx->device));
    gc_status st = gc_count_device(ctx, n, colors, s, true);
    if (st) return st;
    st = gc_sync_scalars(ctx, s);
    if (st) return st;
    int64_t maxc = (int64_t)(int32_t)ctx->hscal[S_MAXC];
    if (maxc > ctx->bitmap_bits) {
        // some color lies above the bitmap: grow it to cover every int32 color seen, count again
        int64_t bits = (maxc + 64) / 64 * 64;
        uint32_t *nb = nullptr;
        GC_HIP(hipStreamSynchronize(s));
        if (hipMalloc((void **)&nb, (size_t)bits / 8) != hipSuccess) return gc_fail(ctx, GC_ERR_OOM, "bitmap of %lld bits", (long long)bits);
        GC_HIP(hipMemsetAsync(nb, 0, (size_t)bits / 8, s));
        GC_HIP(hipStreamSynchronize(s));
        GC_HIP(hipFree(ctx->bitmap));
        ctx->bitmap = nb;
        ctx->bitmap_bits = bits;
        st = gc_count_device(ctx, n, colors, s, true);
        if (st) return st;
        st = gc_sync_scalars(ctx, s);
        if (st) return st;
    }
    if (num_colors) *num_colors = (int32_t)ctx->hscal[S_NUMC];
    if (max_color) *max_color = (int32_t)ctx->hscal[S_MAXC];
    return GC_OK;
}

// ---------------------------------------------------------------------------
// gc_count_colors_static: gc_count_colors without a context and without any
// allocation.  Its kernels (the ones above) work in one file-scope device
// array: 64 scalar slots, then the distinct-color bitmap for colors
// 1 .. GC_STATIC_MAX_COLOR.  Each device holds its own copy at its own
// address, looked up once per device with hipGetSymbolAddress; host code
// uses only that address.
// ---------------------------------------------------------------------------

#define STATIC_SLOTS 64
static __device__ __align__(256) unsigned long long scratch[STATIC_SLOTS + GC_STATIC_MAX_COLOR / 64];

#define STATIC_MAX_DEVICES 64
static unsigned long long *g_scratch[STATIC_MAX_DEVICES];  // device address of `scratch`, per device
static std::mutex g_scratch_mu;

__global__ void k_fill_u64(unsigned long long *p, int64_t words, unsigned long long value) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < words; i += stride) p[i] = value;
}

extern "C" gc_status gc_count_colors_static(int32_t n, const int32_t *colors, int32_t *num_colors, int32_t *max_color,
                                            void *stream) {
    if (n < 0) return GC_ERR_ARG;
    if (n > 0 && !colors) return GC_ERR_ARG;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= STATIC_MAX_DEVICES) return GC_ERR_DEVICE;
    unsigned long long *ptr;
    {
        std::lock_guard<std::mutex> lock(g_scratch_mu);
        if (!g_scratch[dev]) {
            void *p = nullptr;
            if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return GC_ERR_DEVICE;
            g_scratch[dev] = (unsigned long long *)p;
        }
        ptr = g_scratch[dev];
    }
    hipStream_t s = (hipStream_t)stream;
    uint32_t *bitmap = (uint32_t *)(ptr + STATIC_SLOTS);
    const int64_t bits = GC_STATIC_MAX_COLOR;
    // start from a clear array whatever an earlier call left (fill kernels, no memset nodes)
    k_fill_u64<<<64, 256, 0, s>>>(ptr, STATIC_SLOTS + GC_STATIC_MAX_COLOR / 64, 0ull);
    k_init_minmax<<<1, 64, 0, s>>>(ptr);
    if (n > 0) {
        int ncu = 0;
        if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || ncu < 1) ncu = 1;
        const int block = 256;
        const int64_t want = ((int64_t)n + block - 1) / block;
        const int grid = (int)(want < 2 * ncu ? want : 2 * ncu);
        k_minmax<<<grid, block, 0, s>>>(n, colors, ptr);
        k_bitmap<<<grid, block, 0, s>>>(n, colors, bitmap, bits);
        k_popcount_clear<<<(int)((bits / 32 + block - 1) / block), block, 0, s>>>(bitmap, bits, ptr);
    }
    if (hipGetLastError() != hipSuccess) return GC_ERR_DEVICE;
    static_assert(S_MAXC < 16 && S_NUMC < 16, "the slots read back");
    unsigned long long hs[16];  // host stack copy of the first scalar slots
    if (hipMemcpyAsync(hs, ptr, sizeof(hs), hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
        return GC_ERR_DEVICE;
    const int32_t maxc = (int32_t)hs[S_MAXC];
    if (maxc > GC_STATIC_MAX_COLOR) return GC_ERR_ARG;  // above the static bitmap
    if (num_colors) *num_colors = (int32_t)hs[S_NUMC];
    if (max_color) *max_color = maxc;
    return GC_OK;
}

// ---------------------------------------------------------------------------
// CSR precondition check
// ---------------------------------------------------------------------------

__global__ void k_check_rows(const int32_t *__restrict__ rp, int32_t n, int64_t nnz, unsigned long long *scal) {
    unsigned long long bad = 0, unsorted = 0;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += stride) {
        int32_t a = rp[v], b = rp[v + 1];
        if (a < 0 || b < a || b > nnz) bad++;
        if (v == 0 && a != 0) bad++;
        if (v == n - 1 && (int64_t)b != nnz) bad++;
    }
    bad = wave_sum_u64(bad);
    if (__lane_id() == 0 && bad) atomicAdd(&scal[S_GRAPHERR], bad);
    (void)unsorted;
}

__global__ void k_check_sorted(const int32_t *__restrict__ rp, const int32_t *__restrict__ col, int32_t n,
                               unsigned long long *scal) {
    unsigned long long uns = 0;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += stride) {
        for (int32_t e = rp[v] + 1; e < rp[v + 1]; e++)
            if (col[e - 1] > col[e]) { uns++; break; }
    }
    uns = wave_sum_u64(uns);
    if (__lane_id() == 0 && uns) atomicAdd(&scal[S_DONE], uns);
}

// count of x in the sorted (or, if !sorted, arbitrary) range col[a..b)
__device__ inline int32_t count_in_row(const int32_t *__restrict__ col, int32_t a, int32_t b, int32_t x, bool sorted) {
    if (!sorted) {
        int32_t c = 0;
        for (int32_t e = a; e < b; e++) c += col[e] == x;
        return c;
    }
    int32_t lo = a, hi = b;
    while (lo < hi) { int32_t m = lo + ((hi - lo) >> 1); if (col[m] < x) lo = m + 1; else hi = m; }
    int32_t first = lo;
    hi = b;
    while (lo < hi) { int32_t m = lo + ((hi - lo) >> 1); if (col[m] <= x) lo = m + 1; else hi = m; }
    return lo - first;
}

__global__ void k_check_entries(const int32_t *__restrict__ rp, const int32_t *__restrict__ col, int32_t n,
                                unsigned long long *scal) {
    bool sorted = scal[S_DONE] == 0;
    unsigned long long bad = 0;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += stride) {
        int32_t a = rp[v], b = rp[v + 1];
        for (int32_t e = a; e < b; e++) {
            int32_t w = col[e];
            if ((uint32_t)w >= (uint32_t)n || w == v) { bad++; continue; }
            // multiplicity of w in row v (count each run once, at its first entry when sorted)
            if (sorted && e > a && col[e - 1] == w) continue;
            int32_t fwd = count_in_row(col, a, b, w, sorted);
            int32_t back = count_in_row(col, rp[w], rp[w + 1], (int32_t)v, sorted);
            if (fwd != back) bad++;
        }
    }
    bad = wave_sum_u64(bad);
    if (__lane_id() == 0 && bad) atomicAdd(&scal[S_GRAPHERR], bad);
}

static gc_status gc_check_csr_impl(gc_ctx *ctx, const gc_csr *g, void *stream) {
    gc_status st = gc_check_graph_args(ctx, g);
    if (st) return st;
    hipStream_t s = (hipStream_t)stream;
    GC_HIP(hipSetDevice(ctx->device));
    GC_HIP(hipMemsetAsync(ctx->scal + S_GRAPHERR, 0, 8, s));
    GC_HIP(hipMemsetAsync(ctx->scal + S_DONE, 0, 8, s));
    if (g->n == 0) return g->nnz == 0 ? GC_OK : gc_fail(ctx, GC_ERR_GRAPH, "n = 0 with nnz > 0");
    int block = 256;
    GC_TIMED(GC_K_OTHER, s, k_check_rows<<<gc_grid(ctx, g->n, block), block, 0, s>>>(g->row_ptr, g->n, g->nnz, ctx->scal));
    GC_LAUNCHED();
    st = gc_sync_scalars(ctx, s);
    if (st) return st;
    if (ctx->hscal[S_GRAPHERR]) return gc_fail(ctx, GC_ERR_GRAPH, "row_ptr is not a valid offset array for nnz = %lld", (long long)g->nnz);
    GC_TIMED(GC_K_OTHER, s, k_check_sorted<<<gc_grid(ctx, g->n, block), block, 0, s>>>(g->row_ptr, g->col_idx, g->n, ctx->scal));
    GC_LAUNCHED();
    GC_TIMED(GC_K_OTHER, s, k_check_entries<<<gc_grid(ctx, g->n, block), block, 0, s>>>(g->row_ptr, g->col_idx, g->n, ctx->scal));
    GC_LAUNCHED();
    st = gc_sync_scalars(ctx, s);
    if (st) return st;
    if (ctx->hscal[S_GRAPHERR])
        return gc_fail(ctx, GC_ERR_GRAPH, "%llu adjacency entries out of range, self-loops or without a matching reverse entry",
                       (unsigned long long)ctx->hscal[S_GRAPHERR]);
    return GC_OK;
}

extern "C" uint64_t gc_batch_graph_seed(uint64_t base_seed, int32_t g) {
    return gc_mix64(base_seed + GC_GOLDEN * (((uint64_t)GC_TAG_GRAPH << 32) | (uint32_t)g));
}

gc_status gc_ensure_hub_slots(gc_ctx *ctx, int64_t nnz, int32_t deg_split, hipStream_t s) {
    const int64_t need = nnz / ((int64_t)deg_split + 1) + 1;
    if (need <= ctx->hub_cap) return GC_OK;
    GC_HIP(hipStreamSynchronize(s));
    void **bufs[4] = {(void **)&ctx->hub_bits, (void **)&ctx->hub_cnt, (void **)&ctx->hub_v, (void **)&ctx->hub_first};
    for (void **b : bufs)
        if (*b) { GC_HIP(hipFree(*b)); *b = nullptr; }
    ctx->hub_cap = 0;
    const int64_t cap = need + 64;
    if (hipMalloc((void **)&ctx->hub_bits, (size_t)cap * GC_HUB_WORDS * 8) != hipSuccess ||
        hipMalloc((void **)&ctx->hub_cnt, (size_t)cap * 4) != hipSuccess ||
        hipMalloc((void **)&ctx->hub_v, (size_t)cap * 4) != hipSuccess ||
        hipMalloc((void **)&ctx->hub_first, (size_t)cap * 4) != hipSuccess)
        return gc_fail(ctx, GC_ERR_OOM, "hub slots (%lld)", (long long)cap);
    GC_HIP(hipMemsetAsync(ctx->hub_bits, 0, (size_t)cap * GC_HUB_WORDS * 8, s));
    GC_HIP(hipMemsetAsync(ctx->hub_cnt, 0, (size_t)cap * 4, s));
    ctx->hub_cap = cap;
    return GC_OK;
}

__global__ void k_max_degree(const int32_t *__restrict__ rp, int32_t n, int64_t nnz, unsigned long long *scal) {
    __shared__ int32_t lds[32];
    int32_t mx = 0;
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x) {
        int32_t e0, e1;
        row_range(rp, (int32_t)v, nnz, e0, e1);
        mx = max(mx, e1 - e0);
    }
    const int32_t bm = block_max_i32(mx, lds);
    if (threadIdx.x == 0) atomicMax((int *)&scal[S_MAXDEG], bm);
}

// Far entries (|u - w| >= GC_NEAR).  The entries are cut into flat chunks of
// FAR_CHUNK, a wavefront per chunk, so that a long row spreads over many
// wavefronts.  A chunk finds the row of its first entry by a binary search of
// the row pointers, then takes its rows 64 at a time: lane l holds the end of
// row u + l, and the row of an entry is u plus the number of those ends at or
// before it, found by a binary search across the lanes.  Row pointers that
// are not monotone give a wrong count, never an access out of bounds.
constexpr int32_t FAR_CHUNK = 64 * 64;

__global__ void __launch_bounds__(256) k_far_entries(const int32_t *__restrict__ rp, const int32_t *__restrict__ col,
                                                     int32_t n, int64_t nnz, unsigned long long *scal) {
    __shared__ unsigned long long lds[16];
    unsigned long long far = 0;
    const int lane = __lane_id();
    const int64_t wave = (int64_t)blockIdx.x * (blockDim.x >> 6) + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int64_t waves = (int64_t)gridDim.x * (blockDim.x >> 6);
    const int32_t m = (int32_t)nnz;  // row pointers are int32, so nnz fits
    for (int64_t c = wave * FAR_CHUNK; c < nnz; c += waves * FAR_CHUNK) {
        const int64_t c1 = c + FAR_CHUNK < nnz ? c + FAR_CHUNK : nnz;  // (64-bit: no wrap near 2^31 entries)
        int32_t lo = 0, hi = n;  // the last row whose first entry is at or before c
        while (hi - lo > 1) {
            const int32_t mid = lo + ((hi - lo) >> 1);
            if (rp[mid] <= c) lo = mid;
            else hi = mid;
        }
        int64_t e = c;
        for (int64_t u = lo; u < n && e < c1; u += 64) {
            const int64_t r = u + lane;
            int32_t end = m;
            if (r < n) {
                end = rp[r + 1];
                end = end < 0 ? 0 : (end > m ? m : end);
            }
            const int64_t w_end = min(c1, (int64_t)__shfl(end, 63));
            for (; e < w_end; e += 64) {
                const int64_t x = e + lane;
                int32_t k = 0;
#pragma unroll
                for (int32_t s = 32; s; s >>= 1)
                    if (__shfl(end, k + s - 1) <= x) k += s;
                if (x < w_end) {
                    const int64_t d = (int64_t)col[x] - (u + k);
                    far += (d >= GC_NEAR || d <= -GC_NEAR) ? 1ull : 0ull;
                }
            }
            e = e > w_end ? w_end : e;  // the last step may overrun the window by up to 63
        }
    }
    far = block_sum_u64(far, lds);
    if (threadIdx.x == 0 && far) atomicAdd(&scal[S_FAR], far);
}

// Longest row of g and the fraction of far entries, computed once per graph
// (keyed by its arrays and sizes; they only pick kernel variants, every
// variant colors any graph correctly).
gc_status gc_graph_max_degree(gc_ctx *ctx, const gc_csr *g, hipStream_t s, int32_t *out) {
    if (ctx->deg_key_rp == g->row_ptr && ctx->deg_key_col == g->col_idx && ctx->deg_key_n == g->n &&
        ctx->deg_key_nnz == g->nnz) {
        *out = ctx->deg_max;
        return GC_OK;
    }
    GC_HIP(hipMemsetAsync(ctx->scal + S_MAXDEG, 0, 8, s));
    GC_HIP(hipMemsetAsync(ctx->scal + S_FAR, 0, 8, s));
    const int grid = gc_grid(ctx, g->n, 256) < 2 * ctx->num_cu ? gc_grid(ctx, g->n, 256) : 2 * ctx->num_cu;
    k_max_degree<<<grid, 256, 0, s>>>(g->row_ptr, g->n, g->nnz, ctx->scal);
    GC_LAUNCHED();
    if (g->nnz > 0) {
        const int64_t blocks = (g->nnz + 4 * FAR_CHUNK - 1) / (4 * FAR_CHUNK);  // four wavefronts a block
        k_far_entries<<<(int)(blocks < 8 * ctx->num_cu ? blocks : 8 * ctx->num_cu), 256, 0, s>>>(
            g->row_ptr, g->col_idx, g->n, g->nnz, ctx->scal);
        GC_LAUNCHED();
    }
    gc_status st = gc_sync_scalars(ctx, s);
    if (st) return st;
    ctx->deg_max = (int32_t)ctx->hscal[S_MAXDEG];
    ctx->deg_far_n = g->nnz > 0 ? (int64_t)ctx->hscal[S_FAR] : 0;
    ctx->deg_far = g->nnz > 0 ? (double)ctx->deg_far_n / (double)g->nnz : 0.0;
    ctx->deg_known = 1;
    ctx->deg_key_rp = g->row_ptr;
    ctx->deg_key_col = g->col_idx;
    ctx->deg_key_n = g->n;
    ctx->deg_key_nnz = g->nnz;
    *out = ctx->deg_max;
    return GC_OK;
}

gc_status gc_graph_far_fraction(gc_ctx *ctx, const gc_csr *g, hipStream_t s, double *out) {
    int32_t maxdeg = 0;
    gc_status st = gc_graph_max_degree(ctx, g, s, &maxdeg);
    if (st) return st;
    *out = ctx->deg_far;
    return GC_OK;
}


extern "C" int32_t gc_schedule_perm(int32_t schedule, int32_t base, int32_t x, int32_t t) {
    if (t < 1) return -1;
    switch (schedule) {
        case GC_SCHED_FIXED: return (base >= GC_PERM_REVERSE && base <= GC_PERM_RANDOM) ? base : -1;
        case GC_SCHED_ND_RAND_X:
            if (x < 1) return -1;
            return t % x == 0 ? GC_PERM_RANDOM : GC_PERM_NONDEC;
        case GC_SCHED_ND_RAND_POW2: return (t >= 2 && (t & (t - 1)) == 0) ? GC_PERM_RANDOM : GC_PERM_NONDEC;
        default: return -1;
    }
}

static gc_status gc_color_preset_impl(gc_ctx *ctx, const gc_csr *g, int32_t preset, uint64_t seed, int32_t *colors,
                                     gc_stats *st, void *stream) {
    if (!ctx) return GC_ERR_ARG;
    if (preset == GC_PRESET_SPEED) return gc_init_color(ctx, g, GC_FIRST_FIT, 1, seed, 0, 0, colors, st, stream);
    if (preset != GC_PRESET_QUALITY) return gc_fail(ctx, GC_ERR_ARG, "unknown preset %d", preset);
    gc_status s = gc_init_color(ctx, g, GC_RANDOM_X, 5, seed, 0, 0, colors, st, stream);
    if (s) return s;
    gc_stats rs{};
    s = gc_recolor(ctx, g, GC_PERM_NONDEC, seed, 0, colors, colors, st ? &rs : nullptr, stream);
    if (s) return s;
    if (st) {
        st->num_colors = rs.num_colors;
        st->max_color = rs.max_color;
        st->k_classes = rs.k_classes;
    }
    return GC_OK;
}

// Public entry points: the implementations above, with any sticky device
// failure harvested on the way reported in the returned status.
extern "C" gc_status gc_validate(gc_ctx *ctx, const gc_csr *g, const int32_t *colors, int64_t *conflict_edges,
                                 int64_t *uncolored, void *stream) {
    return gc_report(ctx, gc_validate_impl(ctx, g, colors, conflict_edges, uncolored, stream));
}

extern "C" gc_status gc_count_colors(gc_ctx *ctx, int32_t n, const int32_t *colors, int32_t *num_colors,
                                     int32_t *max_color, void *stream) {
    return gc_report(ctx, gc_count_colors_impl(ctx, n, colors, num_colors, max_color, stream));
}

extern "C" gc_status gc_check_csr(gc_ctx *ctx, const gc_csr *g, void *stream) {
    return gc_report(ctx, gc_check_csr_impl(ctx, g, stream));
}

extern "C" gc_status gc_color_preset(gc_ctx *ctx, const gc_csr *g, int32_t preset, uint64_t seed, int32_t *colors,
                                     gc_stats *st, void *stream) {
    return gc_report(ctx, gc_color_preset_impl(ctx, g, preset, seed, colors, st, stream));
}
