// gc_init.hip - speculative round-synchronous initial coloring
// (section 2.2 framework, one superstep per round over every uncolored
// vertex; First Fit of section 2.1 or Random-X Fit of section 3.2).
//
// In-place encoding of the colors array C during the rounds:
//   C[v] > 0   committed color (final);
//   C[v] < 0   v is in the current round's set W_r with tentative color -C[v]
//              (or lost the previous round and waits for a new one);
//   C[v] = 0   never written (only before round 0).
// Readers of the assign step treat every value <= 0 as "no color", which is
// exactly the start-of-round snapshot: a value only becomes positive in the
// detect step.  The detect step compares |C[w]| with v's tentative color: a
// neighbor w with |C[w]| = T_v is necessarily in W_r (T_v avoids every color
// committed before the round), whether w has already flipped its own sign to
// commit or not.  Losers keep -T until the next assign overwrites it, so every
// detect read of the round sees every tentative color.
#include "gc_internal.h"

#include <vector>

// Round 0: every vertex is uncolored and no neighbor holds a color, so the
// tentative color of any vertex is a pure function of its id: 1 + j(v).
// Detect directly from the hash; no color is read.
template <bool RANDX>
__global__ void k_round0(const int32_t *__restrict__ rp, const int32_t *__restrict__ col, int64_t nnz, int32_t n,
                         int32_t *__restrict__ C, int32_t *__restrict__ wl_out, unsigned long long *wcount_out,
                         uint32_t s_prio, uint32_t s_color, uint32_t X) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t base = (int64_t)blockIdx.x * blockDim.x; base < n; base += stride) {
        int64_t i = base + threadIdx.x;
        bool lose = false;
        if (i < n) {
            int32_t v = (int32_t)i;
            int32_t e0, e1;
            row_range(rp, v, nnz, e0, e1);
            uint32_t tv = RANDX ? gc_pick(s_color, v, X) : 0u;
            uint32_t pv = gc_prio(s_prio, v);
            for (int32_t e = e0; e < e1; e++) {
                int32_t w = col[e];
                if ((uint32_t)w >= (uint32_t)n) continue;
                uint32_t tw = RANDX ? gc_pick(s_color, w, X) : 0u;
                if (tw == tv && gc_prio(s_prio, w) > pv) { lose = true; break; }
            }
            int32_t t = (int32_t)tv + 1;
            C[v] = lose ? -t : t;
        }
        wave_push(wl_out, wcount_out, lose, (int32_t)i);
    }
}

// Assign step of round r >= 1 over the worklist: tentative color into C[v] as -T.
__global__ void k_assign(const int32_t *__restrict__ rp, const int32_t *__restrict__ col, int64_t nnz, int32_t n,
                         int32_t *C, const int32_t *__restrict__ wl, const unsigned long long *__restrict__ wcount,
                         uint32_t s_color, uint32_t X, int randx, int64_t *round_stats_r) {
    const int64_t cnt = (int64_t)*wcount;
    unsigned long long degs = 0;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < cnt; i += stride) {
        int32_t v = wl[i];
        int32_t e0, e1;
        row_range(rp, v, nnz, e0, e1);
        degs += (unsigned long long)(e1 - e0);
        uint32_t j = randx ? gc_pick(s_color, v, X) : 0u;
        C[v] = -select_color_lane(col, e0, e1, C, n, j);
    }
    degs = wave_sum_u64(degs);
    if (__lane_id() == 0 && degs) atomicAdd((unsigned long long *)&round_stats_r[1], degs);
}

// Detect step of round r >= 1: v loses when a neighbor has the same tentative
// color and a larger priority; winners commit (flip the sign), losers go to wl_out.
__global__ void k_detect(const int32_t *__restrict__ rp, const int32_t *__restrict__ col, int64_t nnz, int32_t n,
                         int32_t *C, const int32_t *__restrict__ wl, const unsigned long long *__restrict__ wcount,
                         int32_t *__restrict__ wl_out, unsigned long long *wcount_out, uint32_t s_prio) {
    const int64_t cnt = (int64_t)*wcount;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t base = (int64_t)blockIdx.x * blockDim.x; base < cnt; base += stride) {
        int64_t i = base + threadIdx.x;
        bool lose = false;
        int32_t v = 0;
        if (i < cnt) {
            v = wl[i];
            int32_t t = -C[v];
            int32_t e0, e1;
            row_range(rp, v, nnz, e0, e1);
            uint32_t pv = gc_prio(s_prio, v);
            for (int32_t e = e0; e < e1; e++) {
                int32_t w = col[e];
                if ((uint32_t)w >= (uint32_t)n) continue;
                int32_t cw = C[w];
                if ((cw == t || cw == -t) && gc_prio(s_prio, w) > pv) { lose = true; break; }
            }
            if (!lose) C[v] = t;
        }
        wave_push(wl_out, wcount_out, lose, v);
    }
}

extern "C" gc_status gc_init_color(gc_ctx *ctx, const gc_csr *g, int32_t select, int32_t X, uint64_t seed,
                                   int32_t max_rounds, uint32_t flags, int32_t *colors, gc_stats *st, void *stream) {
    gc_status status = gc_check_graph_args(ctx, g);
    if (status) return status;
    if (select != GC_FIRST_FIT && select != GC_RANDOM_X) return gc_fail(ctx, GC_ERR_ARG, "select must be GC_FIRST_FIT or GC_RANDOM_X");
    if (select == GC_RANDOM_X && (X < 1 || X > GC_MAX_X)) return gc_fail(ctx, GC_ERR_ARG, "X must be in [1, %d]", GC_MAX_X);
    if (max_rounds < 0) return gc_fail(ctx, GC_ERR_ARG, "max_rounds must be >= 0");
    if (g->n > 0 && !colors) return gc_fail(ctx, GC_ERR_ARG, "colors is NULL");
    if (select == GC_FIRST_FIT) X = 1;
    const bool randx = select == GC_RANDOM_X;
    hipStream_t s = (hipStream_t)stream;
    GC_HIP(hipSetDevice(ctx->device));
    const int32_t n = g->n;
    if (n == 0) {
        if (st) {
            st->rounds = 0; st->num_colors = 0; st->max_color = 0; st->k_classes = 0; st->losers_total = 0;
        }
        return GC_OK;
    }
    auto prio_stream = [&](int32_t r) {
        return gc_stream_value(seed, GC_TAG_PRIO, (flags & GC_FLAG_FIXED_PRIORITY) ? 0u : (uint32_t)r);
    };
    const int block = 256;
    std::vector<int64_t> sizes;
    sizes.push_back(n);
    std::vector<int64_t> degsum;
    degsum.push_back(g->nnz);
    GC_HIP(hipMemsetAsync(ctx->scal + S_WCOUNT0, 0, 2 * 8, s));
    if (randx)
        k_round0<true><<<gc_grid(ctx, n, block), block, 0, s>>>(g->row_ptr, g->col_idx, g->nnz, n, colors, ctx->wl[0],
                                                              ctx->scal + S_WCOUNT0, prio_stream(0),
                                                              gc_stream_value(seed, GC_TAG_COLOR, 0), (uint32_t)X);
    else
        k_round0<false><<<gc_grid(ctx, n, block), block, 0, s>>>(g->row_ptr, g->col_idx, g->nnz, n, colors, ctx->wl[0],
                                                               ctx->scal + S_WCOUNT0, prio_stream(0), 0u, 1u);
    GC_LAUNCHED();
    int32_t r = 1, cur = 0;
    for (;;) {
        gc_status ss = gc_sync_scalars(ctx, s);
        if (ss) return ss;
        int64_t cnt = (int64_t)ctx->hscal[S_WCOUNT0 + cur];
        if (r > 1) degsum.push_back((int64_t)ctx->hscal[S_COUNT - 1]);
        if (cnt == 0) break;
        if (max_rounds > 0 && r == max_rounds) { status = GC_ERR_NOT_CONVERGED; break; }
        if (r > n) return gc_fail(ctx, GC_ERR_DEVICE, "no progress after %d rounds", r);  // each round commits >= 1 vertex
        sizes.push_back(cnt);
        int nxt = cur ^ 1;
        GC_HIP(hipMemsetAsync(ctx->scal + S_WCOUNT0 + nxt, 0, 8, s));
        GC_HIP(hipMemsetAsync(ctx->scal + S_COUNT - 2, 0, 16, s));
        int grid = gc_grid(ctx, cnt, block);
        k_assign<<<grid, block, 0, s>>>(g->row_ptr, g->col_idx, g->nnz, n, colors, ctx->wl[cur], ctx->scal + S_WCOUNT0 + cur,
                                        gc_stream_value(seed, GC_TAG_COLOR, (uint32_t)r), (uint32_t)X, randx ? 1 : 0,
                                        (int64_t *)(ctx->scal + S_COUNT - 2));
        GC_LAUNCHED();
        k_detect<<<grid, block, 0, s>>>(g->row_ptr, g->col_idx, g->nnz, n, colors, ctx->wl[cur], ctx->scal + S_WCOUNT0 + cur,
                                        ctx->wl[nxt], ctx->scal + S_WCOUNT0 + nxt, prio_stream(r));
        GC_LAUNCHED();
        cur = nxt;
        r++;
    }
    if (st) {
        st->rounds = (int32_t)sizes.size();
        int64_t tot = 0;
        for (int64_t x : sizes) tot += x;
        st->losers_total = tot - n;
        st->k_classes = 0;
        for (int32_t i = 0; i < st->round_cap && i < (int32_t)sizes.size(); i++) {
            if (st->round_sizes) st->round_sizes[i] = sizes[i];
            if (st->round_degsum) st->round_degsum[i] = i < (int32_t)degsum.size() ? degsum[i] : 0;
        }
        gc_status cs = gc_count_device(ctx, n, colors, s, true);
        if (cs) return cs;
        cs = gc_sync_scalars(ctx, s);
        if (cs) return cs;
        st->num_colors = (int32_t)ctx->hscal[S_NUMC];
        st->max_color = (int32_t)ctx->hscal[S_MAXC];
        if (status == GC_ERR_NOT_CONVERGED) gc_fail(ctx, status, "not converged after %d rounds", max_rounds);
    }
    return status;
}
