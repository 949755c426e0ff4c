// gc_d2.hip - distance-2 coloring (section 1: vertices joined by a path of at
// most two edges get different colors; the paper expects its techniques to
// carry over to such variants).  The same speculative rounds as the distance-1
// initial coloring (section 2.2 framework; First Fit of section 2.1 or
// Random-X Fit of section 3.2) and the same recoloring passes (section 3),
// with every neighborhood read as the distance-2 neighborhood
// N2(v) = N(v) u N(N(v)) minus v.
//
// Work layout: one wavefront per vertex.  The wavefront reads v's row in
// chunks of 64 entries (one neighbor u per lane), then the rows of those
// neighbors flattened over its 64 lanes: the lane holding entry t of the
// batch finds its row by a binary search over the chunk's prefix sums of row
// lengths (cross-lane reads, no LDS), so short and long rows alike keep every
// lane busy.  A vertex reached along several paths is seen once per path,
// which changes no result: colors go into a bitmap, and a conflict is "some
// neighbor".
//
// Encoding of C during the rounds is the distance-1 one: C[v] > 0 committed,
// C[v] < 0 tentative (or a loser waiting for the next round).  A tentative
// color T_v avoids every color committed in N2(v) before the round, so a w in
// N2(v) with |C[w]| = T_v belongs to the same round, whether it has already
// committed in this detect step or not.
#include "gc_internal.h"

#include <vector>

#define D2_BLOCK 256
#define D2_WORDS 64                // color-window bitmap words per wavefront (one per lane)
#define D2_WINDOW (32 * D2_WORDS)  // colors per window
#define D2_UNROLL 4

// Calls f(w) for every w in N2(v) (repeats allowed), v's row being
// col[e0, e1).  All 64 lanes must call it with the same v, e0, e1.  f returns
// true to stop; the visit then ends after the current step (v's own chunk of
// neighbors, or D2_UNROLL batches of 64 two-hop entries) and the call returns
// true (uniform over the wavefront).  Ids outside [0, n) are skipped.
template <class F>
__device__ inline bool d2_visit(const int32_t *__restrict__ rp, const int32_t *__restrict__ col, int64_t nnz,
                                int32_t n, int32_t v, int32_t e0, int32_t e1, F &&f) {
    const int lane = __lane_id();
    for (int32_t c = e0; c < e1; c += 64) {
        const int32_t m = min(64, e1 - c);
        int32_t a = 0, len = 0;
        bool stop = false;
        if (lane < m) {
            const int32_t u = col[c + lane];
            if ((uint32_t)u < (uint32_t)n) {
                int32_t b;
                row_range(rp, u, nnz, a, b);
                len = b - a;
                stop = f(u);
            }
        }
        if (__ballot(stop)) return true;
        int32_t incl = len;
        for (int o = 1; o < 64; o <<= 1) {
            const int32_t y = __shfl_up(incl, o);
            if (lane >= o) incl += y;
        }
        const int32_t excl = incl - len;
        const int32_t total = __shfl(incl, 63);
        // D2_UNROLL batches of 64 entries per step: their loads are in flight together
        for (int32_t t0 = 0; t0 < total; t0 += 64 * D2_UNROLL) {
            int32_t w[D2_UNROLL];
#pragma unroll
            for (int k = 0; k < D2_UNROLL; k++) {
                const int32_t t = t0 + 64 * k + lane;
                // last neighbor slot i < m whose range starts at or before t
                int32_t lo = 0, hi = m - 1;
#pragma unroll
                for (int step = 0; step < 6; step++) {
                    const int32_t mid = (lo + hi + 1) >> 1;
                    if (__shfl(excl, mid) <= t) lo = mid;
                    else hi = mid - 1;
                }
                const int32_t ra = __shfl(a, lo), rx = __shfl(excl, lo);
                w[k] = t < total ? col[ra + (t - rx)] : v;
            }
#pragma unroll
            for (int k = 0; k < D2_UNROLL; k++)
                if (w[k] != v && (uint32_t)w[k] < (uint32_t)n) stop |= f(w[k]);
            if (__ballot(stop)) return true;
        }
    }
    return false;
}

// (j+1)-th smallest positive color held by no w in N2(v) as a positive value
// of C.  bits: the wavefront's D2_WORDS words of LDS.  Windows of D2_WINDOW
// colors; a window without enough free colors rescans N2(v) for the next.
__device__ inline int32_t d2_select(const int32_t *__restrict__ rp, const int32_t *__restrict__ col, int64_t nnz,
                                    int32_t n, const int32_t *C, int32_t v, int32_t e0, int32_t e1, uint32_t j,
                                    uint32_t *bits) {
    const int lane = __lane_id();
    uint32_t base = 1;
    for (;;) {
        bits[lane] = 0u;
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        d2_visit(rp, col, nnz, n, v, e0, e1, [&](int32_t w) {
            const int32_t c = C[w];
            const uint32_t d = (uint32_t)c - base;  // colors below the window wrap to large values
            if (c > 0 && d < (uint32_t)D2_WINDOW) atomicOr(&bits[d >> 5], 1u << (d & 31));
            return false;
        });
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        const uint32_t fw = ~bits[lane];
        const uint32_t f = (uint32_t)__popc(fw);
        uint32_t incl = f;
        for (int o = 1; o < 64; o <<= 1) {
            const uint32_t y = __shfl_up(incl, o);
            if (lane >= o) incl += y;
        }
        const uint32_t tot = __shfl(incl, 63);
        if (j < tot) {
            const uint32_t ex = incl - f;
            const bool mine = ex <= j && j < incl;
            const unsigned long long b = __ballot(mine);
            const int src = __ffsll((long long)b) - 1;
            uint32_t pos = 0;
            if (mine) pos = nth_set_bit((uint64_t)fw, j - ex);
            pos = __shfl(pos, src);
            return (int32_t)(base + 32u * (uint32_t)src + pos);
        }
        j -= tot;
        base += (uint32_t)D2_WINDOW;
    }
}

// Per-wavefront queue of losers in LDS: one global atomic per 64 entries.
struct WaveQueue {
    int32_t *q;  // 64 LDS slots of the wavefront
    int32_t len = 0;

    __device__ void flush(int32_t *wl, unsigned long long *count) {
        if (len == 0) return;
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        const int lane = __lane_id();
        unsigned int base = 0;
        if (lane == 0) base = (unsigned int)atomicAdd(count, (unsigned long long)len);
        base = __shfl(base, 0);
        if (lane < len) wl[base + lane] = q[lane];
        __builtin_amdgcn_wave_barrier();
        len = 0;
    }
    __device__ void push(int32_t v, int32_t *wl, unsigned long long *count) {
        if (__lane_id() == 0) q[len] = v;
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        if (++len == 64) flush(wl, count);
    }
};

__device__ inline int32_t d2_round0_color(uint32_t s_color, int32_t w, uint32_t X, int randx) {
    return randx ? (int32_t)gc_pick(s_color, w, X) + 1 : 1;
}

// Round 0: every vertex's tentative color follows from the hash alone (no
// color is held yet), so assign and detect fuse: v keeps T_v unless a
// vertex of N2(v) with the same T has a larger key.
__global__ void __launch_bounds__(D2_BLOCK) k_d2_round0(const int32_t *__restrict__ rp,
                                                        const int32_t *__restrict__ col, int64_t nnz, int32_t n,
                                                        int32_t *C, Prio pr, uint32_t s_color, uint32_t X, int randx,
                                                        int32_t *wl_out, unsigned long long *c_out) {
    __shared__ int32_t qs[D2_BLOCK];
    const int wpb = D2_BLOCK / 64;
    const int wib = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    WaveQueue lq{qs + wib * 64};
    for (int32_t v = blockIdx.x * wpb + wib; v < n; v += gridDim.x * wpb) {
        int32_t e0, e1;
        row_range(rp, v, nnz, e0, e1);
        const int32_t T = d2_round0_color(s_color, v, X, randx);
        const uint64_t pv = round_prio(pr, v);
        const bool lose = d2_visit(rp, col, nnz, n, v, e0, e1, [&](int32_t w) {
            return d2_round0_color(s_color, w, X, randx) == T && round_prio(pr, w) > pv;
        });
        if (__lane_id() == 0) C[v] = lose ? -T : T;
        if (lose) lq.push(v, wl_out, c_out);
    }
    lq.flush(wl_out, c_out);
}

// Rounds >= 1, assign step: every vertex of the worklist takes the (j+1)-th
// smallest color free in N2(v) among the colors committed before the round.
__global__ void __launch_bounds__(D2_BLOCK) k_d2_assign(const int32_t *__restrict__ rp,
                                                        const int32_t *__restrict__ col, int64_t nnz, int32_t n,
                                                        int32_t *C, const int32_t *__restrict__ wl,
                                                        const unsigned long long *__restrict__ wc, uint32_t s_color,
                                                        uint32_t X, int randx) {
    __shared__ uint32_t bits_all[D2_BLOCK / 64 * D2_WORDS];
    const int wpb = D2_BLOCK / 64;
    const int wib = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    uint32_t *bits = bits_all + wib * D2_WORDS;
    const int64_t cnt = (int64_t)*wc;
    for (int64_t i = (int64_t)blockIdx.x * wpb + wib; i < cnt; i += (int64_t)gridDim.x * wpb) {
        const int32_t v = __builtin_amdgcn_readfirstlane(wl[i]);
        int32_t e0, e1;
        row_range(rp, v, nnz, e0, e1);
        const uint32_t j = randx ? gc_pick(s_color, v, X) : 0u;
        const int32_t c = d2_select(rp, col, nnz, n, C, v, e0, e1, j, bits);
        if (__lane_id() == 0) C[v] = -c;
    }
}

// Rounds >= 1, detect step: v loses iff some w in N2(v) holds the same
// tentative color (|C[w]| = T_v) with a larger key; winners commit.
__global__ void __launch_bounds__(D2_BLOCK) k_d2_detect(const int32_t *__restrict__ rp,
                                                        const int32_t *__restrict__ col, int64_t nnz, int32_t n,
                                                        int32_t *C, const int32_t *__restrict__ wl,
                                                        const unsigned long long *__restrict__ wc, Prio pr,
                                                        int32_t *wl_out, unsigned long long *c_out) {
    __shared__ int32_t qs[D2_BLOCK];
    const int wpb = D2_BLOCK / 64;
    const int wib = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    WaveQueue lq{qs + wib * 64};
    const int64_t cnt = (int64_t)*wc;
    for (int64_t i = (int64_t)blockIdx.x * wpb + wib; i < cnt; i += (int64_t)gridDim.x * wpb) {
        const int32_t v = __builtin_amdgcn_readfirstlane(wl[i]);
        int32_t e0, e1;
        row_range(rp, v, nnz, e0, e1);
        const int32_t T = -__builtin_amdgcn_readfirstlane(C[v]);
        const uint64_t pv = round_prio(pr, v);
        const bool lose = d2_visit(rp, col, nnz, n, v, e0, e1, [&](int32_t w) {
            const int32_t c = C[w];
            return (c == T || c == -T) && round_prio(pr, w) > pv;
        });
        if (!lose && __lane_id() == 0) C[v] = T;
        if (lose) lq.push(v, wl_out, c_out);
    }
    lq.flush(wl_out, c_out);
}

// One class of a recoloring pass: every vertex of rank s takes the smallest
// color free among the new colors (positive values) of N2(v).
__global__ void __launch_bounds__(D2_BLOCK) k_d2_class(const int32_t *__restrict__ rp, const int32_t *__restrict__ col,
                                                       int64_t nnz, int32_t n, int32_t *C,
                                                       const int32_t *__restrict__ list, int32_t a, int32_t b) {
    __shared__ uint32_t bits_all[D2_BLOCK / 64 * D2_WORDS];
    const int wpb = D2_BLOCK / 64;
    const int wib = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    uint32_t *bits = bits_all + wib * D2_WORDS;
    for (int32_t i = a + blockIdx.x * wpb + wib; i < b; i += gridDim.x * wpb) {
        const int32_t v = __builtin_amdgcn_readfirstlane(list[i]);
        int32_t e0, e1;
        row_range(rp, v, nnz, e0, e1);
        const int32_t c = d2_select(rp, col, nnz, n, C, v, e0, e1, 0u, bits);
        if (__lane_id() == 0) C[v] = c;
    }
}

// Vertices sharing their positive color with a vertex of N2(v), and vertices
// with color <= 0.
__global__ void __launch_bounds__(D2_BLOCK) k_d2_validate(const int32_t *__restrict__ rp,
                                                          const int32_t *__restrict__ col, int64_t nnz, int32_t n,
                                                          const int32_t *__restrict__ C, unsigned long long *conflicts,
                                                          unsigned long long *uncolored) {
    const int wpb = D2_BLOCK / 64;
    const int wib = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    unsigned long long nc = 0, nu = 0;
    for (int32_t v = blockIdx.x * wpb + wib; v < n; v += gridDim.x * wpb) {
        const int32_t cv = __builtin_amdgcn_readfirstlane(C[v]);
        if (cv <= 0) {
            nu++;
            continue;
        }
        int32_t e0, e1;
        row_range(rp, v, nnz, e0, e1);
        if (d2_visit(rp, col, nnz, n, v, e0, e1, [&](int32_t w) { return C[w] == cv; })) nc++;
    }
    if (__lane_id() == 0) {
        if (nc) atomicAdd(conflicts, nc);
        if (nu) atomicAdd(uncolored, nu);
    }
}

static int d2_grid(const gc_ctx *ctx, int64_t items) {
    const int64_t cap = (int64_t)ctx->num_cu * ctx->tune.grid_per_cu;
    const int64_t want = (items + D2_BLOCK / 64 - 1) / (D2_BLOCK / 64);
    return (int)(want < 1 ? 1 : (want > cap ? cap : want));
}

gc_status gc_spec_rounds_d2(gc_ctx *ctx, const gc_csr *g, int32_t select, int32_t X, uint64_t seed, int32_t max_rounds,
                            uint32_t flags, int32_t *colors, gc_stats *st, hipStream_t s) {
    gc_status status = GC_OK;
    if (select == GC_FIRST_FIT) X = 1;
    const int randx = select == GC_RANDOM_X ? 1 : 0;
    const int32_t n = g->n;
    const int pmode = (flags & GC_FLAG_PRIO_NATURAL) ? PRIO_NATURAL : PRIO_HASH;
    auto prio_of = [&](int32_t r) {
        const bool fixed = (flags & GC_FLAG_FIXED_PRIORITY) != 0;
        return Prio{pmode, gc_stream_value(seed, GC_TAG_PRIO, fixed ? 0u : (uint32_t)r), nullptr, g->row_ptr};
    };
    // worklists wl[0] / wl[1], their counts in scal[S_WL] / scal[S_WL + 1]
    unsigned long long *cnt = ctx->scal + S_WL;
    std::vector<int64_t> sizes;
    sizes.push_back(n);
    GC_HIP(hipMemsetAsync(cnt, 0, 2 * 8, s));
    GC_TIMED(GC_K_ROUND0, s, k_d2_round0<<<d2_grid(ctx, n), D2_BLOCK, 0, s>>>(
                                 g->row_ptr, g->col_idx, g->nnz, n, colors, prio_of(0),
                                 gc_stream_value(seed, GC_TAG_COLOR, 0), (uint32_t)X, randx, ctx->wl[0], cnt));
    GC_LAUNCHED();
    int32_t r = 1, cur = 0;
    for (;;) {
        gc_status ss = gc_sync_scalars(ctx, s);
        if (ss) return ss;
        const int64_t tot = (int64_t)ctx->hscal[S_WL + cur];
        if (tot == 0) break;
        if (max_rounds > 0 && r == max_rounds) { status = GC_ERR_NOT_CONVERGED; break; }
        if (r > n) return gc_fail(ctx, GC_ERR_DEVICE, "no progress after %d rounds", r);  // each round commits >= 1 vertex
        sizes.push_back(tot);
        const int nxt = cur ^ 1;
        GC_HIP(hipMemsetAsync(cnt + nxt, 0, 8, s));
        const int grid = d2_grid(ctx, tot);
        GC_TIMED(GC_K_ASSIGN, s, k_d2_assign<<<grid, D2_BLOCK, 0, s>>>(g->row_ptr, g->col_idx, g->nnz, n, colors,
                                                                       ctx->wl[cur], cnt + cur,
                                                                       gc_stream_value(seed, GC_TAG_COLOR, (uint32_t)r),
                                                                       (uint32_t)X, randx));
        GC_LAUNCHED();
        GC_TIMED(GC_K_DETECT, s, k_d2_detect<<<grid, D2_BLOCK, 0, s>>>(g->row_ptr, g->col_idx, g->nnz, n, colors,
                                                                       ctx->wl[cur], cnt + cur, prio_of(r),
                                                                       ctx->wl[nxt], cnt + nxt));
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
            if (st->round_degsum) st->round_degsum[i] = 0;
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

gc_status gc_d2_classes(gc_ctx *ctx, const gc_csr *g, int32_t *C, int32_t k, const int32_t *off_host, int seg_per_rank,
                        hipStream_t s) {
    for (int32_t r = 0; r < k; r++) {
        const int32_t a = off_host[seg_per_rank * r], b = off_host[seg_per_rank * r + seg_per_rank];
        if (b <= a) continue;
        GC_TIMED(GC_K_WALK, s, k_d2_class<<<d2_grid(ctx, b - a), D2_BLOCK, 0, s>>>(g->row_ptr, g->col_idx, g->nnz,
                                                                                   g->n, C, ctx->list, a, b));
        GC_LAUNCHED();
    }
    return GC_OK;
}

extern "C" gc_status gc_validate_d2(gc_ctx *ctx, const gc_csr *g, const int32_t *colors, int64_t *conflict_vertices,
                                    int64_t *uncolored, void *stream) {
    gc_status status = gc_check_graph_args(ctx, g);
    if (status) return status;
    if (g->n > 0 && !colors) return gc_fail(ctx, GC_ERR_ARG, "colors is NULL");
    hipStream_t s = (hipStream_t)stream;
    GC_HIP(hipSetDevice(ctx->device));
    int64_t nc = 0, nu = 0;
    if (g->n > 0) {
        int32_t maxdeg = 0;
        status = gc_graph_max_degree(ctx, g, s, &maxdeg);
        if (status) return status;
        if (maxdeg >= GC_D2_MAX_DEGREE)
            return gc_fail(ctx, GC_ERR_ARG, "distance-2 validation takes rows below %d entries", GC_D2_MAX_DEGREE);
        GC_HIP(hipMemsetAsync(ctx->scal + S_CONFLICTS, 0, 2 * 8, s));
        k_d2_validate<<<d2_grid(ctx, g->n), D2_BLOCK, 0, s>>>(g->row_ptr, g->col_idx, g->nnz, g->n, colors,
                                                              ctx->scal + S_CONFLICTS, ctx->scal + S_UNCOLORED);
        GC_LAUNCHED();
        status = gc_sync_scalars(ctx, s);
        if (status) return status;
        nc = (int64_t)ctx->hscal[S_CONFLICTS];
        nu = (int64_t)ctx->hscal[S_UNCOLORED];
    }
    if (conflict_vertices) *conflict_vertices = nc;
    if (uncolored) *uncolored = nu;
    return GC_OK;
}
