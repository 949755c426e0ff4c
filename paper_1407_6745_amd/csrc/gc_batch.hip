// gc_batch.hip - batched coloring: many independent graphs in one persistent
// launch.  Each workgroup pulls graph ids from an atomic ticket and runs the
// whole method on that graph (speculative initial coloring, section 2.2 with
// First Fit / Random-X Fit; then recoloring passes, section 3) with
// workgroup barriers only: no grid-wide synchronisation and no host round
// trip.  Small class tables live in LDS; larger ones fall back to a
// per-workgroup slice of global workspace.  The semantics are those of
// gc_init_color / gc_recolor, so colors match the single-graph calls made
// with the graph's seed.
#include "gc_internal.h"

#define BT 256            // threads per workgroup
#define BK 1024           // colors below BK keep their class tables in LDS
#define BBITS 1024        // LDS bitmap words for distinct counts (colors up to 32768)
#define BU 16             // neighbor ids in flight per lane in the row scans

// workspace slice layout per workgroup (int32 units)
struct BatchSlice {
    int32_t *wl0, *wl1, *list, *hist, *rank, *pi, *cls, *off, *cursor;
    uint32_t *bits;
};

__host__ __device__ inline int64_t batch_slice_ints(int32_t V, int32_t X) {
    int64_t CC = (int64_t)V + X + 64;
    int64_t ints = 3LL * V + 6 * (CC + 4) + CC / 32 + 4;
    return (ints + 63) / 64 * 64;
}

__device__ inline BatchSlice batch_slice(int32_t *base, int32_t V, int32_t X) {
    int64_t CC = (int64_t)V + X + 64;
    BatchSlice s;
    s.wl0 = base;
    s.wl1 = s.wl0 + V;
    s.list = s.wl1 + V;
    s.hist = s.list + V;
    s.rank = s.hist + (CC + 4);
    s.pi = s.rank + (CC + 4);
    s.cls = s.pi + (CC + 4);
    s.off = s.cls + (CC + 4);
    s.cursor = s.off + (CC + 4);
    s.bits = (uint32_t *)(s.cursor + (CC + 4));
    return s;
}

// Appends v to wl when pred holds, reserving slots on an LDS counter (one atomic per wavefront).
__device__ inline void wave_push_lds(int32_t *wl, int32_t *count, bool pred, int32_t v) {
    unsigned long long b = __ballot(pred);
    if (b == 0) return;
    int lane = __lane_id();
    int leader = __ffsll((long long)b) - 1;
    int32_t base = 0;
    if (lane == leader) base = atomicAdd(count, (int32_t)__popcll(b));
    base = __shfl(base, leader);
    if (pred) wl[base + __popcll(b & ((1ull << lane) - 1))] = v;
}

// distinct positive colors of C[0..n) (colors <= maxc), bits zero on entry and on exit
__device__ int32_t block_distinct(const int32_t *C, int32_t n, int32_t maxc, uint32_t *bits, int32_t *lds) {
    for (int32_t v = threadIdx.x; v < n; v += BT) {
        int32_t c = C[v];
        if (c > 0 && c <= maxc) atomicOr(&bits[(c - 1) >> 5], 1u << ((c - 1) & 31));
    }
    __syncthreads();
    int32_t words = (maxc + 31) >> 5, cnt = 0;
    for (int32_t i = threadIdx.x; i < words; i += BT) {
        cnt += __popc(bits[i]);
        bits[i] = 0;
    }
    int32_t tot;
    (void)block_exclusive_scan(cnt, &tot, lds);
    return tot;
}

// Speculative initial coloring of one graph by one workgroup.  Returns rounds
// run; *status = GC_ERR_NOT_CONVERGED when max_rounds stops it.
__device__ int32_t block_init(const int32_t *rp, const int32_t *col, int64_t nnz, int32_t n, int32_t *C,
                              int32_t *wl0, int32_t *wl1, bool randx, uint32_t X, uint64_t seed, int32_t max_rounds,
                              int32_t *sh_cnt, int32_t *status) {
    if (threadIdx.x == 0) { sh_cnt[0] = 0; sh_cnt[1] = 0; }
    __syncthreads();
    {
        // round 0: tentative colors are functions of the vertex ids alone
        const uint32_t sp = (uint32_t)(gc_mix64(seed + GC_GOLDEN * ((uint64_t)GC_TAG_PRIO << 32)) >> 32);
        const uint32_t sc = (uint32_t)(gc_mix64(seed + GC_GOLDEN * ((uint64_t)GC_TAG_COLOR << 32)) >> 32);
        for (int32_t base = 0; base < n; base += BT) {
            int32_t v = base + (int32_t)threadIdx.x;
            bool lose = false;
            if (v < n) {
                int32_t e0, e1;
                row_range(rp, v, nnz, e0, e1);
                uint32_t tv = randx ? gc_pick(sc, v, X) : 0u;
                uint32_t pv = gc_prio(sp, v);
                for (int32_t eb = e0; eb < e1 && !lose; eb += BU) {
                    int32_t w[BU];
#pragma unroll
                    for (int u = 0; u < BU; u++) w[u] = eb + u < e1 ? col[eb + u] : -1;
#pragma unroll
                    for (int u = 0; u < BU; u++) {
                        if ((uint32_t)w[u] >= (uint32_t)n) continue;
                        const uint32_t tw = randx ? gc_pick(sc, w[u], X) : 0u;
                        if (tw == tv && gc_prio(sp, w[u]) > pv) lose = true;
                    }
                }
                int32_t t = (int32_t)tv + 1;
                C[v] = lose ? -t : t;
            }
            wave_push_lds(wl0, &sh_cnt[0], lose, v);
        }
    }
    __syncthreads();
    int32_t rounds = 1, cur = 0;
    for (;;) {
        const int32_t cnt = sh_cnt[cur];
        if (cnt == 0) break;
        if (max_rounds > 0 && rounds == max_rounds) { *status = GC_ERR_NOT_CONVERGED; break; }
        if (rounds > n) { *status = GC_ERR_DEVICE; break; }  // each round commits >= 1 vertex: unreachable
        const int32_t nxt = cur ^ 1;
        int32_t *win = cur ? wl1 : wl0, *wout = cur ? wl0 : wl1;
        __syncthreads();  // every thread has read sh_cnt[cur] before it is reset below on the next round
        if (threadIdx.x == 0) sh_cnt[nxt] = 0;
        const uint32_t sc = (uint32_t)(gc_mix64(seed + GC_GOLDEN * (((uint64_t)GC_TAG_COLOR << 32) | (uint32_t)rounds)) >> 32);
        const uint32_t sp = (uint32_t)(gc_mix64(seed + GC_GOLDEN * (((uint64_t)GC_TAG_PRIO << 32) | (uint32_t)rounds)) >> 32);
        for (int32_t i = threadIdx.x; i < cnt; i += BT) {
            int32_t v = win[i];
            int32_t e0, e1;
            row_range(rp, v, nnz, e0, e1);
            C[v] = -select_color_lane<BU>(col, e0, e1, C, n, randx ? gc_pick(sc, v, X) : 0u);
        }
        __syncthreads();
        for (int32_t base = 0; base < cnt; base += BT) {
            int32_t i = base + (int32_t)threadIdx.x;
            bool lose = false;
            int32_t v = 0;
            if (i < cnt) {
                v = win[i];
                int32_t t = -C[v];
                int32_t e0, e1;
                row_range(rp, v, nnz, e0, e1);
                uint32_t pv = gc_prio(sp, v);
                for (int32_t eb = e0; eb < e1 && !lose; eb += BU) {
                    int32_t w[BU], cw[BU];
#pragma unroll
                    for (int u = 0; u < BU; u++) w[u] = eb + u < e1 ? col[eb + u] : -1;
#pragma unroll
                    for (int u = 0; u < BU; u++) cw[u] = (uint32_t)w[u] < (uint32_t)n ? C[w[u]] : 0;
#pragma unroll
                    for (int u = 0; u < BU; u++)
                        if ((uint32_t)w[u] < (uint32_t)n && (cw[u] == t || cw[u] == -t) && gc_prio(sp, w[u]) > pv)
                            lose = true;
                }
                if (!lose) C[v] = t;
            }
            wave_push_lds(wout, &sh_cnt[nxt], lose, v);
        }
        __syncthreads();
        cur = nxt;
        rounds++;
    }
    __syncthreads();
    return rounds;
}

// One recoloring pass of one graph by one workgroup; returns the new color count.
__device__ int32_t block_pass(const int32_t *rp, const int32_t *col, int64_t nnz, int32_t n, int32_t *C, int32_t perm,
                              uint32_t s_perm, const BatchSlice &ws, int32_t *l_hist, int32_t *l_rank, int32_t *l_pi,
                              int32_t *l_cls, int32_t *l_off, int32_t *l_cursor, int32_t *lds) {
    int32_t mx = 0;
    for (int32_t v = threadIdx.x; v < n; v += BT) mx = max(mx, C[v]);
    const int32_t maxc = block_max_i32(mx, lds);
    const bool small = maxc < BK;
    int32_t *hist = small ? l_hist : ws.hist;
    int32_t *rank = small ? l_rank : ws.rank;
    int32_t *pi = small ? l_pi : ws.pi;
    int32_t *cls = small ? l_cls : ws.cls;
    int32_t *off = small ? l_off : ws.off;
    int32_t *cursor = small ? l_cursor : ws.cursor;
    for (int32_t v = threadIdx.x; v < n; v += BT) {
        int32_t c = C[v];
        if (c >= 1) atomicAdd(&hist[c], 1);
    }
    __syncthreads();
    const int32_t k = block_class_order(maxc, perm, s_perm, hist, cls, pi, rank, off, cursor, lds);
    for (int32_t c = threadIdx.x; c <= maxc; c += BT) hist[c] = 0;
    for (int32_t v = threadIdx.x; v < n; v += BT) {
        int32_t c = C[v];
        if (c < 1) continue;
        int32_t s = rank[c];
        int32_t p = atomicAdd(&cursor[s], 1);
        ws.list[p] = v;
        C[v] = -(s + 1);
    }
    __syncthreads();
    int32_t newmax = 0;
    for (int32_t s = 0; s < k; s++) {
        const int32_t a = off[s], b = off[s + 1];
        for (int32_t i = a + (int32_t)threadIdx.x; i < b; i += BT) {
            int32_t v = ws.list[i];
            int32_t e0, e1;
            row_range(rp, v, nnz, e0, e1);
            int32_t c = select_color_lane<BU>(col, e0, e1, C, n, 0u);
            C[v] = c;
            newmax = max(newmax, c);
        }
        __syncthreads();
    }
    return block_max_i32(newmax, lds);
}

__global__ void __launch_bounds__(BT) k_batch(int32_t G, const int64_t *__restrict__ vtx_off,
                                              const int64_t *__restrict__ edge_off, const int32_t *__restrict__ row_ptr,
                                              const int32_t *__restrict__ col_idx, int32_t randx, uint32_t X,
                                              int32_t perm, int32_t passes, uint64_t base_seed, int32_t max_rounds,
                                              int32_t V, int32_t *colors, gc_graph_stats *per_graph, int32_t *ws_all,
                                              int64_t ws_ints, unsigned long long *ticket,
                                              const int32_t *__restrict__ order) {
    __shared__ int32_t sh[4];
    __shared__ int32_t lds[32];
    __shared__ int32_t l_hist[BK + 1], l_rank[BK + 1], l_pi[BK + 1], l_cls[BK + 1], l_off[BK + 2], l_cursor[BK + 1];
    __shared__ uint32_t l_bits[BBITS];
    for (int i = threadIdx.x; i <= BK; i += BT) l_hist[i] = 0;
    for (int i = threadIdx.x; i < BBITS; i += BT) l_bits[i] = 0;
    const BatchSlice ws = batch_slice(ws_all + (int64_t)blockIdx.x * ws_ints, V, (int32_t)X);
    __syncthreads();
    for (;;) {
        if (threadIdx.x == 0) {
            const int32_t t = (int32_t)atomicAdd(ticket, 1ull);
            sh[0] = (t < G && order) ? order[t] : t;  // the graph of ticket t
        }
        __syncthreads();
        const int32_t g = sh[0];
        __syncthreads();
        if (g >= G) break;
        const int64_t v0 = vtx_off[g], n64 = vtx_off[g + 1] - v0;
        const int64_t eo = edge_off[g], nnz = edge_off[g + 1] - eo;
        int32_t status = GC_OK, rounds = 0, c_init = 0, c_final = 0;
        if (n64 < 0 || n64 > V || nnz < 0 || nnz >= 2147483647LL) {
            status = GC_ERR_ARG;
        } else if (n64 > 0) {
            const int32_t n = (int32_t)n64;
            const int32_t *rp = row_ptr + v0 + g;
            const int32_t *col = col_idx + eo;
            int32_t *C = colors + v0;
            const uint64_t seed = gc_mix64(base_seed + GC_GOLDEN * (((uint64_t)GC_TAG_GRAPH << 32) | (uint32_t)g));
            rounds = block_init(rp, col, nnz, n, C, ws.wl0, ws.wl1, randx != 0, X, seed, max_rounds, &sh[1], &status);
            int32_t mx = 0;
            for (int32_t v = threadIdx.x; v < n; v += BT) mx = max(mx, C[v]);
            const int32_t maxc = block_max_i32(mx, lds);
            c_init = block_distinct(C, n, maxc, maxc <= BBITS * 32 ? l_bits : ws.bits, lds);
            c_final = c_init;
            if (status == GC_OK) {
                for (int32_t p = 0; p < passes; p++) {
                    const uint32_t s_perm = (uint32_t)(gc_mix64(seed + GC_GOLDEN * (((uint64_t)GC_TAG_PERM << 32) | (uint32_t)p)) >> 32);
                    c_final = block_pass(rp, col, nnz, n, C, perm, s_perm, ws, l_hist, l_rank, l_pi, l_cls, l_off, l_cursor, lds);
                }
            }
        }
        if (threadIdx.x == 0 && per_graph) {
            gc_graph_stats st;
            st.rounds = rounds;
            st.colors_init = c_init;
            st.colors_final = c_final;
            st.status = status;
            per_graph[g] = st;
        }
        __syncthreads();
    }
}

// Graph order for the tickets: graphs by decreasing entry count, ties by
// increasing id (one workgroup, bitonic sort of G <= ORDER_MAX keys in LDS).
// Only the schedule changes: every graph's colors are the same in any order.
#define ORDER_MAX 8192
__global__ void __launch_bounds__(1024) k_batch_order(int32_t G, const int64_t *__restrict__ edge_off,
                                                      int32_t *__restrict__ order) {
    __shared__ unsigned long long key[ORDER_MAX];
    int32_t P = 1;
    while (P < G) P <<= 1;
    for (int32_t i = threadIdx.x; i < P; i += blockDim.x) {
        if (i < G) {
            int64_t e = edge_off[i + 1] - edge_off[i];
            e = e < 0 ? 0 : (e > 0x7FFFFFFF ? 0x7FFFFFFF : e);
            key[i] = ((unsigned long long)(0x7FFFFFFFu - (uint32_t)e) << 32) | (uint32_t)i;  // ascending = largest first
        } else {
            key[i] = ~0ull;
        }
    }
    __syncthreads();
    for (int32_t k = 2; k <= P; k <<= 1) {
        for (int32_t j = k >> 1; j > 0; j >>= 1) {
            for (int32_t i = threadIdx.x; i < P; i += blockDim.x) {
                const int32_t l = i ^ j;
                if (l > i) {
                    const unsigned long long a = key[i], c = key[l];
                    const bool up = (i & k) == 0;
                    if ((a > c) == up) {
                        key[i] = c;
                        key[l] = a;
                    }
                }
            }
            __syncthreads();
        }
    }
    for (int32_t i = threadIdx.x; i < G; i += blockDim.x) order[i] = (int32_t)(uint32_t)key[i];
}

static gc_status gc_batch_color_impl(gc_ctx *ctx, const gc_batch_csr *b, int32_t select, int32_t X, int32_t perm,
                                    int32_t passes, uint64_t base_seed, int32_t max_rounds, int32_t max_vertices_per_graph,
                                    int32_t *colors, gc_graph_stats *per_graph, void *stream) {
    if (!ctx) return GC_ERR_ARG;
    if (!b) return gc_fail(ctx, GC_ERR_ARG, "batch is NULL");
    if (b->num_graphs < 0) return gc_fail(ctx, GC_ERR_ARG, "num_graphs < 0");
    if (select != GC_FIRST_FIT && select != GC_RANDOM_X) return gc_fail(ctx, GC_ERR_ARG, "select must be GC_FIRST_FIT or GC_RANDOM_X");
    if (select == GC_RANDOM_X && (X < 1 || X > GC_MAX_X)) return gc_fail(ctx, GC_ERR_ARG, "X must be in [1, %d]", GC_MAX_X);
    if (perm < 0 || perm > 3) return gc_fail(ctx, GC_ERR_ARG, "perm must be in [0, 3]");
    if (passes < 0 || max_rounds < 0) return gc_fail(ctx, GC_ERR_ARG, "passes and max_rounds must be >= 0");
    if (max_vertices_per_graph < 0 || max_vertices_per_graph > 2147483647 - GC_MAX_X - 4096)
        return gc_fail(ctx, GC_ERR_ARG, "max_vertices_per_graph out of range");
    if (b->num_graphs == 0) return GC_OK;
    if (!b->vtx_off || !b->edge_off || !b->row_ptr || !colors) return gc_fail(ctx, GC_ERR_ARG, "NULL batch array");
    if (select == GC_FIRST_FIT) X = 1;
    hipStream_t s = (hipStream_t)stream;
    GC_HIP(hipSetDevice(ctx->device));
    const int32_t V = max_vertices_per_graph > 0 ? max_vertices_per_graph : 1;
    const int64_t slice = batch_slice_ints(V, X);
    int grid = ctx->num_cu * (ctx->tune.batch_wg_per_cu > 0 ? ctx->tune.batch_wg_per_cu : 4);
    if (grid > b->num_graphs) grid = b->num_graphs;
    const int32_t *order = nullptr;
    if (ctx->tune.batch_order == 1 && b->num_graphs <= ORDER_MAX) {
        if (b->num_graphs > ctx->border_cap) {
            GC_HIP(hipStreamSynchronize(s));
            if (ctx->border) { GC_HIP(hipFree(ctx->border)); ctx->border = nullptr; ctx->border_cap = 0; }
            if (hipMalloc((void **)&ctx->border, (size_t)ORDER_MAX * 4) != hipSuccess)
                return gc_fail(ctx, GC_ERR_OOM, "batch graph order");
            ctx->border_cap = ORDER_MAX;
        }
        GC_TIMED(GC_K_OTHER, s, k_batch_order<<<1, 1024, 0, s>>>(b->num_graphs, b->edge_off, ctx->border));
        GC_LAUNCHED();
        order = ctx->border;
    }
    const int64_t need = slice * 4 * grid;
    if (need > ctx->bws_bytes) {
        GC_HIP(hipStreamSynchronize(s));
        if (ctx->bws) { GC_HIP(hipFree(ctx->bws)); ctx->bws = nullptr; ctx->bws_bytes = 0; }
        if (hipMalloc((void **)&ctx->bws, (size_t)need) != hipSuccess)
            return gc_fail(ctx, GC_ERR_OOM, "batch workspace of %lld bytes", (long long)need);
        ctx->bws_bytes = need;
        ctx->bws_layout = -1;  // zeroed below
    }
    // The global class tables of a slice (used when a graph has >= BK colors)
    // must be zero on entry; every pass leaves them zero, but only for the
    // slice layout it ran with: when (V, X) move the layout, the tables would
    // lie on old worklist data, so the workspace is cleared again.
    const int64_t layout = ((int64_t)V << 16) | X;  // X <= GC_MAX_X < 2^16
    if (ctx->bws_layout != layout) {
        GC_HIP(hipMemsetAsync(ctx->bws, 0, (size_t)ctx->bws_bytes, s));
        ctx->bws_layout = layout;
    }
    GC_HIP(hipMemsetAsync(ctx->scal + S_TICKET, 0, 8, s));
    GC_TIMED(GC_K_BATCH, s, k_batch<<<grid, BT, 0, s>>>(b->num_graphs, b->vtx_off, b->edge_off, b->row_ptr, b->col_idx, select == GC_RANDOM_X,
                                (uint32_t)X, perm, passes, base_seed, max_rounds, V, colors, per_graph, ctx->bws, slice,
                                ctx->scal + S_TICKET, order));
    GC_LAUNCHED();
    return GC_OK;
}

// Public entry points: the implementations above, with any sticky device
// failure harvested on the way reported in the returned status.
extern "C" gc_status gc_batch_color(gc_ctx *ctx, const gc_batch_csr *b, int32_t select, int32_t X, int32_t perm,
                                    int32_t passes, uint64_t base_seed, int32_t max_rounds, int32_t max_vertices_per_graph,
                                    int32_t *colors, gc_graph_stats *per_graph, void *stream) {
    return gc_report(ctx, gc_batch_color_impl(ctx, b, select, X, perm, passes, base_seed, max_rounds, max_vertices_per_graph, colors, per_graph, stream));
}
