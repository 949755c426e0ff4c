// gc_recolor.hip - one iterated-greedy recoloring pass (section 2.1,
// Culberson's Iterated Greedy; section 3, synchronous recoloring RC with the
// RV / NI / ND / RAND class permutations).
//
// Steps on the device:
//   1. class histogram of the input colors (workgroup-private in LDS) and
//      the min / max color;
//   2. class order: one workgroup compacts the non-empty classes, orders
//      them, and writes the rank of every color and the start offset of every
//      rank in the grouped vertex list (exclusive scan of the class sizes);
//   3. scatter: vertices grouped by rank (counting sort, per-workgroup
//      reservation of each class's range), and the output array initialised
//      to -(rank + 1): negative means "not yet recolored in this pass";
//   4. class walk: ranks in order; every vertex of the current class takes
//      the smallest positive color not held by a recolored neighbor.
#include "gc_internal.h"

#define HIST_LDS 4096   // colors below this use the workgroup-private histogram
#define PERM_THREADS 1024
#define SCATTER_BINS 1024
#define SCATTER_ITEMS 4

__global__ void k_hist(int32_t n, const int32_t *__restrict__ Cin, int32_t ccap, int32_t *__restrict__ hist,
                       unsigned long long *scal) {
    __shared__ int32_t h[HIST_LDS];
    for (int i = threadIdx.x; i < HIST_LDS; i += blockDim.x) h[i] = 0;
    __syncthreads();
    int32_t mx = 0, mn = 0x7fffffff;
    bool bad = false;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += stride) {
        int32_t c = Cin[v];
        mx = max(mx, c);
        mn = min(mn, c);
        if (c < 1 || c > ccap) { bad = true; continue; }
        if (c < HIST_LDS) atomicAdd(&h[c], 1);
        else atomicAdd(&hist[c], 1);
    }
    __syncthreads();
    for (int i = threadIdx.x; i < HIST_LDS; i += blockDim.x)
        if (h[i]) atomicAdd(&hist[i], h[i]);
    mx = wave_max_i32(mx);
    mn = wave_min_i32(mn);
    unsigned long long anybad = __ballot(bad);
    if (__lane_id() == 0) {
        atomicMax((int *)&scal[S_MAXC], mx);
        atomicMin((int *)&scal[S_MINC], mn);
        if (anybad) atomicOr(&scal[S_ERR], 1ull);
    }
}

// Class order (one workgroup of PERM_THREADS), global-memory arrays.
__global__ void __launch_bounds__(PERM_THREADS) k_class_order(int32_t ccap, int32_t perm, uint32_t s_perm,
                                                               int32_t *hist, int32_t *cls, int32_t *pi, int32_t *rank,
                                                               int32_t *off, int32_t *cursor, unsigned long long *scal) {
    __shared__ int32_t lds[32];
    int32_t maxc = (int32_t)scal[S_MAXC];
    if (maxc > ccap) maxc = ccap;
    int32_t k = block_class_order(maxc, perm, s_perm, hist, cls, pi, rank, off, cursor, lds);
    if (threadIdx.x == 0) scal[S_K] = (unsigned long long)k;
}

// Counting-sort scatter: one tile of SCATTER_ITEMS * blockDim vertices per
// workgroup; ranks below SCATTER_BINS reserve their range once per workgroup.
__global__ void k_scatter(int32_t n, const int32_t *Cin, int32_t *Cout, int32_t ccap, const int32_t *__restrict__ rank,
                          int32_t *__restrict__ cursor, int32_t *__restrict__ list, const unsigned long long *__restrict__ scal) {
    __shared__ int32_t cnt[SCATTER_BINS];
    __shared__ int32_t basepos[SCATTER_BINS];
    const int32_t k = (int32_t)scal[S_K];
    const int32_t bins = k < SCATTER_BINS ? k : SCATTER_BINS;
    for (int i = threadIdx.x; i < bins; i += blockDim.x) cnt[i] = 0;
    __syncthreads();
    const int64_t tile = (int64_t)blockIdx.x * blockDim.x * SCATTER_ITEMS;
    int32_t rk[SCATTER_ITEMS], loc[SCATTER_ITEMS];
#pragma unroll
    for (int it = 0; it < SCATTER_ITEMS; it++) {
        int64_t v = tile + (int64_t)it * blockDim.x + threadIdx.x;
        rk[it] = -1;
        loc[it] = -1;
        if (v < n) {
            int32_t c = Cin[v];
            if (c >= 1 && c <= ccap && k > 0) {
                int32_t s = rank[c];
                if ((uint32_t)s >= (uint32_t)k) s = k - 1;  // unreachable for a ranked color; keeps indices in bounds
                rk[it] = s;
                if (s < SCATTER_BINS) loc[it] = atomicAdd(&cnt[s], 1);
                else {
                    int32_t p = atomicAdd(&cursor[s], 1);
                    list[p] = (int32_t)v;
                    Cout[v] = -(s + 1);
                }
            } else {
                Cout[v] = 0;
            }
        }
    }
    __syncthreads();
    for (int i = threadIdx.x; i < bins; i += blockDim.x)
        if (cnt[i]) basepos[i] = atomicAdd(&cursor[i], cnt[i]);
    __syncthreads();
#pragma unroll
    for (int it = 0; it < SCATTER_ITEMS; it++) {
        int64_t v = tile + (int64_t)it * blockDim.x + threadIdx.x;
        if (loc[it] >= 0) {
            list[basepos[rk[it]] + loc[it]] = (int32_t)v;
            Cout[v] = -(rk[it] + 1);
        }
    }
}

// One class step: every vertex of rank s takes the smallest positive color
// not held by a neighbor (neighbors not yet recolored hold negative values).
__global__ void k_walk_class(const int32_t *__restrict__ rp, const int32_t *__restrict__ col, int64_t nnz, int32_t n,
                             int32_t *C, const int32_t *__restrict__ list, const int32_t *__restrict__ off, int32_t s) {
    const int32_t a = off[s], b = off[s + 1];
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = a + (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < b; i += stride) {
        int32_t v = list[i];
        int32_t e0, e1;
        row_range(rp, v, nnz, e0, e1);
        C[v] = select_color_lane(col, e0, e1, C, n, 0u);
    }
}

extern "C" gc_status gc_recolor(gc_ctx *ctx, const gc_csr *g, int32_t perm, uint64_t seed, int32_t pass,
                                const int32_t *colors_in, int32_t *colors_out, gc_stats *st, void *stream) {
    gc_status status = gc_check_graph_args(ctx, g);
    if (status) return status;
    if (perm < 0 || perm > 3) return gc_fail(ctx, GC_ERR_ARG, "perm must be in [0, 3]");
    if (pass < 0) return gc_fail(ctx, GC_ERR_ARG, "pass must be >= 0");
    if (g->n > 0 && (!colors_in || !colors_out)) return gc_fail(ctx, GC_ERR_ARG, "colors is NULL");
    hipStream_t s = (hipStream_t)stream;
    GC_HIP(hipSetDevice(ctx->device));
    const int32_t n = g->n;
    if (n == 0) {
        if (st) { st->rounds = 0; st->num_colors = 0; st->max_color = 0; st->k_classes = 0; st->losers_total = 0; }
        return GC_OK;
    }
    const int block = 256;
    GC_HIP(hipMemsetAsync(ctx->scal + S_ERR, 0, 8, s));
    GC_HIP(hipMemsetAsync(ctx->scal + S_MAXC, 0, 8, s));
    GC_HIP(hipMemsetAsync(ctx->scal + S_MINC, 0x7f, 4, s));
    GC_HIP(hipMemsetAsync((char *)(ctx->scal + S_MINC) + 4, 0, 4, s));
    k_hist<<<gc_grid(ctx, n, block), block, 0, s>>>(n, colors_in, ctx->ccap, ctx->hist, ctx->scal);
    GC_LAUNCHED();
    k_class_order<<<1, PERM_THREADS, 0, s>>>(ctx->ccap, perm, gc_stream_value(seed, GC_TAG_PERM, (uint32_t)pass),
                                            ctx->hist, (int32_t *)ctx->keys, ctx->pi, ctx->rank, ctx->off, ctx->cursor, ctx->scal);
    GC_LAUNCHED();
    int64_t tiles = ((int64_t)n + block * SCATTER_ITEMS - 1) / (block * SCATTER_ITEMS);
    k_scatter<<<(unsigned)tiles, block, 0, s>>>(n, colors_in, colors_out, ctx->ccap, ctx->rank, ctx->cursor, ctx->list, ctx->scal);
    GC_LAUNCHED();
    status = gc_sync_scalars(ctx, s);
    if (status) return status;
    if (ctx->hscal[S_ERR]) return gc_fail(ctx, GC_ERR_COLORING, "input color outside [1, %d]", ctx->ccap);
    const int32_t k = (int32_t)ctx->hscal[S_K];
    for (int32_t r = 0; r < k; r++) {
        k_walk_class<<<gc_grid(ctx, n, block), block, 0, s>>>(g->row_ptr, g->col_idx, g->nnz, n, colors_out, ctx->list, ctx->off, r);
        GC_LAUNCHED();
    }
    if (st) {
        status = gc_count_device(ctx, n, colors_out, s, true);
        if (status) return status;
        status = gc_sync_scalars(ctx, s);
        if (status) return status;
        st->rounds = 0;
        st->losers_total = 0;
        st->k_classes = k;
        st->num_colors = (int32_t)ctx->hscal[S_NUMC];
        st->max_color = (int32_t)ctx->hscal[S_MAXC];
    }
    return GC_OK;
}
