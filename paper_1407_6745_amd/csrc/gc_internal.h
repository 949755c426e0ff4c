// gc_internal.h - shared internals of libgc (HIP, gfx950): context layout,
// device helpers (hash, wavefront primitives, first-fit selection).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stdarg.h>
#include <stdio.h>

#include "gc.h"

// ---------------------------------------------------------------------------
// context
// ---------------------------------------------------------------------------

// Recoloring histogram: colors below GC_HIST_LDS are counted in workgroup
// LDS and flushed into one of GC_HIST_COPIES copies (bin-0 counts, then bin-1
// counts, GC_HIST_LDS entries per copy), chosen by the histogram tile, so that
// concurrent flushes land on different cache lines.  A third array holds, per
// copy and color, the copy's cursor inside the color's bin-0 segment (relative
// to the segment start): the copies fill consecutive parts of the segment.
// The counts are zero between calls; the cursors are rewritten every pass.
#define GC_HIST_LDS 4096
#define GC_HIST_COPIES 16
#define GC_HCOPY_INTS (3 * GC_HIST_COPIES * GC_HIST_LDS)
#define GC_SYNC_BYTES 4096  // grid-barrier counters, one 128-byte line each

// Device scalar slots (int64 each) in ctx->scal.
enum {
    S_WCOUNT0 = 0,   // worklist length, buffer 0
    S_WCOUNT1 = 1,   // worklist length, buffer 1
    S_MAXC = 2,      // max color seen
    S_MINC = 3,      // min color seen
    S_ERR = 4,       // error flags of the current pass (bit 0: color out of range, bit 1: wait limit,
                     // bit 2: not resident); cleared at the start of every pass
    S_CONFLICTS = 5,
    S_UNCOLORED = 6,
    S_K = 7,         // number of non-empty classes
    S_NUMC = 8,      // distinct colors
    S_GRAPHERR = 9,  // csr check failures
    S_TICKET = 10,   // work ticket of persistent kernels
    S_DONE = 11,
    S_MAXDEG = 12,   // longest row of the graph
    S_PLAN = 13,     // split plans of the initial coloring, two rounds (13, 14): rows << 32 | chunks
    S_WL = 16,       // initial coloring: 4 worklist counts + two degree-sum slots (16..21)
    S_SUM = 24,      // checksum of a color array (autotuning)
    S_NLONG = 25,    // long rows of the initial coloring's masks
    S_FAR = 26,      // adjacency entries (u, w) with |u - w| >= GC_NEAR (locality of a graph)
    S_NZSEG = 27,    // recoloring: segments with at least one work chunk (their list is ctx->segnz)
    S_REC = 64,      // rounds queued ahead (64..127): input size, previous round's degree sum
    S_VLONG = 35,    // validation: (row, chunk) pairs of long rows listed
    S_TAIL = 36,     // initial coloring's persistent tail launch (36..45): check-in, decision, barrier count and
                     // generation, two list counts, two degree sums, rounds run, status
    S_STICKY = 34,   // device failures kept until a synchronizing call reports them (bit 1: a walk wait
                     // gave up, bit 2: walk workgroups not all resident); never cleared by a pass
    S_COUNT = 128
};

struct gc_ctx {
    int device;
    int num_cu;              // compute units this context's launches are sized for (the cu_count knob, else all)
    int dev_cu;              // compute units of the device
    int64_t max_n;
    int64_t max_nnz;
    int32_t ccap;            // largest color any buffer indexed by color can hold
    gc_tuning tune;
    // device workspace
    int32_t *wl[4];          // init worklists (max_n each): [2 * buffer + bin]
    int32_t *list;           // recolor: vertices grouped by class rank (max_n + padding)
    int2 *rows;              // recolor: row range of list[i] (same layout)
    int32_t *hist;           // class sizes by color (ccap + 2), all zero between calls
    int32_t *histw;          // per color: vertices in the wavefront-per-vertex degree bin; zero between calls
    int32_t *coff;           // recolor: work-chunk offsets per (rank, bin) segment (3 * ccap + 4)
    int32_t *segnz;          // recolor: the segments with work chunks, in order (3 * ccap + 4)
    int32_t *hist_s;         // per color: vertices of the split bin; zero between calls
    int32_t *hist_sc;        // per color: work chunks of those vertices; zero between calls
    int32_t *hcopy;          // recoloring's histogram copies and per-copy scatter cursors (GC_HCOPY_INTS)
    int32_t *sbase;          // per rank: first hub slot of the rank's split segment (ccap + 2)
    int32_t *hsub;           // per list slot of a split row: its first chunk inside the segment (max_n + 64)
    unsigned long long *hub_bits;  // per hub slot: HUB_WORDS color-mask words, zero between calls
    int32_t *hub_cnt;        // per hub slot: finished chunks, zero between calls
    void *shadow;            // recoloring walk: compact copy of the colors (2 bytes per vertex)
    int32_t *hub_v;          // initial coloring: per hub slot, the long row's vertex
    int32_t *hub_first;      // initial coloring: per hub slot, its first chunk
    int64_t hub_cap;         // hub slots allocated
    int walk_blocks;         // co-resident workgroups of the last persistent walk launched (0 = none yet)
    int walk_blocks_v[260];  // measured per walk variant (4 * group + 2 * options + full); 0 = not measured
    // longest row of the last graph seen by the recoloring (keyed by its arrays and sizes)
    const void *deg_key_rp, *deg_key_col;
    int64_t deg_key_n, deg_key_nnz;
    int32_t deg_max;
    double deg_far;          // fraction of its entries with |u - w| >= GC_NEAR
    int64_t deg_far_n;       // how many entries that is
    int deg_known;           // set once a graph has been analysed
    int32_t *rank;           // rank of a color in the class order (ccap + 2)
    int32_t *pi;             // class order (ccap + 2)
    int32_t *off;            // list offsets per (rank, bin) segment (3 * ccap + 4)
    int32_t *cursor;         // scatter cursors per segment (3 * ccap + 4)
    uint64_t *keys;          // sort keys (ccap + 2)
    uint32_t *bitmap;        // distinct-color bitmap, all zero between calls
    int64_t bitmap_bits;
    int64_t *round_stats;    // 2 * (max_n + 2): |W_r|, degree sum of W_r
    unsigned long long *scal;  // S_COUNT device scalars
    unsigned long long *hscal; // pinned host mirror
    struct gc_timer *timer;  // kernel timing (NULL when off)
    unsigned long long *d2mask;  // distance-2 coloring: per-vertex color masks (allocated on first use, max_n * 2 words)
    int32_t *bws;            // batched coloring: per-workgroup workspace (grown on demand)
    int32_t *longidx;        // initial coloring: index of each long row's mask (-1: short row), max_n
    unsigned long long *fm;  // initial coloring: committed-color masks of the long rows, grown on demand
    int64_t fm_cap;          // masks allocated
    int32_t *act;            // initial coloring: active lists of the split rows, two buffers of act_cap entries
    int64_t act_cap;
    int32_t *alen;           // their lengths, two arrays of alen_cap (by long-row index)
    int64_t alen_cap;
    int32_t *border;         // batched coloring: graph order (largest first), grown on demand
    int64_t border_cap;
    int64_t bws_bytes;
    int64_t bws_layout;      // batched coloring: (V << 16 | X) the workspace slices were last laid out for
    unsigned long long sticky;  // device failures harvested from S_STICKY, not yet reported
    unsigned long long *trace;  // class-completion trace of the last persistent walk (tuning.trace), on demand
    unsigned long long *sync;   // grid-barrier counters of the initial coloring's tail launch (GC_SYNC_BYTES)
    int32_t *vround;            // during gc_init_color_rounds: the caller's per-vertex commit rounds, else NULL
    char err[512];
};

// Records a message and returns the status.
gc_status gc_fail(gc_ctx *ctx, gc_status s, const char *fmt, ...);

#define GC_HIP(call)                                                                   \
    do {                                                                               \
        hipError_t e_ = (call);                                                        \
        if (e_ != hipSuccess)                                                          \
            return gc_fail(ctx, GC_ERR_DEVICE, "%s failed: %s", #call, hipGetErrorString(e_)); \
    } while (0)

#define GC_LAUNCHED()                                                                  \
    do {                                                                               \
        hipError_t e_ = hipGetLastError();                                             \
        if (e_ != hipSuccess)                                                          \
            return gc_fail(ctx, GC_ERR_DEVICE, "kernel launch failed: %s", hipGetErrorString(e_)); \
    } while (0)

// Kernel timing: events around a launch (no-ops unless timing is enabled).
void gc_time_begin(gc_ctx *ctx, int kind, hipStream_t s);
void gc_time_end(gc_ctx *ctx, int kind, hipStream_t s);

#define GC_TIMED(kind, stream, ...)        \
    do {                                  \
        gc_time_begin(ctx, kind, stream); \
        __VA_ARGS__;                      \
        gc_time_end(ctx, kind, stream);   \
    } while (0)

// Common argument checks for a single-graph call.
gc_status gc_check_graph_args(gc_ctx *ctx, const gc_csr *g);

// Host-side grid size for grid-stride kernels over `work` items.
int gc_grid(const gc_ctx *ctx, int64_t work, int block);

// Launch helpers shared between files (defined in gc_api.hip).
gc_status gc_count_device(gc_ctx *ctx, int32_t n, const int32_t *colors, hipStream_t s, bool reset_minmax);
// Copies the device scalars to the host mirror (synchronizes s) and moves
// any sticky device failure into ctx->sticky.
gc_status gc_sync_scalars(gc_ctx *ctx, hipStream_t s);
// Status a public call returns: st itself when it is an error, else
// GC_ERR_DEVICE (and the record cleared) when a sticky device failure was
// harvested, else GC_OK.
gc_status gc_report(gc_ctx *ctx, gc_status st);
// gc_validate / gc_validate_d2 without the sticky report (used by the input
// check of the recoloring calls).
gc_status gc_validate_impl(gc_ctx *ctx, const gc_csr *g, const int32_t *colors, int64_t *conflict_edges,
                           int64_t *uncolored, void *stream);
gc_status gc_validate_d2_impl(gc_ctx *ctx, const gc_csr *g, const int32_t *colors, int64_t *conflict_pairs,
                              int64_t *uncolored, void *stream);
// With the check_input knob: GC_ERR_COLORING unless colors is a proper
// coloring (distance `dist`) with every color >= 1; synchronizes.
gc_status gc_check_input_coloring(gc_ctx *ctx, const gc_csr *g, const int32_t *colors, void *stream, int dist);
// Longest row of g, computed once per graph (keyed by its arrays and sizes;
// it only picks kernel variants, never results).  Synchronizes the stream on
// a new graph.
gc_status gc_graph_max_degree(gc_ctx *ctx, const gc_csr *g, hipStream_t s, int32_t *out);
// Neighbor ids at least this far from the row's own id count as far: their
// colors lie outside the int32 window of 256 KB around the row's.
#define GC_NEAR 32768
// Fraction of g's adjacency entries that are far (computed with the longest row).
gc_status gc_graph_far_fraction(gc_ctx *ctx, const gc_csr *g, hipStream_t s, double *out);

// Speculative rounds over every vertex of g (arguments checked, n > 0):
// prank == NULL gives the initial coloring (hash priorities); a per-vertex
// class rank instead decides conflicts by rank (asynchronous recoloring).
gc_status gc_spec_rounds(gc_ctx *ctx, const gc_csr *g, int32_t select, int32_t X, uint64_t seed, int32_t max_rounds,
                         uint32_t flags, int32_t *colors, gc_stats *st, hipStream_t s, const int32_t *prank);

// Distance-2 coloring (gc_d2.hip): the speculative rounds over distance-2
// neighborhoods (arguments checked, n > 0), and the classes of one
// recoloring pass, class r being list[off_host[spr * r], off_host[spr * r + spr]).
gc_status gc_spec_rounds_d2(gc_ctx *ctx, const gc_csr *g, int32_t select, int32_t X, uint64_t seed, int32_t max_rounds,
                            uint32_t flags, int32_t *colors, gc_stats *st, hipStream_t s);
gc_status gc_d2_classes(gc_ctx *ctx, const gc_csr *g, int32_t *C, int32_t k, const int32_t *off_host, int spr,
                        hipStream_t s);
// Longest row accepted by the distance-2 calls: 64 rows of this length still
// sum below 2^31 entries.
#define GC_D2_MAX_DEGREE (1 << 25)

// Lanes per vertex of the recoloring walk: the walk_group knob, or when it is
// 0, 8 for graphs whose rows are all shorter than 64 entries (full = false)
// and the group knob otherwise.
// Automatic: 8 lanes per vertex for graphs whose rows are all under 64
// entries; 2 in the variant with split rows, whose graphs (skewed degrees)
// hold many rows of a few entries (more vertices per chunk; rows past
// deg_wave take a whole wavefront anyway).
inline int gc_walk_group(const gc_ctx *ctx, bool full) {
    return ctx->tune.walk_group ? ctx->tune.walk_group : (full ? 2 : 8);
}

// Mask words of one split row (colors 1 .. 64 * GC_HUB_WORDS).
#define GC_HUB_WORDS 64
// Hub slots for rows longer than deg_split (at most nnz / (deg_split + 1)
// rows), zeroed; grown on demand (synchronizes the stream when it grows).
gc_status gc_ensure_hub_slots(gc_ctx *ctx, int64_t nnz, int32_t deg_split, hipStream_t s);

// ---------------------------------------------------------------------------
// hash: counter-based randomness of the method (written from the published
// definitions of the SplitMix64 output function and the MurmurHash3 32-bit
// finalizer)
// ---------------------------------------------------------------------------

#define GC_GOLDEN 0x9E3779B97F4A7C15ULL
enum { GC_TAG_PRIO = 1, GC_TAG_COLOR = 2, GC_TAG_PERM = 3, GC_TAG_GRAPH = 4 };

__host__ __device__ inline uint64_t gc_mix64(uint64_t z) {
    z ^= z >> 30;
    z *= 0xBF58476D1CE4E5B9ULL;
    z ^= z >> 27;
    z *= 0x94D049BB133111EBULL;
    z ^= z >> 31;
    return z;
}

__host__ __device__ inline uint32_t gc_fmix32(uint32_t h) {
    h ^= h >> 16;
    h *= 0x85EBCA6BU;
    h ^= h >> 13;
    h *= 0xC2B2AE35U;
    h ^= h >> 16;
    return h;
}

// Per-round (or per-pass) stream value: the top 32 bits of
// mix64(seed + golden * (tag << 32 | counter)).  Uniform over a launch, so the
// host computes it once and passes it to the kernels.
__host__ __device__ inline uint32_t gc_stream_value(uint64_t seed, uint32_t tag, uint32_t counter) {
    return (uint32_t)(gc_mix64(seed + GC_GOLDEN * (((uint64_t)tag << 32) | counter)) >> 32);
}

// priority of v for a round with stream value s (larger wins; a bijection of v)
__device__ inline uint32_t gc_prio(uint32_t s, int32_t v) { return gc_fmix32(s ^ (uint32_t)v); }

// Random-X offset in [0, X): multiply-shift of the vertex hash
__device__ inline uint32_t gc_pick(uint32_t s, int32_t v, uint32_t X) {
    return (uint32_t)(((uint64_t)gc_fmix32(s ^ (uint32_t)v) * X) >> 32);
}

// Conflict priority of a round (the larger key keeps its color):
//   PRIO_HASH:    the hash of (seed, v, round) (s_prio holds the round's stream);
//   PRIO_RANK:    a per-vertex class rank, the earlier class first
//                 (asynchronous recoloring);
//   PRIO_LF:      Largest First: larger degree first, ties by round 0's hash;
//   PRIO_NATURAL: smaller vertex id first.
enum { PRIO_HASH = 0, PRIO_RANK = 1, PRIO_LF = 2, PRIO_NATURAL = 3 };

struct Prio {
    int mode;
    uint32_t s_prio;
    const int32_t *prank;  // PRIO_RANK
    const int32_t *rp;     // PRIO_LF: row pointers
};

__device__ inline uint64_t round_prio(const Prio &p, int32_t v) {
    switch (p.mode) {
        case PRIO_RANK: return ~(uint32_t)p.prank[v];
        case PRIO_LF: return ((uint64_t)(uint32_t)(p.rp[v + 1] - p.rp[v]) << 32) | gc_prio(p.s_prio, v);
        case PRIO_NATURAL: return 0xFFFFFFFFu - (uint32_t)v;
        default: return gc_prio(p.s_prio, v);
    }
}

// ---------------------------------------------------------------------------
// wavefront helpers (wave64)
// ---------------------------------------------------------------------------

__device__ inline unsigned long long wave_sum_u64(unsigned long long x) {
    for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o);
    return x;
}
__device__ inline int32_t wave_max_i32(int32_t x) {
    for (int o = 32; o > 0; o >>= 1) x = max(x, __shfl_xor(x, o));
    return x;
}
__device__ inline int32_t wave_min_i32(int32_t x) {
    for (int o = 32; o > 0; o >>= 1) x = min(x, __shfl_xor(x, o));
    return x;
}
__device__ inline uint64_t wave_or_u64(uint64_t x) {
    for (int o = 32; o > 0; o >>= 1) x |= __shfl_xor(x, o);
    return x;
}

// Appends v (where pred holds) to wl, one atomic per wavefront.  Every lane of
// the wavefront must call it (converged).
__device__ inline void wave_push(int32_t *wl, unsigned long long *count, bool pred, int32_t v) {
    unsigned long long b = __ballot(pred);
    if (b == 0) return;
    int lane = __lane_id();
    int leader = __ffsll((long long)b) - 1;
    unsigned int base = 0;
    if (lane == leader) base = (unsigned int)atomicAdd(count, (unsigned long long)__popcll(b));
    base = __shfl(base, leader);
    if (pred) wl[base + __popcll(b & ((1ull << lane) - 1))] = v;
}

// row range of v clamped to [0, nnz]
__device__ inline void row_range(const int32_t *__restrict__ rp, int32_t v, int64_t nnz, int32_t &e0, int32_t &e1) {
    int64_t a = rp[v], b = rp[v + 1];
    a = a < 0 ? 0 : (a > nnz ? nnz : a);
    b = b < a ? a : (b > nnz ? nnz : b);
    e0 = (int32_t)a;
    e1 = (int32_t)b;
}

// Position (0-based) of the (j+1)-th set bit of x; x must have more than j set bits.
__device__ inline uint32_t nth_set_bit(uint64_t x, uint32_t j) {
    for (uint32_t i = 0; i < j; i++) x &= x - 1;
    return (uint32_t)(__ffsll((long long)x) - 1);
}

// (j+1)-th smallest positive color absent from {C[w] > 0 : w in col[e0..e1)},
// one lane per vertex, 64 colors per window; UNR neighbor ids, then their UNR
// colors, in flight per lane.
template <int UNR = 8>
__device__ inline int32_t select_color_lane(const int32_t *__restrict__ col, int32_t e0, int32_t e1,
                                            const int32_t *C, int32_t n, uint32_t j) {
    uint32_t base = 0;
    for (;;) {
        uint64_t mask = 0;
        for (int32_t eb = e0; eb < e1; eb += UNR) {
            int32_t w[UNR], x[UNR];
#pragma unroll
            for (int u = 0; u < UNR; u++) w[u] = eb + u < e1 ? col[eb + u] : -1;
#pragma unroll
            for (int u = 0; u < UNR; u++) x[u] = (uint32_t)w[u] < (uint32_t)n ? C[w[u]] : 0;
#pragma unroll
            for (int u = 0; u < UNR; u++) {
                const uint32_t d = (uint32_t)x[u] - base - 1u;  // colors <= base (incl. <= 0) wrap to >= 64
                if (d < 64u) mask |= 1ull << d;
            }
        }
        uint64_t fr = ~mask;
        uint32_t cnt = (uint32_t)__popcll(fr);
        if (j < cnt) return (int32_t)(base + 1u + nth_set_bit(fr, j));
        j -= cnt;
        base += 64u;
    }
}

// ---------------------------------------------------------------------------
// workgroup-level routines (blockDim.x a multiple of 64, at most 1024)
// ---------------------------------------------------------------------------

// Exclusive scan of x across the workgroup; *total = sum.  lds: >= 17 ints.
// Every thread of the workgroup must call it.
__device__ inline int32_t block_exclusive_scan(int32_t x, int32_t *total, int32_t *lds) {
    const int lane = __lane_id(), wid = threadIdx.x >> 6, nw = blockDim.x >> 6;
    int32_t incl = x;
    for (int o = 1; o < 64; o <<= 1) {
        int32_t y = __shfl_up(incl, o);
        if (lane >= o) incl += y;
    }
    if (lane == 63) lds[wid] = incl;
    __syncthreads();
    if (threadIdx.x == 0) {
        int32_t acc = 0;
        for (int w = 0; w < nw; w++) { int32_t t = lds[w]; lds[w] = acc; acc += t; }
        lds[16] = acc;
    }
    __syncthreads();
    int32_t ex = incl - x + lds[wid];
    *total = lds[16];
    __syncthreads();
    return ex;
}

// Sum over the workgroup (every thread must call; lds: >= 16 words of 8 bytes).
__device__ inline unsigned long long block_sum_u64(unsigned long long x, unsigned long long *lds) {
    x = wave_sum_u64(x);
    const int wid = threadIdx.x >> 6, nw = blockDim.x >> 6;
    if (__lane_id() == 0) lds[wid] = x;
    __syncthreads();
    unsigned long long t = 0;
    for (int w = 0; w < nw; w++) t += lds[w];
    __syncthreads();
    return t;
}

__device__ inline int32_t block_min_i32(int32_t x, int32_t *lds) {
    x = wave_min_i32(x);
    const int wid = threadIdx.x >> 6, nw = blockDim.x >> 6;
    if (__lane_id() == 0) lds[wid] = x;
    __syncthreads();
    int32_t m = lds[0];
    for (int w = 1; w < nw; w++) m = min(m, lds[w]);
    __syncthreads();
    return m;
}

__device__ inline int32_t block_max_i32(int32_t x, int32_t *lds) {
    x = wave_max_i32(x);
    const int wid = threadIdx.x >> 6, nw = blockDim.x >> 6;
    if (__lane_id() == 0) lds[wid] = x;
    __syncthreads();
    int32_t m = lds[0];
    for (int w = 1; w < nw; w++) m = max(m, lds[w]);
    __syncthreads();
    return m;
}

// Class order of one recoloring pass, computed by one workgroup (section 3:
// RV, NI, ND and RAND permutations of the color classes).
//   hist[c]  : class sizes for c in [1, maxc] (left as they are);
//   cls      : scratch, receives the increasing list of non-empty colors;
//   pi[s]    : color visited at step s, s < k;
//   rank[c]  : s such that pi[s] = c (for present colors);
//   off[s]   : first slot of rank s in the grouped list (off[k] = total);
//   cursor[s]: copy of off[s] (scatter cursors); off / cursor may be NULL.
// Arrays may live in LDS or global memory.  Returns k (same in every thread).
// s_perm is the pass's stream value for the RAND shuffle.
__device__ inline int32_t block_class_order(int32_t maxc, int32_t perm, uint32_t s_perm, int32_t *hist, int32_t *cls,
                                            int32_t *pi, int32_t *rank, int32_t *off, int32_t *cursor, int32_t *lds) {
    // compact the non-empty classes in increasing color order
    int32_t k = 0;
    for (int32_t base = 1; base <= maxc; base += blockDim.x) {
        int32_t c = base + (int32_t)threadIdx.x;
        int32_t f = (c <= maxc && hist[c] > 0) ? 1 : 0;
        int32_t tot;
        int32_t ex = block_exclusive_scan(f, &tot, lds);
        if (f) cls[k + ex] = c;
        k += tot;
    }
    __syncthreads();
    if (perm == GC_PERM_REVERSE) {
        for (int32_t i = threadIdx.x; i < k; i += blockDim.x) pi[i] = cls[k - 1 - i];
    } else if (perm == GC_PERM_NONINC || perm == GC_PERM_NONDEC) {
        // position of class i = number of classes ordered before it by (size, color)
        const bool noninc = perm == GC_PERM_NONINC;
        for (int32_t i = threadIdx.x; i < k; i += blockDim.x) {
            int32_t ci = cls[i];
            int32_t si = hist[ci];
            int32_t r = 0;
            for (int32_t j = 0; j < k; j++) {
                int32_t cj = cls[j];
                int32_t sj = hist[cj];
                r += noninc ? (sj > si || (sj == si && cj < ci)) : (sj < si || (sj == si && cj < ci));
            }
            pi[r] = ci;
        }
    } else {
        for (int32_t i = threadIdx.x; i < k; i += blockDim.x) pi[i] = cls[i];
        __syncthreads();
        if (threadIdx.x == 0) {
            // Knuth shuffle from the top index down: swap i with a uniform index in [0, i]
            for (int32_t i = k - 1; i >= 1; i--) {
                uint32_t j = (uint32_t)(((uint64_t)gc_fmix32(s_perm ^ (uint32_t)i) * (uint32_t)(i + 1)) >> 32);
                int32_t t = pi[i];
                pi[i] = pi[j];
                pi[j] = t;
            }
        }
    }
    __syncthreads();
    int32_t acc = 0;
    for (int32_t base = 0; base < k; base += blockDim.x) {
        int32_t s = base + (int32_t)threadIdx.x;
        int32_t sz = 0;
        if (s < k) {
            int32_t c = pi[s];
            rank[c] = s;
            sz = hist[c];
        }
        int32_t tot;
        int32_t ex = block_exclusive_scan(sz, &tot, lds);
        if (s < k && off) { off[s] = acc + ex; cursor[s] = acc + ex; }
        acc += tot;
    }
    if (threadIdx.x == 0 && off) off[k] = acc;
    __syncthreads();
    return k;
}

// ---------------------------------------------------------------------------
// lane groups: G consecutive lanes (G a power of two dividing 64) work on one
// vertex; neighbor lists are read U entries per lane at a time so that U
// independent loads are in flight before the first wait.
// ---------------------------------------------------------------------------

#define GC_UNROLL 4

template <int G>
__device__ inline uint64_t group_or_u64(uint64_t x) {
    for (int o = G >> 1; o > 0; o >>= 1) x |= __shfl_xor(x, o);
    return x;
}

// true in every lane of the group if pred holds in any lane of it (whole wave must call)
template <int G>
__device__ inline bool group_any(bool pred) {
    unsigned long long b = __ballot(pred);
    if (G == 64) return b != 0;
    const unsigned long long gm = (G == 64) ? ~0ull : ((1ull << G) - 1ull);
    return ((b >> (__lane_id() & ~(G - 1))) & gm) != 0;
}

// For every valid lane: counter[key] is raised by the number of valid lanes
// holding that key (one LDS/global atomic per distinct key of the wave); the
// lane gets the old value plus the number of lower lanes with the same key.
__device__ inline int32_t wave_match_reserve(int32_t *counter, int32_t key, bool valid) {
    unsigned long long pending = __ballot(valid);
    const int lane = __lane_id();
    const unsigned long long below = (1ull << lane) - 1ull;
    int32_t pos = 0;
    while (pending) {
        const int leader = __ffsll((long long)pending) - 1;
        const int32_t k = __shfl(key, leader);
        const bool mine = valid && key == k;
        const unsigned long long same = __ballot(mine);
        int32_t base = 0;
        if (lane == leader) base = atomicAdd(&counter[k], (int32_t)__popcll(same));
        base = __shfl(base, leader);
        if (mine) pos = base + (int32_t)__popcll(same & below);
        pending &= ~same;
    }
    return pos;
}

// Same contract as wave_match_reserve for keys in [0, 2^bits): lanes with
// equal keys are found with `bits` ballots (no loop over distinct keys); the
// lowest lane of each key does the atomic and every lane reads its base back
// with one cross-lane read.  bits must be uniform over the wave.
__device__ inline int32_t wave_match_reserve_bits(int32_t *counter, int32_t key, bool valid, int bits) {
    unsigned long long same = __ballot(valid);
    for (int b = 0; b < bits; b++) {
        const bool bit = (key >> b) & 1;
        const unsigned long long bb = __ballot(bit);
        same &= bit ? bb : ~bb;
    }
    const int lane = __lane_id();
    int leader = valid ? __ffsll((long long)same) - 1 : lane;
    int32_t base = 0;
    if (valid && leader == lane) base = atomicAdd(&counter[key], (int32_t)__popcll(same));
    base = __shfl(base, leader);
    return valid ? base + (int32_t)__popcll(same & ((1ull << lane) - 1ull)) : 0;
}

// number of bits needed for keys in [0, count)
__device__ inline int key_bits(int32_t count) { return count <= 1 ? 0 : 32 - __clz(count - 1); }

// Block-aggregated append queue: entries collect in an LDS buffer and go to
// the global list in one copy per flush (one global atomic per flush).
// Every loop iteration may add at most blockDim.x entries.
#define GC_QCAP 2048

__device__ inline void bq_push(int32_t *lbuf, int32_t *lcnt, bool pred, int32_t v) {
    unsigned long long b = __ballot(pred);
    if (b == 0) return;
    const int lane = __lane_id();
    const int leader = __ffsll((long long)b) - 1;
    int32_t base = 0;
    if (lane == leader) base = atomicAdd(lcnt, (int32_t)__popcll(b));
    base = __shfl(base, leader);
    if (pred) lbuf[base + __popcll(b & ((1ull << lane) - 1ull))] = v;
}

// Call with every thread of the block, right after a __syncthreads().
// Flushes when `force` or when the buffer could not take one more iteration.
__device__ inline void bq_flush(int32_t *lbuf, int32_t *lcnt, int32_t *lbase, int32_t *gl, unsigned long long *gcount,
                                bool force) {
    const int32_t c = *lcnt;
    if (c == 0 || (!force && c <= GC_QCAP - (int32_t)blockDim.x)) return;
    if (threadIdx.x == 0) *lbase = (int32_t)atomicAdd(gcount, (unsigned long long)c);
    __syncthreads();
    const int32_t base = *lbase;
    for (int32_t i = threadIdx.x; i < c; i += blockDim.x) gl[base + i] = lbuf[i];
    __syncthreads();
    if (threadIdx.x == 0) *lcnt = 0;
    __syncthreads();
}

// (j+1)-th smallest positive color absent from {C[w] > 0 : w in row}, by a
// group of G lanes (group-uniform result).  Colors <= 0 are "no color".
// Colors read by agent-scope atomic loads: values written by other
// workgroups of the same launch, with no cache maintenance in between.
struct CoherentColors {
    const int32_t *p;
    __device__ int32_t operator[](int64_t i) const {
        return __hip_atomic_load(p + i, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
};

// In the helpers below, C is any color accessor: a pointer to int32 or int8
// colors, or CoherentColors.
template <int G, typename CA>
__device__ inline int32_t group_select(const int32_t *__restrict__ col, int32_t e0, int32_t e1, CA C,
                                       int32_t n, uint32_t j, uint32_t base = 0) {
    const int l = __lane_id() & (G - 1);
    for (;;) {
        uint64_t mask = 0;
        for (int32_t eb = e0 + l; eb < e1; eb += G * GC_UNROLL) {
            int32_t w[GC_UNROLL], x[GC_UNROLL];
#pragma unroll
            for (int u = 0; u < GC_UNROLL; u++) {
                const int32_t e = eb + u * G;
                const int32_t wl = col[e < e1 ? e : eb];
                w[u] = e < e1 ? wl : -1;
            }
#pragma unroll
            for (int u = 0; u < GC_UNROLL; u++) {
                const bool ok = (uint32_t)w[u] < (uint32_t)n;
                const int32_t xl = (int32_t)C[ok ? w[u] : 0];
                x[u] = ok ? xl : 0;
            }
#pragma unroll
            for (int u = 0; u < GC_UNROLL; u++) {
                uint32_t d = (uint32_t)x[u] - base - 1u;
                if (d < 64u) mask |= 1ull << d;
            }
        }
        mask = group_or_u64<G>(mask);
        const uint64_t fr = ~mask;
        const uint32_t cnt = (uint32_t)__popcll(fr);
        if (j < cnt) return (int32_t)(base + 1u + nth_set_bit(fr, j));
        j -= cnt;
        base += 64u;
    }
}

// ---------------------------------------------------------------------------
// color masks wider than one register word
// ---------------------------------------------------------------------------

// Marks color x (> base) for First Fit: colors base+1 .. base+64 in the
// register word m; with WIDE also colors base+65 .. base+64*(gw+1) in the
// group's LDS words lw[gfirst + o].  Values <= base (no color, a tentative
// color, a class not recolored yet) fall outside both.
template <bool WIDE>
__device__ inline void mask_mark(int32_t x, uint32_t base, uint64_t &m, unsigned long long *lw, int gfirst, int gw) {
    const uint32_t d = (uint32_t)x - base - 1u;
    m |= (d < 64u ? 1ull : 0ull) << (d & 63u);
    if (WIDE) {
        const uint32_t o = (d >> 6) - 1u;
        if (o < (uint32_t)gw) atomicOr(&lw[gfirst + (int)o], 1ull << (d & 63u));
    }
}

// OR of m over the aligned group of gsz lanes (gsz a power of two <= 64).
__device__ inline uint64_t group_or_rt(uint64_t m, int gsz) {
    for (int o = gsz >> 1; o > 0; o >>= 1) m |= __shfl_xor(m, o);
    return m;
}

// First color of the j-th (0-based) unmarked position of 64 words, one word
// per lane (bit d of lane L's word marks color 64 L + d + 1): the color, or 0
// when the words hold at most j unmarked positions.  Whole wavefront.
__device__ inline uint32_t wave_nth_free(uint64_t word, uint32_t j) {
    const int lane = __lane_id();
    const uint64_t fr = ~word;
    const uint32_t cnt = (uint32_t)__popcll(fr);
    uint32_t inc = cnt;
    for (int o = 1; o < 64; o <<= 1) {
        const uint32_t y = __shfl_up(inc, o);
        if (lane >= o) inc += y;
    }
    const uint32_t ex = inc - cnt;
    const bool mine = j >= ex && j < inc;  // exactly one lane when any
    const uint64_t hit = __ballot(mine);
    if (!hit) return 0u;
    const int fl = __ffsll((long long)hit) - 1;
    const uint32_t r = mine ? 64u * (uint32_t)lane + 1u + nth_set_bit(fr, j - ex) : 0u;
    return __shfl(r, fl);
}

// (j+1)-th smallest positive color absent from {C[w] > 0 : w in col[e0..e1)}
// for a group of G lanes in one scan: colors 1..64 in a register word,
// 65 .. 64 * G in the group's LDS words (lw: the wavefront's 64 words, lane L
// owns lw[L]); colors beyond rescan the row in 64-color windows.  Result
// uniform over the group.
template <int G, int UNR = GC_UNROLL, typename CA>
__device__ inline int32_t group_select_wide(const int32_t *__restrict__ col, int32_t e0, int32_t e1, CA C,
                                            int32_t n, uint32_t j, unsigned long long *lw) {
    const int lane = __lane_id();
    const int o = lane & (G - 1);
    const int gfirst = lane - o;
    lw[lane] = 0ull;
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    uint64_t m = 0;
    for (int32_t eb = e0 + o; eb < e1; eb += G * UNR) {
        int32_t w[UNR], x[UNR];
#pragma unroll
        for (int u = 0; u < UNR; u++) {
            const int32_t e = eb + u * G;
            const int32_t wl = col[e < e1 ? e : eb];
            w[u] = e < e1 ? wl : -1;
        }
#pragma unroll
        for (int u = 0; u < UNR; u++) {
            const bool ok = (uint32_t)w[u] < (uint32_t)n;
            const int32_t xl = (int32_t)C[ok ? w[u] : 0];
            x[u] = ok ? xl : 0;
        }
#pragma unroll
        for (int u = 0; u < UNR; u++) mask_mark<true>(x[u], 0u, m, lw, gfirst, G - 1);
    }
    m = group_or_u64<G>(m);
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    // lane o of the group holds colors 64 o + 1 .. 64 o + 64
    const uint64_t word = o == 0 ? m : lw[lane - 1];
    const uint64_t fr = ~word;
    const uint32_t cnt = (uint32_t)__popcll(fr);
    uint32_t inc = cnt;
    for (int d = 1; d < G; d <<= 1) {
        const uint32_t y = __shfl_up(inc, d, G);
        if (o >= d) inc += y;
    }
    const uint32_t ex = inc - cnt;
    const bool mine = j >= ex && j < inc;
    const uint64_t gmask = G == 64 ? ~0ull : (((1ull << G) - 1ull) << gfirst);
    const uint64_t hit = __ballot(mine) & gmask;
    if (hit) {
        const int fl = __ffsll((long long)hit) - 1;
        const uint32_t r = mine ? 64u * (uint32_t)o + 1u + nth_set_bit(fr, j - ex) : 0u;
        return (int32_t)__shfl(r, fl);
    }
    const uint32_t total = __shfl(inc, gfirst + G - 1);
    return group_select<G>(col, e0, e1, C, n, j - total, 64u * G);
}
