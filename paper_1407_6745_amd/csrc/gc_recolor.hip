// gc_recolor.hip - one iterated-greedy recoloring pass (section 2.1,
// Culberson's Iterated Greedy; section 3, synchronous recoloring RC with the
// RV / NI / ND / RAND class permutations).
//
// Steps on the device:
//   1. histogram of the input colors (workgroup-private in LDS) split by
//      degree bin, and the max color;
//   2. class order (one workgroup): compacts the non-empty classes, orders
//      them, gives every color its rank, and lays out the grouped vertex list
//      as segments (rank, bin) with list offsets and work-chunk offsets;
//   3. scatter: counting sort of the vertices into their segments; the output
//      array is set to -(rank + 1), i.e. "not yet recolored, class rank r";
//   4. class walk: every vertex of rank s takes the smallest positive color
//      not held by a neighbor of lower rank (those are recolored before it).
//
// Degree bins (per rank): bin 0 rows up to deg_wave entries, one group of G
// lanes per vertex; bin 1 rows up to deg_split entries, one wavefront per
// vertex; bin 2 longer rows, cut into split_len-entry sub-chunks scanned by
// different wavefronts, whose partial color masks meet in a per-row global
// bitmap; the wavefront that finishes last publishes the color.
//
// The walk runs as ONE persistent launch (every workgroup resident) without
// grid barriers.  Work chunks never straddle two segments and every
// wavefront takes its chunks in increasing order, so a vertex only ever waits
// for vertices of earlier chunks: a vertex of rank s reads each neighbor's
// word; a positive word is a final color of a lower rank; a negative word
// names the neighbor's rank, and only ranks below s are waited for (an
// agent-scope load loop, bounded).  With every workgroup co-resident the
// earliest unfinished chunk can always proceed, so the walk cannot deadlock
// (a split row's color appears when its last sub-chunk ends, and all its
// sub-chunks come before any chunk that waits for it).  Final colors are
// written with agent-scope stores so that waiting wavefronts on other XCDs
// see them; a word only ever changes from negative to its final positive
// value, so a plain (possibly L2-stale) load that sees a positive value is
// exact, and a stale negative value of a lower rank just falls into the
// coherent wait loop.
#include "gc_internal.h"

#include <vector>

#define HIST_LDS GC_HIST_LDS  // colors below this use the workgroup-private histogram
#define HIST_ITEMS 8        // vertices per thread of one histogram tile
#define PERM_THREADS 1024
#define PERM_THREADS_SMALL 256  // class order when every class count fits the LDS path: shorter barriers
#define ORDER_LDS 2048      // colors up to this run the class order on LDS copies
#define SCATTER_BINS 1024   // segments below this reserve list ranges once per workgroup
#define SCATTER_ITEMS 4
#define SCATTER_BLOCK 256
#define WALK_BLOCK 256
#define SPIN_LIMIT (1u << 20)
#define NSEG_PER_RANK 3
#define CT_MAX_K1 127    // classes that fit the one-byte compact color copy
#define CT_MAX_K2 32767  // classes that fit the two-byte compact color copy
#define HUB_WORDS GC_HUB_WORDS  // hub slot stride; ranks above 64 * hub_words - 1 keep long rows in bin 1
// the histogram copy of a vertex is (histogram tile) mod GC_HIST_COPIES; a
// scatter tile (same block size) lies inside one histogram tile
static_assert(HIST_ITEMS % SCATTER_ITEMS == 0, "scatter tiles must nest in histogram tiles");
static_assert(ORDER_LDS < HIST_LDS, "the class order's LDS path takes all its counts from the copies");

// bin of a row of length d (a split row of a rank above hub_max_rank goes to bin 1 later)
__device__ inline int row_bin(int32_t d, int32_t deg_wave, int32_t deg_split) {
    return d <= deg_wave ? 0 : ((deg_split > 0 && d > deg_split) ? 2 : 1);
}

// Histogram copy of the vertices of histogram tile t when the histogram runs
// on `grid` workgroups: workgroup w takes the consecutive tiles
// [w * tpw, (w + 1) * tpw), and the copies take consecutive blocks of
// workgroups, so a copy's part of a segment lists its vertices in about
// ascending order (neighboring rows stay close in the class walk).
__device__ inline int hist_copy_of_tile(int64_t t, int64_t tpw, int grid) {
    return (int)((t / tpw) * GC_HIST_COPIES / grid);
}

__device__ inline int64_t hist_tiles_per_wg(int32_t n, int block, int grid) {
    const int64_t tiles = ((int64_t)n + (int64_t)HIST_ITEMS * block - 1) / ((int64_t)HIST_ITEMS * block);
    return (tiles + grid - 1) / grid;
}

// Class sizes by degree bin.  Colors below HIST_LDS: bin-0 and bin-1 counts
// in LDS, flushed into the workgroup's histogram copy; bin 2 always, and
// every bin of larger colors, straight into the global arrays.  bins == 0:
// every row is in bin 0 (no row is longer than deg_wave), and the row
// pointers are not read.
__global__ void k_hist(int32_t n, const int32_t *__restrict__ Cin, const int32_t *__restrict__ rp, int64_t nnz,
                       int32_t bins, int32_t deg_wave, int32_t deg_split, int32_t split_len, int32_t ccap,
                       int32_t *__restrict__ hist, int32_t *__restrict__ histw, int32_t *__restrict__ hist_s,
                       int32_t *__restrict__ hist_sc, int32_t *__restrict__ hcopy, unsigned long long *scal) {
    __shared__ int32_t h[2 * HIST_LDS];  // bin 0 at [c], bin 1 at [HIST_LDS + c]
    __shared__ int32_t lds[32];
    for (int i = threadIdx.x; i < 2 * HIST_LDS; i += blockDim.x) h[i] = 0;
    __syncthreads();
    int32_t mx = 0;
    bool bad = false;
    // tiles of HIST_ITEMS * blockDim vertices; every load of a tile is issued before any is used
    const int64_t tile_sz = (int64_t)HIST_ITEMS * blockDim.x;
    const int64_t tpw = hist_tiles_per_wg(n, blockDim.x, gridDim.x);
    const int64_t tile_end = ((int64_t)blockIdx.x + 1) * tpw * tile_sz;
    for (int64_t tile = (int64_t)blockIdx.x * tpw * tile_sz; tile < n && tile < tile_end; tile += tile_sz) {
        int32_t cs[HIST_ITEMS], a0[HIST_ITEMS], a1[HIST_ITEMS];
#pragma unroll
        for (int it = 0; it < HIST_ITEMS; it++) {
            const int64_t v = tile + (int64_t)it * blockDim.x + threadIdx.x;
            const bool in = v < n;
            const int64_t vv = in ? v : 0;
            cs[it] = in ? Cin[vv] : 0;
            a0[it] = bins ? rp[vv] : 0;
            a1[it] = bins ? rp[vv + 1] : 0;
        }
#pragma unroll
        for (int it = 0; it < HIST_ITEMS; it++) {
            const int64_t v = tile + (int64_t)it * blockDim.x + threadIdx.x;
            const int32_t c = cs[it];
            int32_t bin = 0, d = 0;
            bool valid = false;
            if (v < n) {
                mx = max(mx, c);
                if (c < 1 || c > ccap) bad = true;
                else {
                    valid = true;
                    // row_range's clamping, on the preloaded row bounds
                    int64_t e0 = a0[it], e1 = a1[it];
                    e0 = e0 < 0 ? 0 : (e0 > nnz ? nnz : e0);
                    e1 = e1 < e0 ? e0 : (e1 > nnz ? nnz : e1);
                    d = (int32_t)(e1 - e0);
                    bin = row_bin(d, deg_wave, deg_split);
                }
            }
            const bool in_lds = valid && c < HIST_LDS;
            // plain LDS adds: equal colors in a wavefront only serialize in the LDS
            if (in_lds && bin < 2) atomicAdd(&h[bin * HIST_LDS + c], 1);
            if (valid && !in_lds) {
                atomicAdd(&hist[c], 1);
                if (bin == 1) atomicAdd(&histw[c], 1);
            }
            if (valid && bin == 2) {  // rare: long rows
                atomicAdd(&hist_s[c], 1);
                atomicAdd(&hist_sc[c], (d + split_len - 1) / split_len);
            }
        }
    }
    const int32_t bmax = block_max_i32(mx, lds);  // synchronizes the block
    const int32_t top = bmax < HIST_LDS - 1 ? bmax : HIST_LDS - 1;
    int32_t *h0c = hcopy + (size_t)hist_copy_of_tile((int64_t)blockIdx.x * tpw, tpw, gridDim.x) * HIST_LDS;
    int32_t *h1c = h0c + (size_t)GC_HIST_COPIES * HIST_LDS;
    for (int i = threadIdx.x + 1; i <= top; i += blockDim.x) {
        if (h[i]) atomicAdd(&h0c[i], h[i]);
        if (h[HIST_LDS + i]) atomicAdd(&h1c[i], h[HIST_LDS + i]);
    }
    unsigned long long anybad = __ballot(bad);
    if (__lane_id() == 0 && anybad) atomicOr(&scal[S_ERR], 1ull);
    if (threadIdx.x == 0) atomicMax((int *)&scal[S_MAXC], bmax);
}

// Class order and segment layout (one workgroup).  Segment 3s + b holds the
// rank-s vertices of bin b.  off[g] / coff[g]: first list slot / first work
// chunk of segment g (off[3k] = n, coff[3k] = chunks); cursor[g] = off[g];
// sbase[s]: first hub slot of segment 3s + 2.  A chunk is 64 / G vertices of
// a bin-0 segment, one vertex of a bin-1 segment, split_len entries of a row
// of a bin-2 segment.
template <int THREADS>
__global__ void __launch_bounds__(THREADS) k_class_order(int32_t ccap, int32_t perm, uint32_t s_perm, int32_t vpc,
                                                               int32_t hub_max_rank, int32_t *hist, int32_t *histw, int32_t *hist_s,
                                                               int32_t *hist_sc, int32_t *cls, int32_t *pi,
                                                               int32_t *rank, int32_t *off, int32_t *coff,
                                                               int32_t *cursor, int32_t *sbase, int32_t *hcopy,
                                                               int32_t *segnz, unsigned long long *scal) {
    __shared__ int32_t lds[32];
    // up to ORDER_LDS colors every step below runs on LDS copies of the class
    // counts (one workgroup: global round trips would dominate)
    __shared__ int32_t l_h[ORDER_LDS + 1], l_hw[ORDER_LDS + 1], l_hs[ORDER_LDS + 1], l_hsc[ORDER_LDS + 1];
    __shared__ int32_t l_cls[ORDER_LDS + 1], l_pi[ORDER_LDS + 1];
    int32_t maxc = (int32_t)scal[S_MAXC];
    if (maxc > ccap) maxc = ccap;
    int32_t *H = hist, *HW = histw, *HS = hist_s, *HSC = hist_sc, *CL = cls, *PI = pi;
    const bool local = maxc <= ORDER_LDS;
    // colors below HIST_LDS: class sizes from the histogram copies (which are
    // cleared for the next call), and every copy's relative cursor in the
    // color's bin-0 segment; with local, into the LDS copies directly
    const int32_t lmax = maxc < HIST_LDS - 1 ? maxc : HIST_LDS - 1;
    int32_t *h1c = hcopy + (size_t)GC_HIST_COPIES * HIST_LDS;
    int32_t *rel = hcopy + (size_t)2 * GC_HIST_COPIES * HIST_LDS;
    for (int32_t c = threadIdx.x; c <= lmax; c += blockDim.x) {
        int32_t x[GC_HIST_COPIES], y[GC_HIST_COPIES];
#pragma unroll
        for (int p = 0; p < GC_HIST_COPIES; p++) {
            x[p] = hcopy[(size_t)p * HIST_LDS + c];
            y[p] = h1c[(size_t)p * HIST_LDS + c];
        }
        const int32_t hs = hist_s[c];
        int32_t a = 0, w = 0;
#pragma unroll
        for (int p = 0; p < GC_HIST_COPIES; p++) {
            rel[(size_t)p * HIST_LDS + c] = a;
            a += x[p];
            w += y[p];
            hcopy[(size_t)p * HIST_LDS + c] = 0;
            h1c[(size_t)p * HIST_LDS + c] = 0;
        }
        if (local) {
            l_h[c] = a + w + hs;
            l_hw[c] = w;
            l_hs[c] = hs;
            l_hsc[c] = hist_sc[c];
        } else {
            hist[c] = a + w + hs;
            histw[c] = w;
        }
    }
    __syncthreads();
    if (local) {  // maxc <= ORDER_LDS < HIST_LDS: every color was filled above
        H = l_h;
        HW = l_hw;
        HS = l_hs;
        HSC = l_hsc;
        CL = l_cls;
        PI = l_pi;
    }
    const int32_t k = block_class_order(maxc, perm, s_perm, H, CL, PI, rank, nullptr, nullptr, lds);
    const int32_t nseg = NSEG_PER_RANK * k;
    int32_t acc = 0, cacc = 0, zacc = 0;
    for (int32_t base = 0; base < nseg; base += blockDim.x) {
        const int32_t g = base + (int32_t)threadIdx.x;
        int32_t sz = 0, ch = 0;
        if (g < nseg) {
            const int32_t s = g / NSEG_PER_RANK, b = g % NSEG_PER_RANK;
            const int32_t c = PI[s];
            const bool split = s <= hub_max_rank;
            if (b == 0) {
                sz = H[c] - HW[c] - HS[c];
                ch = (sz + vpc - 1) / vpc;
            } else if (b == 1) {
                sz = HW[c] + (split ? 0 : HS[c]);
                ch = sz;
            } else if (split) {
                sz = HS[c];
                ch = HSC[c];
            }
        }
        int32_t tot, ctot, ztot;
        const int32_t ex = block_exclusive_scan(sz, &tot, lds);
        const int32_t cex = block_exclusive_scan(ch, &ctot, lds);
        // the segments that hold work chunks, in order: the walk visits only these
        const int32_t zex = block_exclusive_scan(ch > 0 ? 1 : 0, &ztot, lds);
        if (g < nseg) {
            off[g] = acc + ex;
            cursor[g] = acc + ex;
            coff[g] = cacc + cex;
            if (ch > 0) segnz[zacc + zex] = g;
        }
        acc += tot;
        cacc += ctot;
        zacc += ztot;
    }
    // hub slot bases: prefix of the split-segment sizes over ranks
    int32_t hacc = 0;
    for (int32_t base = 0; base < k; base += blockDim.x) {
        const int32_t s = base + (int32_t)threadIdx.x;
        int32_t sz = 0;
        if (s < k && s <= hub_max_rank) sz = HS[PI[s]];
        int32_t tot;
        const int32_t ex = block_exclusive_scan(sz, &tot, lds);
        if (s < k) sbase[s] = hacc + ex;
        hacc += tot;
    }
    if (threadIdx.x == 0) {
        off[nseg] = acc;
        coff[nseg] = cacc;
        scal[S_K] = (unsigned long long)k;
        scal[S_NZSEG] = (unsigned long long)zacc;
    }
    if (local)
        for (int32_t i = threadIdx.x; i < k; i += blockDim.x) pi[i] = l_pi[i];
    __syncthreads();
    for (int32_t c = threadIdx.x; c <= maxc; c += blockDim.x) {
        hist[c] = 0;
        histw[c] = 0;
        hist_s[c] = 0;
        hist_sc[c] = 0;
    }
}

// Counting-sort scatter into segments: one tile of SCATTER_ITEMS * blockDim
// vertices per workgroup; segments below SCATTER_BINS reserve their list
// range once per workgroup, and the tile's entries are staged in LDS in
// segment order so that each segment's run is written out contiguously.
// Writes Cout[v] = -(rank + 1) and the row range next to each list entry.
__global__ void __launch_bounds__(SCATTER_BLOCK) k_scatter(int32_t n, const int32_t *Cin, int32_t *Cout, void *S, const int32_t *__restrict__ rp, int64_t nnz,
                          int32_t deg_wave, int32_t deg_split, int32_t hub_max_rank, int32_t ccap,
                          const int32_t *__restrict__ rank,
                          int32_t *__restrict__ cursor, int32_t *__restrict__ list, int2 *__restrict__ rows,
                          const int32_t *__restrict__ pi, const int32_t *__restrict__ off,
                          int32_t *__restrict__ rel, int hist_grid, const unsigned long long *__restrict__ scal) {
    __shared__ int32_t cnt[SCATTER_BINS];  // per segment: count, then staging offset
    __shared__ int32_t basepos[SCATTER_BINS];
    __shared__ int4 stage[SCATTER_ITEMS * SCATTER_BLOCK];  // (vertex, row begin, row end, list slot)
    __shared__ int32_t lds[32];
    const int32_t k = (int32_t)scal[S_K];
    const int32_t nseg = NSEG_PER_RANK * k;
    const int32_t bins = nseg < SCATTER_BINS ? nseg : SCATTER_BINS;
    const int gbits = key_bits(bins);
    for (int i = threadIdx.x; i < bins; i += blockDim.x) cnt[i] = 0;
    __syncthreads();
    const int64_t tile = (int64_t)blockIdx.x * blockDim.x * SCATTER_ITEMS;
    int32_t sg[SCATTER_ITEMS], loc[SCATTER_ITEMS];
    int2 rw[SCATTER_ITEMS];
    // every load of the tile first (colors, row bounds, then ranks), so that
    // the stores below (Cout may be Cin) do not order them one item at a time
    int32_t cs[SCATTER_ITEMS], a0[SCATTER_ITEMS], a1[SCATTER_ITEMS], rk[SCATTER_ITEMS];
#pragma unroll
    for (int it = 0; it < SCATTER_ITEMS; it++) {
        const int64_t v = tile + (int64_t)it * blockDim.x + threadIdx.x;
        const int64_t vv = v < n ? v : 0;
        cs[it] = Cin[vv];
        a0[it] = rp[vv];
        a1[it] = rp[vv + 1];
    }
#pragma unroll
    for (int it = 0; it < SCATTER_ITEMS; it++) {
        const bool ok = cs[it] >= 1 && cs[it] <= ccap;
        rk[it] = rank[ok ? cs[it] : 0];
    }
#pragma unroll
    for (int it = 0; it < SCATTER_ITEMS; it++) {
        const int64_t v = tile + (int64_t)it * blockDim.x + threadIdx.x;
        sg[it] = -1;
        loc[it] = -1;
        rw[it] = make_int2(0, 0);
        int32_t g = -1;
        if (v < n) {
            const int32_t c = cs[it];
            if (c >= 1 && c <= ccap && k > 0) {
                int32_t s = rk[it];
                if ((uint32_t)s >= (uint32_t)k) s = k - 1;  // unreachable for a ranked color; keeps indices in bounds
                int64_t e0 = a0[it], e1 = a1[it];  // row_range's clamping on the preloaded bounds
                e0 = e0 < 0 ? 0 : (e0 > nnz ? nnz : e0);
                e1 = e1 < e0 ? e0 : (e1 > nnz ? nnz : e1);
                rw[it] = make_int2((int32_t)e0, (int32_t)e1);
                int b = row_bin((int32_t)(e1 - e0), deg_wave, deg_split);
                if (b == 2 && s > hub_max_rank) b = 1;
                g = NSEG_PER_RANK * s + b;
                sg[it] = g;
                if (g >= SCATTER_BINS) {
                    const int32_t p = atomicAdd(&cursor[g], 1);
                    list[p] = (int32_t)v;
                    rows[p] = rw[it];
                    Cout[v] = -(s + 1);
                }
                if (k <= CT_MAX_K1) ((uint8_t *)S)[v] = (uint8_t)(0x80 | s);
                else if (k <= CT_MAX_K2) ((uint16_t *)S)[v] = (uint16_t)(0x8000 | s);
            } else {
                Cout[v] = 0;
            }
        }
        const bool in_lds = g >= 0 && g < SCATTER_BINS;
        const int32_t pos = wave_match_reserve_bits(cnt, g, in_lds, gbits);
        if (in_lds) loc[it] = pos;
    }
    __syncthreads();
    // bin-0 segments of colors with per-copy counts reserve from this tile's
    // copy's part of the segment (the copy the histogram counted it in)
    const int copy = hist_copy_of_tile((int64_t)blockIdx.x * SCATTER_ITEMS / HIST_ITEMS,
                                       hist_tiles_per_wg(n, blockDim.x, hist_grid), hist_grid);
    int32_t staged = 0;
    for (int base = 0; base < bins; base += blockDim.x) {
        const int i = base + (int)threadIdx.x;
        const int32_t ci = i < bins ? cnt[i] : 0;
        if (ci) {
            const int32_t c = i % NSEG_PER_RANK == 0 ? pi[i / NSEG_PER_RANK] : HIST_LDS;
            if (c < HIST_LDS)
                basepos[i] = off[i] + atomicAdd(&rel[(size_t)copy * HIST_LDS + c], ci);
            else
                basepos[i] = atomicAdd(&cursor[i], ci);
        }
        int32_t tot;
        const int32_t ex = block_exclusive_scan(ci, &tot, lds);  // ends with a barrier
        if (i < bins) cnt[i] = staged + ex;
        staged += tot;
    }
    __syncthreads();
#pragma unroll
    for (int it = 0; it < SCATTER_ITEMS; it++) {
        const int64_t v = tile + (int64_t)it * blockDim.x + threadIdx.x;
        if (loc[it] >= 0) {
            const int32_t g = sg[it];
            stage[cnt[g] + loc[it]] = make_int4((int32_t)v, rw[it].x, rw[it].y, basepos[g] + loc[it]);
            Cout[v] = -((g / NSEG_PER_RANK) + 1);
        }
    }
    __syncthreads();
    for (int32_t j = threadIdx.x; j < staged; j += blockDim.x) {
        const int4 e = stage[j];
        list[e.w] = e.x;
        rows[e.w] = make_int2(e.y, e.z);
    }
}

// For every split segment: the first chunk of each of its rows (prefix of
// ceil(len / split_len) in list order).  One thread per rank.
__global__ void k_split_prefix(const int32_t *__restrict__ off, const int2 *__restrict__ rows, int32_t split_len,
                               int32_t *__restrict__ hsub, const unsigned long long *__restrict__ scal) {
    const int32_t k = (int32_t)scal[S_K];
    for (int32_t s = blockIdx.x * blockDim.x + threadIdx.x; s < k; s += gridDim.x * blockDim.x) {
        const int32_t g = NSEG_PER_RANK * s + 2;
        int32_t acc = 0;
        for (int32_t p = off[g]; p < off[g + 1]; p++) {
            hsub[p] = acc;
            const int2 r = rows[p];
            acc += (r.y - r.x + split_len - 1) / split_len;
        }
    }
}

// One work chunk as a wavefront sees it: segment, the vertex of this lane's
// group (-1: none) and the part of its row this chunk scans; for a split row
// also its hub slot and number of sub-chunks.
struct WalkChunk {
    int32_t seg, v, e0, e1, slot, nsub;
};

// Compact copy of the colors for the neighbor gathers of the walk (CT = 1:
// one byte per vertex when there are at most 127 classes, CT = 2: two bytes
// when at most 32767; CT = 0: none).  The top bit marks "not recolored yet"
// with the rank in the low bits; otherwise the word is the final color.  Two
// or four times as many vertices share a cache line as in the int32 array,
// so a gather instruction touches that many fewer lines.  The copy only
// speeds up the first look: pending words are still re-read from the int32
// array (coherently), which stays the reference.
template <int CT>
__device__ inline int32_t compact_load(const void *S, int32_t w) {
    if (CT == 1) {
        const uint32_t x = ((const uint8_t *)S)[w];
        return (x & 0x80u) ? -(int32_t)(x & 0x7Fu) - 1 : (int32_t)x;
    } else {
        const uint32_t x = ((const uint16_t *)S)[w];
        return (x & 0x8000u) ? -(int32_t)(x & 0x7FFFu) - 1 : (int32_t)x;
    }
}

template <int CT>
__device__ inline void compact_store(void *S, int32_t v, int32_t color) {
    if (CT == 1) ((uint8_t *)S)[v] = (uint8_t)color;
    if (CT == 2) ((uint16_t *)S)[v] = (uint16_t)color;
}

// Bounded waits of the walk: polls before giving up, and the scalar slots
// where a wait that gave up is recorded (per pass, and sticky).
// walk_flags knob bits
#define WALK_LONG_FIRST 1u   // inside a rank: split rows, then wavefront rows, then group rows
#define WALK_EARLY_MERGE 2u  // a waiting split-row sub-chunk takes the others' words once they are all in
#define WALK_WAIT_IN_PLACE 4u  // a pending word is waited for where the scan meets it (else after the scan)

struct WaitCtl {
    unsigned long long *scal;
    uint32_t limit;
    uint32_t flags;  // walk_flags
    // class-completion trace (NULL = off): [0] walk start, [1] walk end,
    // [2 + 2s] latest completion of a rank-s vertex, [3 + 2s] of a rank-s split row
    unsigned long long *trace;
};

// Trace record of a split row of rank s that has just published its color
// (the other vertices are recorded per wavefront and rank, see walk_body).
__device__ inline void trace_done(const WaitCtl &wc, int32_t s, bool split) {
    if (wc.trace) {
        const unsigned long long t = wall_clock64();
        atomicMax(&wc.trace[2 + 2 * (int64_t)s], t);
        if (split) atomicMax(&wc.trace[3 + 2 * (int64_t)s], t);
    }
}

// A sub-chunk of a split row while it waits: the row's hub slot (finished
// sub-chunks and their merged mask words).  When every other sub-chunk of the
// row has finished (count nsub - 1), the waiting one takes their words into
// its own mask at once (merged): it is the last, and publishes the row's color
// as soon as its own waits end, with no further round trip through the slot.
struct HubWait {
    int32_t *cnt;
    const unsigned long long *bits;
    int32_t nsub, words;
    bool merged;
};

// Neighbor words -> marks for colors of lower ranks.  Words of lower ranks
// that are not final yet (or whose plain load saw a stale line) are re-read
// in one wavefront-uniform slow path: every pending word of every lane is
// reloaded past the L2 at once, so one round trip settles all words that
// are final by then; the rest is branch-free.
template <int U, bool WIDE>
__device__ inline void absorb(const int32_t *w, int32_t *xv, int32_t s, uint32_t base, uint64_t &m,
                              unsigned long long *lw, int gfirst, int gw, int32_t *C, const WaitCtl &wc,
                              HubWait *hw = nullptr) {
    bool pend[U];
    bool need = false;
#pragma unroll
    for (int u = 0; u < U; u++) {
        pend[u] = xv[u] < 0 && -xv[u] - 1 < s;
        need |= pend[u];
    }
    if (__ballot(need)) {
#pragma unroll
        for (int u = 0; u < U; u++)
            if (xv[u] < 0 && !pend[u]) xv[u] = 0;  // a rank >= s: not a constraint
        for (uint32_t it = 0;; it++) {
            int32_t y[U];
#pragma unroll
            for (int u = 0; u < U; u++) {
                y[u] = 0;
                if (pend[u]) y[u] = __hip_atomic_load(&C[w[u]], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            }
            bool left = false;
#pragma unroll
            for (int u = 0; u < U; u++) {
                if (pend[u] && y[u] > 0) {
                    xv[u] = y[u];
                    pend[u] = false;
                }
                left |= pend[u];
            }
            if (!__ballot(left)) break;
            if (hw && !hw->merged) {
                int32_t done = 0;
                if (__lane_id() == 0) done = __hip_atomic_load(hw->cnt, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                done = __shfl(done, 0);
                if (done == hw->nsub - 1) {
                    // each other sub-chunk's ORs were done before it counted itself;
                    // the words are read with device atomics
                    const int lane = __lane_id();
                    const uint64_t b =
                        lane < hw->words ? __hip_atomic_load(&hw->bits[lane], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)
                                         : 0ull;
                    if (lane == 0) m |= b;  // word 0 lives in the register words (ORed over the wavefront later)
                    else if (b) atomicOr(&lw[lane - 1], b);
                    hw->merged = true;
                }
            }
            if (it >= wc.limit ||
                ((it & 1023u) == 1023u &&
                 (__hip_atomic_load(&wc.scal[S_ERR], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) & 6ull))) {
                if (it >= wc.limit) {  // gives up: wrong result, but the kernel ends; the error is sticky
                    atomicOr(&wc.scal[S_ERR], 2ull);
                    atomicOr(&wc.scal[S_STICKY], 2ull);
                }
#pragma unroll
                for (int u = 0; u < U; u++)
                    if (pend[u]) xv[u] = 0;
                break;
            }
            __builtin_amdgcn_s_sleep(2);
        }
    }
#pragma unroll
    for (int u = 0; u < U; u++) mask_mark<WIDE>(xv[u], base, m, lw, gfirst, gw);
}

// Deferred waits.  A lane's entries whose words were pending (lower rank, not
// final yet) are remembered as bits of their index j in the lane's share of
// the range (entry e + j * gsz, j < 64), and settled together after the whole
// range has been scanned: the scan of the rest of a long row then overlaps
// the wait instead of following it, so a vertex publishes one round trip
// after its last lower-rank neighbor, not one per batch of the row left.
// Batches past index 64 wait in place (absorb).
template <int U, bool WIDE>
__device__ inline void absorb_defer(const int32_t *w, int32_t *xv, int32_t s, uint64_t &m, unsigned long long *lw,
                                    int gfirst, int gw, int32_t *C, const WaitCtl &wc, uint64_t &pm, int j0) {
    if (j0 + U > 64) {
        absorb<U, WIDE>(w, xv, s, 0u, m, lw, gfirst, gw, C, wc);
        return;
    }
#pragma unroll
    for (int u = 0; u < U; u++) {
        if (xv[u] < 0) {
            if (-xv[u] - 1 < s) pm |= 1ull << (j0 + u);
            xv[u] = 0;  // pending: marked when settled; a rank >= s: no constraint
        }
        mask_mark<WIDE>(xv[u], 0u, m, lw, gfirst, gw);
    }
}

// Waits (bounded, as absorb) until every deferred entry's word is final and
// marks its color.  Whole wavefront; e is this lane's first entry.
template <bool WIDE>
__device__ inline void settle(uint64_t pm, int32_t e, int gsz, const int32_t *__restrict__ col, uint64_t &m,
                              unsigned long long *lw, int gfirst, int gw, int32_t *C, const WaitCtl &wc) {
    for (uint32_t it = 0;; it++) {
        uint64_t rest = pm;
        while (__ballot(rest != 0ull)) {
            // up to four of the lane's entries per sweep, their loads issued together
            int32_t jj[4], y[4];
#pragma unroll
            for (int q = 0; q < 4; q++) {
                jj[q] = rest ? __ffsll((long long)rest) - 1 : -1;
                rest &= rest - 1;
            }
            int32_t wq[4];
#pragma unroll
            for (int q = 0; q < 4; q++) wq[q] = jj[q] >= 0 ? col[e + jj[q] * gsz] : 0;
#pragma unroll
            for (int q = 0; q < 4; q++)
                y[q] = jj[q] >= 0 ? __hip_atomic_load(&C[wq[q]], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) : 0;
#pragma unroll
            for (int q = 0; q < 4; q++)
                if (jj[q] >= 0 && y[q] > 0) {
                    mask_mark<WIDE>(y[q], 0u, m, lw, gfirst, gw);
                    pm &= ~(1ull << jj[q]);
                }
        }
        if (!__ballot(pm != 0ull)) break;
        if (it >= wc.limit ||
            ((it & 1023u) == 1023u &&
             (__hip_atomic_load(&wc.scal[S_ERR], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) & 6ull))) {
            if (it >= wc.limit) {  // gives up: wrong result, but the kernel ends; the error is sticky
                atomicOr(&wc.scal[S_ERR], 2ull);
                atomicOr(&wc.scal[S_STICKY], 2ull);
            }
            break;
        }
        __builtin_amdgcn_s_sleep(2);
    }
}

// Gathers the colors of the neighbor ids w (invalid ids read as 0).
template <int U>
__device__ inline void gather(const int32_t *w, int32_t *xv, const int32_t *C, int32_t n) {
#pragma unroll
    for (int u = 0; u < U; u++) {
        const bool ok = (uint32_t)w[u] < (uint32_t)n;
        const int32_t xl = C[ok ? w[u] : 0];
        xv[u] = ok ? xl : 0;
    }
}

// Scans row entries [e, e1) with stride gsz (this lane's share), U at a time.
template <int U, bool WIDE>
__device__ inline void scan_range(int32_t e, int32_t e1, int gsz, const int32_t *__restrict__ col, int32_t n,
                                  int32_t s, uint32_t base, uint64_t &m, unsigned long long *lw, int gfirst, int gw,
                                  int32_t *C, const WaitCtl &wc, HubWait *hw = nullptr, uint64_t *pm = nullptr,
                                  int j0 = 0) {
    for (int32_t eb = e; __ballot(eb < e1); eb += U * gsz, j0 += U) {
        int32_t ww[U], xx[U];
#pragma unroll
        for (int u = 0; u < U; u++) {
            const int32_t eu = eb + u * gsz;
            const bool ok = eu < e1;
            const int32_t wl = col[ok ? eu : 0];
            ww[u] = ok ? wl : -1;
        }
        gather<U>(ww, xx, C, n);
        if (pm) absorb_defer<U, WIDE>(ww, xx, s, m, lw, gfirst, gw, C, wc, *pm, j0);
        else absorb<U, WIDE>(ww, xx, s, base, m, lw, gfirst, gw, C, wc, hw);
    }
}


// First Fit for bins 0 and 1.  Colors 1..64 are tracked in a register word;
// with WIDE (ranks >= 64) each group also owns gsz LDS words (one per lane of
// the group: this lane's word is lw[lane]) for colors 65 .. 64 * (gsz + 1).
// Colors beyond (a free color is at most the row length + 1) rescan the row
// in 64-color windows.  The first window takes the prefetched ids w.
template <int U, bool WIDE, int CT, bool DEFER>
__device__ inline void finish_row(const WalkChunk &t, const int32_t *w, const int32_t *x, int gsz,
                                  const int32_t *__restrict__ col, int32_t n, int32_t *C, void *S,
                                  unsigned long long *lw, const WaitCtl &wc) {
    const int32_t s = t.seg / NSEG_PER_RANK;
    const int lane = __lane_id();
    const int l = lane & (gsz - 1);
    const int gfirst = lane - l;
    if (WIDE) {
        lw[lane] = 0ull;
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
    }
    uint64_t m = 0;
    int32_t xv[U];
#pragma unroll
    for (int u = 0; u < U; u++) xv[u] = x[u];
    const bool defer = DEFER && !(wc.flags & WALK_WAIT_IN_PLACE);
    uint64_t pm = 0;  // deferred entries of this lane
    if (defer) absorb_defer<U, WIDE>(w, xv, s, m, lw, gfirst, gsz, C, wc, pm, 0);
    else absorb<U, WIDE>(w, xv, s, 0u, m, lw, gfirst, gsz, C, wc);
    scan_range<U, WIDE>(t.e0 + l + U * gsz, t.e1, gsz, col, n, s, 0u, m, lw, gfirst, gsz, C, wc, nullptr,
                        defer ? &pm : nullptr, U);
    if (DEFER && __ballot(pm != 0ull)) settle<WIDE>(pm, t.e0 + l, gsz, col, m, lw, gfirst, gsz, C, wc);
    m = group_or_rt(m, gsz);
    uint32_t r = ~m ? (uint32_t)__ffsll((long long)~m) : 0u;
    uint32_t base = 0;
    if (WIDE) {
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        if (r == 0) {
            const uint64_t word = lw[lane];
            const uint64_t gmask = gsz == 64 ? ~0ull : (((1ull << gsz) - 1ull) << gfirst);
            const uint64_t fr = __ballot(~word != 0ull) & gmask;
            if (fr) {
                const int fl = __ffsll((long long)fr) - 1;
                const uint64_t wf = __shfl(word, fl);
                r = 64u * (uint32_t)(fl - gfirst + 1) + (uint32_t)__ffsll((long long)~wf);
            } else {
                base = 64u * (uint32_t)gsz;  // windows beyond the LDS words start above them
            }
        }
    }
    while (r == 0) {
        base += 64u;
        m = 0;
        scan_range<U, false>(t.e0 + l, t.e1, gsz, col, n, s, base, m, lw, gfirst, 0, C, wc);
        m = group_or_rt(m, gsz);
        r = ~m ? (uint32_t)__ffsll((long long)~m) : 0u;
    }
    if (t.v >= 0 && l == 0) {
        __hip_atomic_store(&C[t.v], (int32_t)(base + r), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        compact_store<CT>(S, t.v, (int32_t)(base + r));
    }
}

// One sub-chunk of a split row (bin 2, whole wavefront).  The colors of lower
// ranks among its entries (colors 1..64 in a register word, 65..4096 in the
// wavefront's LDS words) go into the row's global bitmap; the sub-chunk that
// ends last reads the bitmap, publishes the color and clears the slot for the
// next pass.
template <int U, int CT>
__device__ inline void finish_split(const WalkChunk &t, const int32_t *w, const int32_t *x,
                                    const int32_t *__restrict__ col, int32_t n,
                                    int32_t *C, void *S, unsigned long long *lw, unsigned long long *hub_bits,
                                    int32_t *hub_cnt, const WaitCtl &wc) {
    const int32_t s = t.seg / NSEG_PER_RANK;
    const int lane = __lane_id();
    const int32_t words = (s >> 6) + 1;  // lower ranks hold colors 1..s: words 0 .. s / 64
    unsigned long long *bits = hub_bits + (int64_t)t.slot * HUB_WORDS;
    lw[lane] = 0ull;
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    uint64_t m = 0;
    int32_t xv[U];
    #pragma unroll
    for (int u = 0; u < U; u++) xv[u] = x[u];
    HubWait hw{hub_cnt + t.slot, bits, t.nsub, words, false};
    HubWait *hwp = (wc.flags & WALK_EARLY_MERGE) ? &hw : nullptr;
    const bool defer = !hwp && !(wc.flags & WALK_WAIT_IN_PLACE);
    uint64_t pm = 0;  // deferred entries of this lane
    if (defer) absorb_defer<U, true>(w, xv, s, m, lw, 0, HUB_WORDS - 1, C, wc, pm, 0);
    else absorb<U, true>(w, xv, s, 0u, m, lw, 0, HUB_WORDS - 1, C, wc, hwp);
    scan_range<U, true>(t.e0 + lane + U * 64, t.e1, 64, col, n, s, 0u, m, lw, 0, HUB_WORDS - 1, C, wc, hwp,
                        defer ? &pm : nullptr, U);
    if (__ballot(pm != 0ull)) settle<true>(pm, t.e0 + lane, 64, col, m, lw, 0, HUB_WORDS - 1, C, wc);
    m = group_or_rt(m, 64);
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    // word i of the row: register word for i = 0, LDS word i - 1 above
    const uint64_t lword = lane >= 1 ? lw[lane - 1] : 0ull;
    const uint64_t mine = lane == 0 ? m : lword;
    if (hw.merged) {
        // the other sub-chunks' words are already in this mask: publish now,
        // then clear the slot for the next pass
        const uint64_t word = lane < words ? mine : ~0ull;
        const uint64_t fr = __ballot(~word != 0ull);
        uint32_t r = 64u * (uint32_t)words + 1u;  // unreachable: at most s colors are taken
        if (fr) {
            const int first = __ffsll((long long)fr) - 1;
            const uint64_t wf = __shfl(word, first);
            r = 64u * (uint32_t)first + (uint32_t)__ffsll((long long)~wf);
        }
        if (lane == 0) {
            __hip_atomic_store(&C[t.v], (int32_t)r, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            compact_store<CT>(S, t.v, (int32_t)r);
            trace_done(wc, s, true);
        }
        if (lane < words) atomicExch(&bits[lane], 0ull);
        if (lane == 0) atomicExch(&hub_cnt[t.slot], 0);
        return;
    }
    if (lane < words && mine) atomicOr(&bits[lane], mine);
    // the slot is exchanged through device atomics only: wait until this
    // wavefront's ORs are done, then count it in (no cache maintenance)
    __builtin_amdgcn_s_waitcnt(0);
    int32_t done = 0;
    if (lane == 0) done = atomicAdd(&hub_cnt[t.slot], 1) + 1;
    done = __shfl(done, 0);
    if (done == t.nsub) {
        // every sub-chunk's bits are in (read atomically below): first free color of the row
        const uint64_t word = lane < words ? atomicOr(&bits[lane], 0ull) : ~0ull;
        const uint64_t fr = __ballot(~word != 0ull);
        uint32_t r = 64u * (uint32_t)words + 1u;  // unreachable: at most s colors are taken
        if (fr) {
            const int first = __ffsll((long long)fr) - 1;
            const uint64_t wf = __shfl(word, first);
            r = 64u * (uint32_t)first + (uint32_t)__ffsll((long long)~wf);
        }
        if (lane < words) atomicExch(&bits[lane], 0ull);
        if (lane == 0) {
            atomicExch(&hub_cnt[t.slot], 0);
            __hip_atomic_store(&C[t.v], (int32_t)r, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            compact_store<CT>(S, t.v, (int32_t)r);
            trace_done(wc, s, true);
        }
    }
}

#define WALK_TAB 1536  // segment tables of up to WALK_TAB segments (512 classes) live in LDS

template <int G, bool LDS_TAB, bool FULL, int CT>
__device__ __forceinline__ void walk_body(const int32_t *O, const int32_t *CO, const int32_t *NZ, int32_t nnz_seg,
                                          int32_t nseg,
                                          const int2 *__restrict__ rows, const int32_t *__restrict__ col,
                                          int32_t n, int32_t *C, const int32_t *__restrict__ list,
                                          const int32_t *__restrict__ hsub, const int32_t *__restrict__ sbase,
                                          int32_t split_len, unsigned long long *hub_bits, int32_t *hub_cnt,
                                          WaitCtl wc, int32_t xcd, unsigned long long *lw, void *S) {
    // entries per lane and batch: 32 per group, between 4 and 8 (narrow groups
    // keep the registers, and so the occupancy, of four-lane groups)
    constexpr int U = 32 / G > 8 ? 8 : (32 / G > 4 ? 32 / G : 4);
    const int lane = __lane_id();
    const int wpb = WALK_BLOCK / 64;
    const int wib = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int xl = (xcd && (gridDim.x & 7) == 0) ? 3 : 0;  // log2 of the number of parts
    const uint32_t x = xl ? (blockIdx.x & 7) : 0;
    const uint32_t Wx = (gridDim.x >> xl) * wpb;  // wavefronts sharing one part
    const uint32_t me = (blockIdx.x >> xl) * wpb + wib;
    const uint32_t wm = 0xFFFFFFFFu / Wx;  // for s0 mod Wx below
    // cursor over this wavefront's chunks: segment seg, chunk c in [.., hi).
    // Segments are visited rank by rank; inside a rank (whose vertices never
    // wait for each other) the split rows come first, then the wavefront rows,
    // then the group rows: the longest scans of a class start earliest, and a
    // split row's sub-chunks are already waiting when the previous class ends.
    int32_t idx = -1, seg = -1;
    // visit order: every segment with WALK_LONG_FIRST, else only those with
    // work chunks when their list is given (a wavefront passes every segment
    // it visits, while it takes only a few dozen chunks of the pass)
    const bool lfirst = (wc.flags & WALK_LONG_FIRST) != 0;
    const int32_t nvisit = (lfirst || !NZ) ? nseg : nnz_seg;
    uint32_t c = 0, hi = 0;
    // the cursor segment's list range and first chunk, read once per segment
    // rather than once per chunk (mesh walk 141.3 -> 140.0 us)
    int32_t seg_lo = 0, seg_hi = 0;
    uint32_t seg_s0 = 0;
    bool first = true;
    auto advance = [&]() {
        if (!first) c += Wx;
        first = false;
        while (c >= hi) {
            if (++idx >= nvisit) {
                seg = nseg;
                return;
            }
            seg = lfirst ? idx - idx % NSEG_PER_RANK + (NSEG_PER_RANK - 1 - idx % NSEG_PER_RANK) : (NZ ? NZ[idx] : idx);
            const uint32_t s0 = (uint32_t)CO[seg], len = (uint32_t)CO[seg + 1] - s0;
            if (len == 0) continue;  // an empty segment: c >= hi still holds (mesh walk 147.7 -> 143.3 us)
            const uint32_t lo = s0 + (uint32_t)(((uint64_t)len * x) >> xl);
            hi = s0 + (uint32_t)(((uint64_t)len * (x + 1)) >> xl);
            if (hi <= lo) {  // no chunk of this segment in this part (mesh walk 150.8 -> 146.6 us)
                c = hi;
                continue;
            }
            // rotate so that short segments do not all land on the first
            // wavefronts: c - lo = (me - s0) mod Wx, with s0 mod Wx by a
            // multiply-high with floor((2^32 - 1) / Wx) (the quotient is at
            // most one short, fixed by one subtraction; a division here cost
            // the RMAT-22 walk 2.31 -> 2.36 ms)
            uint32_t rm = s0 - __umulhi(s0, wm) * Wx;
            rm = rm >= Wx ? rm - Wx : rm;
            const uint32_t r = me + (Wx - rm);
            c = lo + (r >= Wx ? r - Wx : r);
            if (c < hi) {
                seg_lo = O[seg];
                seg_hi = O[seg + 1];
                seg_s0 = s0;
            }
        }
    };
    // stage A: vertex and row part of the chunk under the cursor, then advance
    auto load_chunk = [&](WalkChunk &t) {
        t.seg = seg;
        t.v = -1;
        t.e0 = t.e1 = 0;
        t.slot = 0;
        t.nsub = 1;
        if (seg >= nseg) return;
        const int32_t lo = seg_lo, hi2 = seg_hi;
        const int32_t j = (int32_t)(c - seg_s0);
        const int b = seg % NSEG_PER_RANK;
        if (b == 2) {
            // split row: the last list slot whose first chunk is <= j
            int32_t a = lo, z = hi2 - 1;
            while (a < z) {
                const int32_t mid = (a + z + 1) >> 1;
                if (hsub[mid] <= j) a = mid;
                else z = mid - 1;
            }
            const int32_t sub = j - hsub[a];
            const int2 r = rows[a];
            const int32_t vv = list[a];
            if (FULL) {
                t.v = vv;
                t.e0 = r.x + sub * split_len;
                t.e1 = min(r.y, t.e0 + split_len);
                t.slot = sbase[seg / NSEG_PER_RANK] + (a - lo);
                t.nsub = (r.y - r.x + split_len - 1) / split_len;
            } else if (sub == 0) {  // the first sub-chunk takes the whole row, the others are empty
                t.v = vv;
                t.e0 = r.x;
                t.e1 = r.y;
            }
        } else {
            const int32_t pos = b == 1 ? lo + j : lo + j * (64 / G) + (lane / G);
            const bool ok = pos < hi2;
            const int32_t p = ok ? pos : lo;  // lo < hi2: the segment is not empty
            const int32_t vv = list[p];
            const int2 r = rows[p];
            if (ok) { t.v = vv; t.e0 = r.x; t.e1 = r.y; }
        }
        advance();
    };
    // stage B: the first U neighbor ids of the chunk (unconditional loads at clamped indices)
    auto load_ids = [&](const WalkChunk &t, int32_t *w) {
        const int gsz = (t.seg % NSEG_PER_RANK) ? 64 : G;
        const int32_t e = t.e0 + (lane & (gsz - 1));
#pragma unroll
        for (int u = 0; u < U; u++) {
            const int32_t eu = e + u * gsz;
            const bool ok = eu < t.e1;
            const int32_t wl = col[ok ? eu : 0];  // col has >= 1 entry (a stand-in when nnz = 0)
            w[u] = ok ? wl : -1;
        }
    };
    // stage C: neighbor colors (from the compact copy when there is one)
    auto gather_c = [&](const int32_t *w, int32_t *x) {
        if (CT == 0) {
            gather<U>(w, x, C, n);
        } else {
#pragma unroll
            for (int u = 0; u < U; u++) {
                const bool ok = (uint32_t)w[u] < (uint32_t)n;
                const int32_t xl = compact_load<CT>(S, ok ? w[u] : 0);
                x[u] = ok ? xl : 0;
            }
        }
    };
    // stage D: wait for lower ranks, First Fit, publish
    auto finish = [&](const WalkChunk &t, const int32_t *w, const int32_t *x) {
        const int b = t.seg % NSEG_PER_RANK;
        const int32_t s = t.seg / NSEG_PER_RANK;
        // (rows under 64 entries, the narrow variant's, span one or two batches:
        // deferring their waits gains nothing and costs registers)
        if (!FULL) finish_row<U, false, CT, false>(t, w, x, b ? 64 : G, col, n, C, S, lw, wc);
        else if (b == 2) finish_split<U, CT>(t, w, x, col, n, C, S, lw, hub_bits, hub_cnt, wc);
        // group rows (at most deg_wave entries, 64 by default) keep to the
        // register word: a color above 64 needs 64 lower-rank neighbors, and
        // the rare row that has them rescans in 64-color windows (RMAT-22
        // walk 2.39 -> 2.36 ms)
        else if (s < 64 || b == 0) finish_row<U, false, CT, true>(t, w, x, b ? 64 : G, col, n, C, S, lw, wc);
        else finish_row<U, true, CT, true>(t, w, x, b ? 64 : G, col, n, C, S, lw, wc);
    };

    // Software pipeline, one stage per iteration: chunk i+3's vertex and row
    // (A), chunk i+2's first U neighbor ids (B), chunk i+1's neighbor colors
    // (C, plain loads; stale or unfinished words are re-read in stage D), and
    // chunk i's waits, First Fit and store (D).  Every stage's inputs were
    // requested one iteration earlier.
    // trace: this wavefront's latest finish time in its current rank, one
    // atomic per (wavefront, rank) instead of one per vertex
    int32_t tr_rank = -1;
    unsigned long long tr_time = 0;
    auto trace_flush = [&]() {
        if (wc.trace && tr_rank >= 0 && lane == 0) atomicMax(&wc.trace[2 + 2 * (int64_t)tr_rank], tr_time);
    };
    advance();
    WalkChunk c0, c1, c2, c3;
    int32_t w0[U], w1[U], w2[U], x0[U], x1[U];
    load_chunk(c0);
    load_chunk(c1);
    load_chunk(c2);
    load_ids(c0, w0);
    load_ids(c1, w1);
    gather_c(w0, x0);
    while (c0.seg < nseg) {
        load_chunk(c3);                                  // A: chunk i+3
        if (c2.seg < nseg) load_ids(c2, w2);             // B: chunk i+2
        if (c1.seg < nseg) gather_c(w1, x1);             // C: chunk i+1
        finish(c0, w0, x0);                              // D: chunk i
        if (wc.trace) {
            const int32_t rk = c0.seg / NSEG_PER_RANK;
            if (rk != tr_rank) {
                trace_flush();
                tr_rank = rk;
            }
            tr_time = wall_clock64();
        }
        c0 = c1;
        c1 = c2;
        c2 = c3;
#pragma unroll
        for (int u = 0; u < U; u++) {
            w0[u] = w1[u];
            x0[u] = x1[u];
            w1[u] = w2[u];
        }
    }
    trace_flush();
}

// Persistent dataflow class walk (one launch per pass).
//
// Chunk assignment.  With xcd != 0 (and a grid that is a multiple of 8) the
// chunks of every segment are cut into 8 consecutive parts and part x goes to
// the workgroups b with b % 8 == x, which the hardware places on XCD x: the
// same region of the vertex order (for a mesh, the same slab) stays on one
// XCD for every class, so the neighbor colors it gathers stay in that XCD's
// L2.  Otherwise chunks go round robin over all wavefronts.  Either way every
// wavefront takes its chunks in increasing global order (segments in order,
// increasing position inside a segment), which the deadlock argument needs.
//
// Software pipeline (per wavefront): while chunk i gathers its neighbors'
// colors (the only loads that depend on earlier classes), chunk i+1's first
// U neighbor ids and chunk i+2's vertex and row are already being loaded.
// OPT: the variant that honours walk_flags and the class-completion trace;
// the other treats both as off (their run-time tests alone cost the mesh's
// walk 2.4 %).
template <int G, bool FULL, bool OPT>
__global__ void __launch_bounds__(WALK_BLOCK) k_walk_flow(const int2 *__restrict__ rows, const int32_t *__restrict__ col,
                                                          int32_t n, int32_t *C, const int32_t *__restrict__ list,
                                                          const int32_t *__restrict__ off,
                                                          const int32_t *__restrict__ coff,
                                                          const int32_t *__restrict__ segnz,
                                                          const int32_t *__restrict__ hsub,
                                                          const int32_t *__restrict__ sbase, int32_t split_len,
                                                          unsigned long long *hub_bits, int32_t *hub_cnt,
                                                          unsigned long long *scal, int32_t xcd, int32_t check_resident,
                                                          uint32_t spin_limit, uint32_t walk_flags,
                                                          unsigned long long *trace, void *S) {
    __shared__ int32_t t_off[WALK_TAB + 1], t_coff[WALK_TAB + 1], t_nz[WALK_TAB];
    __shared__ unsigned long long lmask[WALK_BLOCK];  // per wavefront: 64 mask words for colors above 64
    unsigned long long *lw = lmask + (threadIdx.x & ~63u);
    if (check_resident) {
        // start barrier, bounded: every workgroup checks in and waits for all
        // others; a timeout means they were not all resident (error bit 4).
        // check_resident == 2: residency probe only (short limit, no work).
        const uint32_t limit = check_resident == 2 ? (1u << 14) : spin_limit;
        if (threadIdx.x == 0) {
            atomicAdd(&scal[S_TICKET], 1ull);
            uint32_t it = 0;
            while (__hip_atomic_load(&scal[S_TICKET], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < gridDim.x) {
                if (++it > limit) {
                    atomicOr(&scal[S_ERR], 4ull);
                    if (check_resident == 1) atomicOr(&scal[S_STICKY], 4ull);  // the probe's failures are expected
                    break;
                }
                __builtin_amdgcn_s_sleep(2);
            }
        }
        __syncthreads();
        if (check_resident == 2) return;
    }
    const int32_t k = (int32_t)scal[S_K];
    const int32_t nseg = NSEG_PER_RANK * k;
    int32_t nnz_seg = (int32_t)scal[S_NZSEG];
    nnz_seg = nnz_seg < 0 ? 0 : (nnz_seg > nseg ? nseg : nnz_seg);
    if (!OPT) trace = nullptr;
    const WaitCtl wc = {scal, spin_limit, OPT ? walk_flags : 0u, trace};
    if (trace && threadIdx.x == 0) atomicMin(&trace[0], wall_clock64());
    if (nseg <= WALK_TAB) {
        // segment tables in LDS: their reads are tracked apart from the vector
        // loads in flight, so looking up the next chunk never drains the pipeline
        for (int32_t i = threadIdx.x; i <= nseg; i += WALK_BLOCK) { t_off[i] = off[i]; t_coff[i] = coff[i]; }
        for (int32_t i = threadIdx.x; i < nnz_seg; i += WALK_BLOCK) t_nz[i] = segnz[i];
        __syncthreads();
        if (k <= CT_MAX_K1)
            walk_body<G, true, FULL, 1>(t_off, t_coff, t_nz, nnz_seg, nseg, rows, col, n, C, list, hsub, sbase, split_len, hub_bits,
                                        hub_cnt, wc, xcd, lw, S);
        else
            walk_body<G, true, FULL, 2>(t_off, t_coff, t_nz, nnz_seg, nseg, rows, col, n, C, list, hsub, sbase, split_len, hub_bits,
                                        hub_cnt, wc, xcd, lw, S);
    } else {
        walk_body<G, false, FULL, 0>(off, coff, nullptr, nseg, nseg, rows, col, n, C, list, hsub, sbase, split_len, hub_bits, hub_cnt,
                                     wc, xcd, lw, S);
    }
    if (trace && __lane_id() == 0) atomicMax(&trace[1], wall_clock64());
}

// One launch per class (host loop): every vertex of rank s, one lane each.
__global__ void k_walk_class(const int32_t *__restrict__ rp, const int32_t *__restrict__ col, int64_t nnz, int32_t n,
                             int32_t *C, const int32_t *__restrict__ list, const int32_t *__restrict__ off, int32_t s) {
    const int32_t a = off[NSEG_PER_RANK * s], b = off[NSEG_PER_RANK * s + NSEG_PER_RANK];
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = a + (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < b; i += stride) {
        int32_t v = list[i];
        int32_t e0, e1;
        row_range(rp, v, nnz, e0, e1);
        C[v] = select_color_lane(col, e0, e1, C, n, 0u);
    }
}

typedef void (*walk_fn)(const int2 *, const int32_t *, int32_t, int32_t *, const int32_t *, const int32_t *,
                        const int32_t *, const int32_t *, const int32_t *, const int32_t *, int32_t,
                        unsigned long long *, int32_t *,
                        unsigned long long *, int32_t, int32_t, uint32_t, uint32_t, unsigned long long *, void *);

template <bool FULL, bool OPT>
static walk_fn walk_kernel_t(int G) {
    switch (G) {
        case 1: return k_walk_flow<1, FULL, OPT>;
        case 2: return k_walk_flow<2, FULL, OPT>;
        case 4: return k_walk_flow<4, FULL, OPT>;
        case 8: return k_walk_flow<8, FULL, OPT>;
        case 16: return k_walk_flow<16, FULL, OPT>;
        case 32: return k_walk_flow<32, FULL, OPT>;
        default: return k_walk_flow<64, FULL, OPT>;
    }
}

static walk_fn walk_kernel(int G, bool full, bool opt) {
    if (opt) return full ? walk_kernel_t<true, true>(G) : walk_kernel_t<false, true>(G);
    return full ? walk_kernel_t<true, false>(G) : walk_kernel_t<false, false>(G);
}

// The walk variant of this context's settings.  The variant with split
// rows takes the options-free kernel unless walk_flags or the trace ask for
// them (RMAT-22: 2.71 -> 2.39 ms per walk); the narrow variant keeps the
// run-time tests (measured the other way round there: 151.6 against 155.0 us
// on the mesh, the same GPU).
static bool walk_opt(const gc_ctx *ctx, bool full) {
    return !full || ctx->tune.walk_flags != 0 || ctx->tune.trace != 0;
}

// full: the variant with split rows and LDS mask words (rows of 64 or more
// entries); the narrow one keeps only a 64-color register window (further
// windows rescan the row) and lets the first sub-chunk of a split row scan the
// whole row.
// Histogram grid: one workgroup per tile up to two per CU (longer-lived
// workgroups measured faster than one short one per tile), else consecutive
// tiles per workgroup.
static int hist_grid_for(const gc_ctx *ctx, int32_t n, int block) {
    const int64_t tiles = ((int64_t)n + block * HIST_ITEMS - 1) / (block * HIST_ITEMS);
    const int64_t cap = 2 * (int64_t)ctx->num_cu;
    return (int)(tiles <= cap ? tiles : cap);
}

// Co-resident grid of the walk variant for this graph, measured on its first
// use.  Runs before a pass's own kernels: the probe clears the error slot,
// which would otherwise lose what the pass's histogram recorded there.
static gc_status measure_walk(gc_ctx *ctx, const gc_csr *g, int32_t *C, bool full, hipStream_t s) {
    const int G = gc_walk_group(ctx, full);
    const bool opt = walk_opt(ctx, full);
    walk_fn f = walk_kernel(G, full, opt);
    const int variant = 4 * G + (opt ? 2 : 0) + (full ? 1 : 0);
    // the walk reads col[0] unconditionally (masked afterwards): give it one valid word when the graph has no edges
    const int32_t *col = g->nnz > 0 ? g->col_idx : (const int32_t *)ctx->scal;
    // without split rows the hub arrays are never touched
    int32_t *hub_cnt = ctx->hub_cnt ? ctx->hub_cnt : (int32_t *)ctx->scal;
    unsigned long long *hub_bits = ctx->hub_bits ? ctx->hub_bits : ctx->scal;
    const int32_t split_len = ctx->tune.split_len;
    const uint32_t spin_limit = ctx->tune.spin_limit > 0 ? (uint32_t)ctx->tune.spin_limit : SPIN_LIMIT;
    if (ctx->walk_blocks_v[variant] == 0) {
        // The occupancy query is an upper bound; the walk needs every workgroup
        // resident at once, so measure it: a probe launch (no work) where every
        // workgroup checks in and waits, bounded, for all the others.  Step the
        // grid down one workgroup per CU until the probe passes.
        int per_cu = 0;
        GC_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, reinterpret_cast<const void *>(f), WALK_BLOCK, 0));
        if (per_cu < 1) return gc_fail(ctx, GC_ERR_DEVICE, "walk kernel cannot be resident");
        int blocks = 0;
        for (; per_cu >= 1; per_cu--) {
            blocks = per_cu * ctx->num_cu;
            if (blocks >= 8) blocks -= blocks & 7;
            GC_HIP(hipMemsetAsync(ctx->scal + S_TICKET, 0, 8, s));
            GC_HIP(hipMemsetAsync(ctx->scal + S_ERR, 0, 8, s));
            hipLaunchKernelGGL(f, dim3(blocks), dim3(WALK_BLOCK), 0, s, ctx->rows, col, g->n, C, ctx->list, ctx->off,
                               ctx->coff, ctx->segnz, ctx->hsub, ctx->sbase, split_len, hub_bits, hub_cnt, ctx->scal, 0, 2,
                               spin_limit, 0u, nullptr, ctx->shadow);
            GC_LAUNCHED();
            gc_status st = gc_sync_scalars(ctx, s);
            if (st) return st;
            if (!(ctx->hscal[S_ERR] & 4)) break;
        }
        if (per_cu < 1) return gc_fail(ctx, GC_ERR_DEVICE, "walk kernel: no grid was fully resident");
        GC_HIP(hipMemsetAsync(ctx->scal + S_ERR, 0, 8, s));
        ctx->walk_blocks_v[variant] = blocks;
    }
    return GC_OK;
}

static gc_status launch_walk_flow(gc_ctx *ctx, const gc_csr *g, int32_t *C, bool full, hipStream_t s) {
    const int G = gc_walk_group(ctx, full);
    const bool opt = walk_opt(ctx, full);
    walk_fn f = walk_kernel(G, full, opt);
    const int variant = 4 * G + (opt ? 2 : 0) + (full ? 1 : 0);
    if (ctx->walk_blocks_v[variant] == 0) return gc_fail(ctx, GC_ERR_DEVICE, "walk grid not measured");
    const int32_t *col = g->nnz > 0 ? g->col_idx : (const int32_t *)ctx->scal;
    int32_t *hub_cnt = ctx->hub_cnt ? ctx->hub_cnt : (int32_t *)ctx->scal;
    unsigned long long *hub_bits = ctx->hub_bits ? ctx->hub_bits : ctx->scal;
    const int32_t split_len = ctx->tune.split_len;
    const uint32_t spin_limit = ctx->tune.spin_limit > 0 ? (uint32_t)ctx->tune.spin_limit : SPIN_LIMIT;
    ctx->walk_blocks = ctx->walk_blocks_v[variant];
    // An ordinary stream-ordered launch whose grid is what the device holds at
    // once (measured above): the kernel starts after the previous kernel of the
    // stream has finished, so every workgroup is dispatched at once on an
    // otherwise idle device (kernels of other streams can only delay some
    // workgroups until they finish; the bounded waits keep even that case from
    // hanging).
    // XCD parts keep a region of the vertex order in one XCD's L2 when
    // neighbors are near in that order (the mesh: traffic 2.04 -> 1.39x the
    // algorithmic bytes); with mostly far neighbors there is no such region,
    // and the parts only unbalance the wavefronts (RMAT-22 walk 2.25 -> 1.93 ms
    // round robin).  The far fraction comes with the graph's longest row.
    const int32_t xcd = ctx->tune.xcd_chunks > 0 ? 1 : (ctx->tune.xcd_chunks == 0 ? 0 : (ctx->deg_far <= 0.5 ? 1 : 0));
    if (ctx->tune.check_resident) GC_HIP(hipMemsetAsync(ctx->scal + S_TICKET, 0, 8, s));
    unsigned long long *trace = nullptr;
    if (ctx->tune.trace) {
        const size_t words = 2 + 2 * ((size_t)ctx->ccap + 2);
        if (!ctx->trace) {
            GC_HIP(hipStreamSynchronize(s));
            if (hipMalloc((void **)&ctx->trace, words * 8) != hipSuccess)
                return gc_fail(ctx, GC_ERR_OOM, "walk trace of %zu words", words);
        }
        GC_HIP(hipMemsetAsync(ctx->trace, 0, words * 8, s));
        GC_HIP(hipMemsetAsync(ctx->trace, 0xFF, 8, s));  // walk start: a minimum
        trace = ctx->trace;
    }
    GC_TIMED(GC_K_WALK, s, hipLaunchKernelGGL(f, dim3(ctx->walk_blocks), dim3(WALK_BLOCK), 0, s, ctx->rows, col, g->n, C,
                                              ctx->list, ctx->off, ctx->coff, ctx->segnz, ctx->hsub, ctx->sbase,
                                              split_len,
                                              hub_bits, hub_cnt, ctx->scal, xcd, ctx->tune.check_resident,
                                              spin_limit, (uint32_t)ctx->tune.walk_flags, trace, ctx->shadow));
    GC_LAUNCHED();
    return GC_OK;
}

// One pass; dist 2 recolors a distance-2 coloring (one launch per class over
// the distance-2 neighborhoods).
static gc_status recolor_pass(gc_ctx *ctx, const gc_csr *g, int32_t perm, uint64_t seed, int32_t pass,
                              const int32_t *colors_in, int32_t *colors_out, gc_stats *st, void *stream, int dist) {
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
    status = gc_check_input_coloring(ctx, g, colors_in, stream, dist);
    if (status) return status;
    if (dist == 2) {
        int32_t maxdeg = 0;
        status = gc_graph_max_degree(ctx, g, s, &maxdeg);
        if (status) return status;
        if (maxdeg >= GC_D2_MAX_DEGREE)
            return gc_fail(ctx, GC_ERR_ARG, "distance-2 recoloring takes rows below %d entries", GC_D2_MAX_DEGREE);
    }
    const int block = 256;
    const int32_t deg_wave = ctx->tune.deg_wave;
    // the split bin exists in the persistent walk only
    const bool flow = ctx->tune.walk_mode == 0 && dist == 1;
    bool full = false;
    if (flow) {
        int32_t maxdeg = 0;
        status = gc_graph_max_degree(ctx, g, s, &maxdeg);
        if (status) return status;
        full = maxdeg >= 64;
    }
    const int32_t deg_split = full ? ctx->tune.deg_split : 0;
    const int G = gc_walk_group(ctx, full);  // lanes per vertex of the walk; sets the chunk size of bin 0
    const int32_t split_len = ctx->tune.split_len;
    const int32_t hub_max_rank = 64 * ctx->tune.hub_words - 1;
    if (deg_split > 0) {
        status = gc_ensure_hub_slots(ctx, g->nnz, deg_split, s);
        if (status) return status;
    }
    const int hist_grid = hist_grid_for(ctx, n, block);
    if (flow) {
        status = measure_walk(ctx, g, colors_out, full, s);
        if (status) return status;
    }
    // max, min, error flags (and the conflict count, which its users clear
    // anyway): 32 aligned bytes, one fill launch
    static_assert(S_MAXC == 2 && S_ERR == 4 && S_CONFLICTS == 5, "scalar slots cleared per pass");
    GC_HIP(hipMemsetAsync(ctx->scal + S_MAXC, 0, 32, s));
    int32_t maxdeg_h = 0;
    status = gc_graph_max_degree(ctx, g, s, &maxdeg_h);
    if (status) return status;
    const int32_t bins = maxdeg_h > deg_wave ? 1 : 0;
    GC_TIMED(GC_K_HIST, s, k_hist<<<hist_grid, block, 0, s>>>(n, colors_in, g->row_ptr, g->nnz, bins, deg_wave, deg_split,
                                                             split_len, ctx->ccap, ctx->hist, ctx->histw, ctx->hist_s,
                                                             ctx->hist_sc, ctx->hcopy, ctx->scal));
    GC_LAUNCHED();
    // The methods' colorings use at most (longest row + X) colors.  When that
    // bound fits the class order's LDS path, a quarter of the threads is
    // faster (shorter barriers); an input beyond the bound only takes longer,
    // its result is the same.
    int32_t maxdeg_o = 0;
    status = gc_graph_max_degree(ctx, g, s, &maxdeg_o);
    if (status) return status;
    const bool order_small = (int64_t)maxdeg_o + GC_MAX_X + 1 <= ORDER_LDS;
    const int order_threads = order_small ? PERM_THREADS_SMALL : PERM_THREADS;
    auto order_kernel = order_small ? k_class_order<PERM_THREADS_SMALL> : k_class_order<PERM_THREADS>;
    GC_TIMED(GC_K_ORDER, s, order_kernel<<<1, order_threads, 0, s>>>(
                                ctx->ccap, perm, gc_stream_value(seed, GC_TAG_PERM, (uint32_t)pass), 64 / G, hub_max_rank, ctx->hist,
                                ctx->histw, ctx->hist_s, ctx->hist_sc, (int32_t *)ctx->keys, ctx->pi, ctx->rank,
                                ctx->off, ctx->coff, ctx->cursor, ctx->sbase, ctx->hcopy, ctx->segnz, ctx->scal));
    GC_LAUNCHED();
    static_assert(SCATTER_BLOCK == 256, "scatter tiles share the histogram's block size");
    const int64_t tiles = ((int64_t)n + SCATTER_BLOCK * SCATTER_ITEMS - 1) / (SCATTER_BLOCK * SCATTER_ITEMS);
    GC_TIMED(GC_K_SCATTER, s, k_scatter<<<(unsigned)tiles, SCATTER_BLOCK, 0, s>>>(n, colors_in, colors_out, ctx->shadow, g->row_ptr, g->nnz,
                                                                         deg_wave, deg_split, hub_max_rank, ctx->ccap,
                                                                         ctx->rank,
                                                                         ctx->cursor, ctx->list, ctx->rows, ctx->pi, ctx->off,
                                                                         ctx->hcopy + (size_t)2 * GC_HIST_COPIES * HIST_LDS,
                                                                         hist_grid, ctx->scal));
    GC_LAUNCHED();
    if (deg_split > 0) {
        GC_TIMED(GC_K_SCATTER, s, k_split_prefix<<<4, 256, 0, s>>>(ctx->off, ctx->rows, split_len, ctx->hsub, ctx->scal));
        GC_LAUNCHED();
    }
    if (flow) {
        status = launch_walk_flow(ctx, g, colors_out, full, s);
        if (status) return status;
    } else if (dist == 2) {
        status = gc_sync_scalars(ctx, s);
        if (status) return status;
        if (ctx->hscal[S_ERR] & 1) return gc_fail(ctx, GC_ERR_COLORING, "input color outside [1, %d]", ctx->ccap);
        const int32_t k = (int32_t)ctx->hscal[S_K];
        std::vector<int32_t> off((size_t)NSEG_PER_RANK * k + 1);
        GC_HIP(hipMemcpyAsync(off.data(), ctx->off, off.size() * 4, hipMemcpyDeviceToHost, s));
        GC_HIP(hipStreamSynchronize(s));
        status = gc_d2_classes(ctx, g, colors_out, k, off.data(), NSEG_PER_RANK, s);
        if (status) return status;
    } else {
        status = gc_sync_scalars(ctx, s);
        if (status) return status;
        if (ctx->hscal[S_ERR] & 1) return gc_fail(ctx, GC_ERR_COLORING, "input color outside [1, %d]", ctx->ccap);
        const int32_t k = (int32_t)ctx->hscal[S_K];
        for (int32_t r = 0; r < k; r++) {
            GC_TIMED(GC_K_WALK, s, k_walk_class<<<gc_grid(ctx, n, block), block, 0, s>>>(g->row_ptr, g->col_idx, g->nnz,
                                                                                      n, colors_out, ctx->list,
                                                                                      ctx->off, r));
            GC_LAUNCHED();
        }
    }
    if (st) {
        status = gc_count_device(ctx, n, colors_out, s, true);
        if (status) return status;
        status = gc_sync_scalars(ctx, s);
        if (status) return status;
        if (ctx->hscal[S_ERR] & 1) return gc_fail(ctx, GC_ERR_COLORING, "input color outside [1, %d]", ctx->ccap);
        // a walk failure of this pass (S_ERR bits 1, 2) is also in the sticky
        // record harvested by the synchronization above: the public entry
        // point reports it
        st->rounds = 0;
        st->losers_total = 0;
        st->k_classes = (int32_t)ctx->hscal[S_K];
        st->num_colors = (int32_t)ctx->hscal[S_NUMC];
        st->max_color = (int32_t)ctx->hscal[S_MAXC];
    }
    return GC_OK;
}

static gc_status gc_recolor_impl(gc_ctx *ctx, const gc_csr *g, int32_t perm, uint64_t seed, int32_t pass,
                                const int32_t *colors_in, int32_t *colors_out, gc_stats *st, void *stream) {
    return recolor_pass(ctx, g, perm, seed, pass, colors_in, colors_out, st, stream, 1);
}

static gc_status gc_recolor_d2_impl(gc_ctx *ctx, const gc_csr *g, int32_t perm, uint64_t seed, int32_t pass,
                                   const int32_t *colors_in, int32_t *colors_out, gc_stats *st, void *stream) {
    return recolor_pass(ctx, g, perm, seed, pass, colors_in, colors_out, st, stream, 2);
}

// ---------------------------------------------------------------------------
// Asynchronous recoloring aRC (section 3): the classes of the input coloring,
// ordered by `perm`, give every vertex a rank; the speculative rounds of the
// initial coloring then run with First Fit, and of two neighbors with the
// same tentative color the one of the earlier class keeps it.
// ---------------------------------------------------------------------------

__global__ void k_vertex_rank(int32_t n, const int32_t *__restrict__ C, const int32_t *__restrict__ rank, int32_t ccap,
                              int32_t *__restrict__ prank) {
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x) {
        const int32_t c = C[v];
        prank[v] = (c >= 1 && c <= ccap) ? rank[c] : INT32_MAX;
    }
}

static gc_status gc_arc_recolor_impl(gc_ctx *ctx, const gc_csr *g, int32_t perm, uint64_t seed, int32_t pass,
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
    status = gc_check_input_coloring(ctx, g, colors_in, stream, 1);
    if (status) return status;
    const int block = 256;
    // class sizes and order (no split bins: only the ranks are used)
    const int hist_grid = hist_grid_for(ctx, n, block);
    // max, min, error flags (and the conflict count, which its users clear
    // anyway): 32 aligned bytes, one fill launch
    static_assert(S_MAXC == 2 && S_ERR == 4 && S_CONFLICTS == 5, "scalar slots cleared per pass");
    GC_HIP(hipMemsetAsync(ctx->scal + S_MAXC, 0, 32, s));
    GC_TIMED(GC_K_HIST, s, k_hist<<<hist_grid, block, 0, s>>>(n, colors_in, g->row_ptr, g->nnz, 0, ctx->tune.deg_wave, 0,
                                                             ctx->tune.split_len, ctx->ccap, ctx->hist, ctx->histw,
                                                             ctx->hist_s, ctx->hist_sc, ctx->hcopy, ctx->scal));
    GC_LAUNCHED();
    GC_TIMED(GC_K_ORDER, s, k_class_order<PERM_THREADS><<<1, PERM_THREADS, 0, s>>>(
                                ctx->ccap, perm, gc_stream_value(seed, GC_TAG_PERM, (uint32_t)pass), 1,
                                64 * ctx->tune.hub_words - 1, ctx->hist, ctx->histw, ctx->hist_s, ctx->hist_sc,
                                (int32_t *)ctx->keys, ctx->pi, ctx->rank, ctx->off, ctx->coff, ctx->cursor, ctx->sbase,
                                ctx->hcopy, ctx->segnz, ctx->scal));
    GC_LAUNCHED();
    int32_t *prank = ctx->list;  // free outside the recoloring walk
    GC_TIMED(GC_K_OTHER, s, k_vertex_rank<<<gc_grid(ctx, n, block), block, 0, s>>>(n, colors_in, ctx->rank, ctx->ccap,
                                                                                   prank));
    GC_LAUNCHED();
    status = gc_sync_scalars(ctx, s);
    if (status) return status;
    if (ctx->hscal[S_ERR] & 1) return gc_fail(ctx, GC_ERR_COLORING, "input color outside [1, %d]", ctx->ccap);
    const int32_t k = (int32_t)ctx->hscal[S_K];
    status = gc_spec_rounds(ctx, g, GC_FIRST_FIT, 1, seed, 0, 0, colors_out, st, s, prank);
    if (status) return status;
    if (st) st->k_classes = k;
    return GC_OK;
}

// Public entry points: the implementations above, with any sticky device
// failure harvested on the way reported in the returned status.
extern "C" gc_status gc_recolor(gc_ctx *ctx, const gc_csr *g, int32_t perm, uint64_t seed, int32_t pass,
                                const int32_t *colors_in, int32_t *colors_out, gc_stats *st, void *stream) {
    return gc_report(ctx, gc_recolor_impl(ctx, g, perm, seed, pass, colors_in, colors_out, st, stream));
}

static gc_status gc_recolor_passes_impl(gc_ctx *ctx, const gc_csr *g, const int32_t *perms, int32_t passes,
                                        uint64_t seed, int32_t pass0, const int32_t *colors_in, int32_t *colors_out,
                                        gc_stats *st, void *stream) {
    gc_status status = gc_check_graph_args(ctx, g);
    if (status) return status;
    if (passes < 0 || pass0 < 0 || (int64_t)pass0 + passes > INT32_MAX) return gc_fail(ctx, GC_ERR_ARG, "bad pass range");
    if (passes > 0 && !perms) return gc_fail(ctx, GC_ERR_ARG, "perms is NULL");
    for (int32_t p = 0; p < passes; p++)
        if (perms[p] < 0 || perms[p] > 3) return gc_fail(ctx, GC_ERR_ARG, "perms[%d] must be in [0, 3]", p);
    if (g->n > 0 && (!colors_in || !colors_out)) return gc_fail(ctx, GC_ERR_ARG, "colors is NULL");
    hipStream_t s = (hipStream_t)stream;
    GC_HIP(hipSetDevice(ctx->device));
    if (passes == 0) {
        if (g->n > 0 && colors_out != colors_in)
            GC_HIP(hipMemcpyAsync(colors_out, colors_in, (size_t)g->n * 4, hipMemcpyDeviceToDevice, s));
        return GC_OK;
    }
    for (int32_t p = 0; p < passes; p++) {
        status = recolor_pass(ctx, g, perms[p], seed, pass0 + p, p == 0 ? colors_in : colors_out, colors_out,
                              st ? &st[p] : nullptr, stream, 1);
        if (status) return status;
    }
    return GC_OK;
}

extern "C" gc_status gc_recolor_passes(gc_ctx *ctx, const gc_csr *g, const int32_t *perms, int32_t passes, uint64_t seed,
                                       int32_t pass0, const int32_t *colors_in, int32_t *colors_out, gc_stats *st,
                                       void *stream) {
    return gc_report(ctx, gc_recolor_passes_impl(ctx, g, perms, passes, seed, pass0, colors_in, colors_out, st, stream));
}

extern "C" gc_status gc_recolor_d2(gc_ctx *ctx, const gc_csr *g, int32_t perm, uint64_t seed, int32_t pass,
                                   const int32_t *colors_in, int32_t *colors_out, gc_stats *st, void *stream) {
    return gc_report(ctx, gc_recolor_d2_impl(ctx, g, perm, seed, pass, colors_in, colors_out, st, stream));
}

extern "C" gc_status gc_arc_recolor(gc_ctx *ctx, const gc_csr *g, int32_t perm, uint64_t seed, int32_t pass,
                                    const int32_t *colors_in, int32_t *colors_out, gc_stats *st, void *stream) {
    return gc_report(ctx, gc_arc_recolor_impl(ctx, g, perm, seed, pass, colors_in, colors_out, st, stream));
}
