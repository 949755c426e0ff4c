// gc_recolor.hip - one iterated-greedy recoloring pass (section 2.1,
// Culberson's Iterated Greedy; section 3, synchronous recoloring RC with the
// RV / NI / ND / RAND class permutations).
//
// Steps on the device:
//   1. histogram of the input colors (workgroup-private in LDS), split by
//      degree bin (bin 1 = rows longer than deg_wave), and the max color;
//   2. class order (one workgroup): compacts the non-empty classes, orders
//      them, gives every color its rank, and lays out the grouped vertex list
//      as segments (rank, bin) with list offsets and work-chunk offsets;
//   3. scatter: counting sort of the vertices into their segments; the output
//      array is set to -(rank + 1), i.e. "not yet recolored, class rank r";
//   4. class walk: every vertex of rank s takes the smallest positive color
//      not held by a neighbor of lower rank (those are recolored before it).
//
// The walk runs as ONE persistent launch (every workgroup resident) without
// grid barriers.
// Work chunks never straddle two ranks and every wavefront takes its chunks
// in increasing order, so a vertex only ever waits for vertices of earlier
// chunks: a vertex of rank s reads each neighbor's word; a positive word is a
// final color of a lower rank; a negative word names the neighbor's rank, and
// only ranks below s are waited for (an agent-scope load loop, bounded).
// With every workgroup co-resident the earliest
// unfinished chunk can always proceed, so the walk cannot deadlock.  Final
// colors are written with agent-scope stores so that waiting wavefronts on
// other XCDs see them; a word only ever changes from negative to its final
// positive value, so a plain (possibly L2-stale) load that sees a positive
// value is exact, and a stale negative value of a lower rank just falls into
// the coherent wait loop.
#include "gc_internal.h"

#define HIST_LDS 4096       // colors below this use the workgroup-private histogram
#define HIST_BITS 12
#define PERM_THREADS 1024
#define SCATTER_BINS 1024   // segments below this reserve list ranges once per workgroup
#define SCATTER_ITEMS 4
#define WALK_BLOCK 256
#define SPIN_LIMIT (1u << 20)

__global__ void k_hist(int32_t n, const int32_t *__restrict__ Cin, const int32_t *__restrict__ rp, int64_t nnz,
                       int32_t deg_wave, int32_t ccap, int32_t *__restrict__ hist, int32_t *__restrict__ histw,
                       unsigned long long *scal) {
    __shared__ int32_t h[HIST_LDS], hw[HIST_LDS];
    __shared__ int32_t lds[32];
    for (int i = threadIdx.x; i < HIST_LDS; i += blockDim.x) { h[i] = 0; hw[i] = 0; }
    __syncthreads();
    int32_t mx = 0;
    bool bad = false;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t base = (int64_t)blockIdx.x * blockDim.x; base < n; base += stride) {
        const int64_t v = base + threadIdx.x;
        int32_t c = 0;
        bool valid = false, wave = false;
        if (v < n) {
            c = Cin[v];
            mx = max(mx, c);
            if (c < 1 || c > ccap) bad = true;
            else {
                valid = true;
                int32_t e0, e1;
                row_range(rp, (int32_t)v, nnz, e0, e1);
                wave = e1 - e0 > deg_wave;
            }
        }
        const bool in_lds = valid && c < HIST_LDS;
        (void)wave_match_reserve_bits(h, c, in_lds, HIST_BITS);
        (void)wave_match_reserve_bits(hw, c, in_lds && wave, HIST_BITS);
        if (valid && !in_lds) {
            atomicAdd(&hist[c], 1);
            if (wave) atomicAdd(&histw[c], 1);
        }
    }
    const int32_t bmax = block_max_i32(mx, lds);  // synchronizes the block
    const int32_t top = bmax < HIST_LDS - 1 ? bmax : HIST_LDS - 1;
    for (int i = threadIdx.x + 1; i <= top; i += blockDim.x) {
        if (h[i]) atomicAdd(&hist[i], h[i]);
        if (hw[i]) atomicAdd(&histw[i], hw[i]);
    }
    unsigned long long anybad = __ballot(bad);
    if (__lane_id() == 0 && anybad) atomicOr(&scal[S_ERR], 1ull);
    if (threadIdx.x == 0) atomicMax((int *)&scal[S_MAXC], bmax);
}

// Class order and segment layout (one workgroup).  Segment 2s holds the
// rank-s vertices of the lane-group bin, segment 2s+1 those of the
// wavefront bin.  off[g] / coff[g]: first list slot / first work chunk of
// segment g (off[2k] = n, coff[2k] = chunks); cursor[g] = off[g].  A chunk is
// vpc vertices of a lane-group segment or one vertex of a wavefront segment.
__global__ void __launch_bounds__(PERM_THREADS) k_class_order(int32_t ccap, int32_t perm, uint32_t s_perm, int32_t vpc,
                                                               int32_t *hist, int32_t *histw, int32_t *cls, int32_t *pi,
                                                               int32_t *rank, int32_t *off, int32_t *coff,
                                                               int32_t *cursor, unsigned long long *scal) {
    __shared__ int32_t lds[32];
    int32_t maxc = (int32_t)scal[S_MAXC];
    if (maxc > ccap) maxc = ccap;
    const int32_t k = block_class_order(maxc, perm, s_perm, hist, cls, pi, rank, nullptr, nullptr, lds);
    const int32_t nseg = 2 * k;
    int32_t acc = 0, cacc = 0;
    for (int32_t base = 0; base < nseg; base += blockDim.x) {
        int32_t g = base + (int32_t)threadIdx.x;
        int32_t sz = 0, ch = 0;
        if (g < nseg) {
            int32_t c = pi[g >> 1];
            int32_t w = histw[c];
            sz = (g & 1) ? w : hist[c] - w;
            ch = (g & 1) ? sz : (sz + vpc - 1) / vpc;
        }
        int32_t tot, ctot;
        int32_t ex = block_exclusive_scan(sz, &tot, lds);
        int32_t cex = block_exclusive_scan(ch, &ctot, lds);
        if (g < nseg) {
            off[g] = acc + ex;
            cursor[g] = acc + ex;
            coff[g] = cacc + cex;
        }
        acc += tot;
        cacc += ctot;
    }
    if (threadIdx.x == 0) {
        off[nseg] = acc;
        coff[nseg] = cacc;
        scal[S_K] = (unsigned long long)k;
    }
    __syncthreads();
    for (int32_t c = threadIdx.x; c <= maxc; c += blockDim.x) {
        hist[c] = 0;
        histw[c] = 0;
    }
}

// Counting-sort scatter into segments: one tile of SCATTER_ITEMS * blockDim
// vertices per workgroup; segments below SCATTER_BINS reserve their list
// range once per workgroup.  Writes Cout[v] = -(rank + 1).
__global__ void k_scatter(int32_t n, const int32_t *Cin, int32_t *Cout, const int32_t *__restrict__ rp, int64_t nnz,
                          int32_t deg_wave, int32_t ccap, const int32_t *__restrict__ rank, int32_t *__restrict__ cursor,
                          int32_t *__restrict__ list, int2 *__restrict__ rows,
                          const unsigned long long *__restrict__ scal) {
    __shared__ int32_t cnt[SCATTER_BINS];
    __shared__ int32_t basepos[SCATTER_BINS];
    const int32_t k = (int32_t)scal[S_K];
    const int32_t nseg = 2 * k;
    const int32_t bins = nseg < SCATTER_BINS ? nseg : SCATTER_BINS;
    const int gbits = key_bits(bins);
    for (int i = threadIdx.x; i < bins; i += blockDim.x) cnt[i] = 0;
    __syncthreads();
    const int64_t tile = (int64_t)blockIdx.x * blockDim.x * SCATTER_ITEMS;
    int32_t sg[SCATTER_ITEMS], loc[SCATTER_ITEMS];
    int2 rw[SCATTER_ITEMS];
#pragma unroll
    for (int it = 0; it < SCATTER_ITEMS; it++) {
        int64_t v = tile + (int64_t)it * blockDim.x + threadIdx.x;
        sg[it] = -1;
        loc[it] = -1;
        int32_t g = -1;
        if (v < n) {
            int32_t c = Cin[v];
            if (c >= 1 && c <= ccap && k > 0) {
                int32_t s = rank[c];
                if ((uint32_t)s >= (uint32_t)k) s = k - 1;  // unreachable for a ranked color; keeps indices in bounds
                int32_t e0, e1;
                row_range(rp, (int32_t)v, nnz, e0, e1);
                rw[it] = make_int2(e0, e1);
                g = 2 * s + (e1 - e0 > deg_wave ? 1 : 0);
                sg[it] = g;
                if (g >= SCATTER_BINS) {
                    int32_t p = atomicAdd(&cursor[g], 1);
                    list[p] = (int32_t)v;
                    rows[p] = rw[it];
                    Cout[v] = -(s + 1);
                }
            } else {
                Cout[v] = 0;
            }
        }
        const bool in_lds = g >= 0 && g < SCATTER_BINS;
        const int32_t pos = wave_match_reserve_bits(cnt, g, in_lds, gbits);
        if (in_lds) loc[it] = pos;
    }
    __syncthreads();
    for (int i = threadIdx.x; i < bins; i += blockDim.x)
        if (cnt[i]) basepos[i] = atomicAdd(&cursor[i], cnt[i]);
    __syncthreads();
#pragma unroll
    for (int it = 0; it < SCATTER_ITEMS; it++) {
        int64_t v = tile + (int64_t)it * blockDim.x + threadIdx.x;
        if (loc[it] >= 0) {
            const int32_t p = basepos[sg[it]] + loc[it];
            list[p] = (int32_t)v;
            rows[p] = rw[it];
            Cout[v] = -((sg[it] >> 1) + 1);
        }
    }
}

// Waits (bounded) until *p holds a positive value, reading past the L2.  If
// any wait of the launch has already given up, returns at once, so a broken
// dependency cannot stretch the kernel beyond about one wait limit.
__device__ inline int32_t wait_positive(int32_t *p, unsigned long long *scal) {
    for (uint32_t it = 0; it < SPIN_LIMIT; it++) {
        int32_t x = __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (x > 0) return x;
        if ((it & 1023u) == 1023u &&
            (__hip_atomic_load(&scal[S_ERR], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) & 6ull))
            return 0;
        __builtin_amdgcn_s_sleep(2);
    }
    atomicOr(&scal[S_ERR], 2ull);  // gives up: the result is wrong but the kernel ends
    return 0;
}


// One work chunk as a wavefront sees it: segment (rank 2s / 2s+1 = bin), the
// vertex of this lane's group (-1: none) and its row.
struct WalkChunk {
    int32_t seg, v, e0, e1;
};

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
// U neighbor ids and chunk i+2's vertex and row are already being loaded, so
// one memory round trip per chunk sits on the dependency path instead of
// four.  Group size: G lanes per vertex in even (lane-group) segments, the
// whole wavefront in odd (long-row) segments.
#define WALK_TAB 1024  // segment tables of up to WALK_TAB segments (512 classes) live in LDS

template <int G, bool LDS_TAB>
__device__ __forceinline__ void walk_body(const int32_t *O, const int32_t *CO, int32_t nseg,
                                          const int2 *__restrict__ rows, const int32_t *__restrict__ col, int64_t nnz,
                                          int32_t n, int32_t *C, const int32_t *__restrict__ list,
                                          unsigned long long *scal, int32_t xcd);

template <int G>
__global__ void __launch_bounds__(WALK_BLOCK) k_walk_flow(const int2 *__restrict__ rows, const int32_t *__restrict__ col,
                                                          int64_t nnz, int32_t n, int32_t *C,
                                                          const int32_t *__restrict__ list, const int32_t *__restrict__ off,
                                                          const int32_t *__restrict__ coff, unsigned long long *scal,
                                                          int32_t xcd, int32_t check_resident) {
    __shared__ int32_t t_off[WALK_TAB + 1], t_coff[WALK_TAB + 1];
    if (check_resident) {
        // start barrier, bounded: every workgroup checks in and waits for all
        // others; a timeout means they were not all resident (error bit 4).
        // check_resident == 2: residency probe only (short limit, no work).
        const uint32_t limit = check_resident == 2 ? (1u << 14) : SPIN_LIMIT;
        if (threadIdx.x == 0) {
            atomicAdd(&scal[S_TICKET], 1ull);
            uint32_t it = 0;
            while (__hip_atomic_load(&scal[S_TICKET], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < gridDim.x) {
                if (++it > limit) { atomicOr(&scal[S_ERR], 4ull); break; }
                __builtin_amdgcn_s_sleep(2);
            }
        }
        __syncthreads();
        if (check_resident == 2) return;
    }
    const int32_t k = (int32_t)scal[S_K];
    const int32_t nseg = 2 * k;
    if (nseg <= WALK_TAB) {
        // segment tables in LDS: their reads are tracked apart from the vector
        // loads in flight, so looking up the next chunk never drains the pipeline
        for (int32_t i = threadIdx.x; i <= nseg; i += WALK_BLOCK) { t_off[i] = off[i]; t_coff[i] = coff[i]; }
        __syncthreads();
        walk_body<G, true>(t_off, t_coff, nseg, rows, col, nnz, n, C, list, scal, xcd);
    } else {
        walk_body<G, false>(off, coff, nseg, rows, col, nnz, n, C, list, scal, xcd);
    }
}

template <int G, bool LDS_TAB>
__device__ __forceinline__ void walk_body(const int32_t *O, const int32_t *CO, int32_t nseg,
                                          const int2 *__restrict__ rows, const int32_t *__restrict__ col, int64_t nnz,
                                          int32_t n, int32_t *C, const int32_t *__restrict__ list,
                                          unsigned long long *scal, int32_t xcd) {
    constexpr int U = 32 / G > 4 ? 32 / G : 4;
    const int lane = __lane_id();
    const int wpb = WALK_BLOCK / 64;
    const int wib = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int xl = (xcd && (gridDim.x & 7) == 0) ? 3 : 0;  // log2 of the number of parts
    const uint32_t x = xl ? (blockIdx.x & 7) : 0;
    const uint32_t Wx = (gridDim.x >> xl) * wpb;  // wavefronts sharing one part
    const uint32_t me = (blockIdx.x >> xl) * wpb + wib;
    // cursor over this wavefront's chunks: segment seg, chunk c in [.., hi)
    int32_t seg = -1;
    uint32_t c = 0, hi = 0;
    bool first = true;
    auto advance = [&]() {
        if (!first) c += Wx;
        first = false;
        while (c >= hi) {
            if (++seg >= nseg) return;
            const uint32_t s0 = (uint32_t)CO[seg], len = (uint32_t)CO[seg + 1] - s0;
            const uint32_t lo = s0 + (uint32_t)(((uint64_t)len * x) >> xl);
            hi = s0 + (uint32_t)(((uint64_t)len * (x + 1)) >> xl);
            c = lo + (me + Wx - s0 % Wx) % Wx;  // rotate so that short segments do not all land on the first wavefronts
        }
    };
    // stage A: vertex and row of the chunk under the cursor, then advance
    auto load_chunk = [&](WalkChunk &t) {
        t.seg = seg;
        t.v = -1;
        t.e0 = t.e1 = 0;
        if (seg >= nseg) return;
        const int32_t lo = O[seg], hi2 = O[seg + 1];
        const int32_t j = (int32_t)(c - (uint32_t)CO[seg]);
        const int32_t pos = (seg & 1) ? lo + j : lo + j * (64 / G) + (lane / G);
        const bool ok = pos < hi2;
        const int32_t p = ok ? pos : lo;  // lo < hi2: the segment is not empty
        const int32_t vv = list[p];
        const int2 r = rows[p];
        if (ok) { t.v = vv; t.e0 = r.x; t.e1 = r.y; }
        advance();
    };
    // stage B: the first U neighbor ids of the chunk (unconditional loads at clamped indices)
    auto load_ids = [&](const WalkChunk &t, int32_t *w) {
        const int gsz = (t.seg & 1) ? 64 : G;
        const int32_t e = t.e0 + (lane & (gsz - 1));
#pragma unroll
        for (int u = 0; u < U; u++) {
            const int32_t eu = e + u * gsz;
            const bool ok = eu < t.e1;
            const int32_t wl = col[ok ? eu : 0];  // col has >= 1 entry (a stand-in when nnz = 0)
            w[u] = ok ? wl : -1;
        }
    };
    // neighbor color as First Fit needs it: final colors of lower ranks, 0 otherwise
    auto color_of = [&](int32_t w, int32_t x0, int32_t s) -> int32_t {
        if (x0 >= 0) return x0;
        return (-x0 - 1 < s) ? wait_positive(&C[w], scal) : 0;
    };
    // Gathered words -> First Fit mask bits of colors 1..64.  Words of lower
    // ranks that are not final yet are waited for in one wavefront-uniform
    // slow path; otherwise the update is branch-free (values <= 0 wrap past 64).
    auto absorb = [&](const int32_t *w, int32_t *xv, int32_t s, uint64_t &mask) {
        bool need = false;
#pragma unroll
        for (int u = 0; u < U; u++) need |= xv[u] < 0 && -xv[u] - 1 < s;
        if (__ballot(need)) {
#pragma unroll
            for (int u = 0; u < U; u++) xv[u] = color_of(w[u], xv[u], s);
        }
#pragma unroll
        for (int u = 0; u < U; u++) {
            const uint32_t d = (uint32_t)xv[u] - 1u;
            mask |= (d < 64u ? 1ull : 0ull) << (d & 63u);
        }
    };
    // stage C: gather, wait for lower ranks, First Fit, publish
    auto finish = [&](const WalkChunk &t, const int32_t *w) {
        const int gsz = (t.seg & 1) ? 64 : G;
        const int32_t s = t.seg >> 1;
        const int l = lane & (gsz - 1);
        int32_t xv[U];
#pragma unroll
        for (int u = 0; u < U; u++) {
            const bool ok = (uint32_t)w[u] < (uint32_t)n;
            const int32_t xl = C[ok ? w[u] : 0];
            xv[u] = ok ? xl : 0;
        }
        uint64_t mask = 0;
        absorb(w, xv, s, mask);
        // rows longer than one batch
        for (int32_t eb = t.e0 + l + U * gsz; __ballot(eb < t.e1); eb += U * gsz) {
            int32_t ww[U], xx[U];
#pragma unroll
            for (int u = 0; u < U; u++) {
                const int32_t eu = eb + u * gsz;
                const bool ok = eu < t.e1;
                const int32_t wl = col[ok ? eu : t.e0];
                ww[u] = ok ? wl : -1;
            }
#pragma unroll
            for (int u = 0; u < U; u++) {
                const bool ok = (uint32_t)ww[u] < (uint32_t)n;
                const int32_t xl = C[ok ? ww[u] : 0];
                xx[u] = ok ? xl : 0;
            }
            absorb(ww, xx, s, mask);
        }
        for (int o = gsz >> 1; o > 0; o >>= 1) mask |= __shfl_xor(mask, o);
        int32_t ans;
        if (mask != ~0ull) {
            ans = (int32_t)__ffsll((long long)~mask);
        } else {
            // colors 1..64 all taken: look further, 64 colors per scan (every
            // lower-rank neighbor is final by now; a stale read just waits again)
            uint32_t base = 64;
            for (;;) {
                uint64_t m2 = 0;
                for (int32_t e = t.e0 + l; e < t.e1; e += gsz) {
                    const int32_t w2 = col[e];
                    if ((uint32_t)w2 >= (uint32_t)n) continue;
                    const uint32_t d = (uint32_t)color_of(w2, C[w2], s) - base - 1u;
                    if (d < 64u) m2 |= 1ull << d;
                }
                for (int o = gsz >> 1; o > 0; o >>= 1) m2 |= __shfl_xor(m2, o);
                if (m2 != ~0ull) {
                    ans = (int32_t)(base + (uint32_t)__ffsll((long long)~m2));
                    break;
                }
                base += 64;
            }
        }
        if (t.v >= 0 && l == 0) __hip_atomic_store(&C[t.v], ans, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    };

    advance();
    WalkChunk cur, nxt, nxt2;
    int32_t wcur[U], wnxt[U];
    load_chunk(cur);
    load_ids(cur, wcur);
    load_chunk(nxt);
    while (cur.seg < nseg) {
        load_chunk(nxt2);                          // A: chunk i+2
        if (nxt.seg < nseg) load_ids(nxt, wnxt);   // B: chunk i+1
        finish(cur, wcur);                         // C: chunk i
        cur = nxt;
        nxt = nxt2;
#pragma unroll
        for (int u = 0; u < U; u++) wcur[u] = wnxt[u];
    }
}

// One launch per class (host loop): every vertex of rank s, one lane each.
__global__ void k_walk_class(const int32_t *__restrict__ rp, const int32_t *__restrict__ col, int64_t nnz, int32_t n,
                             int32_t *C, const int32_t *__restrict__ list, const int32_t *__restrict__ off, int32_t s) {
    const int32_t a = off[2 * s], b = off[2 * s + 2];
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = a + (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < b; i += stride) {
        int32_t v = list[i];
        int32_t e0, e1;
        row_range(rp, v, nnz, e0, e1);
        C[v] = select_color_lane(col, e0, e1, C, n, 0u);
    }
}

typedef void (*walk_fn)(const int2 *, const int32_t *, int64_t, int32_t, int32_t *, const int32_t *, const int32_t *,
                        const int32_t *, unsigned long long *, int32_t, int32_t);

static walk_fn walk_kernel(int G) {
    switch (G) {
        case 1: return k_walk_flow<1>;
        case 2: return k_walk_flow<2>;
        case 4: return k_walk_flow<4>;
        case 8: return k_walk_flow<8>;
        case 16: return k_walk_flow<16>;
        case 32: return k_walk_flow<32>;
        default: return k_walk_flow<64>;
    }
}

static gc_status launch_walk_flow(gc_ctx *ctx, const gc_csr *g, int32_t *C, hipStream_t s) {
    const int G = ctx->tune.group;
    walk_fn f = walk_kernel(G);
    if (ctx->walk_blocks == 0 || ctx->walk_blocks_group != G) {
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
            hipLaunchKernelGGL(f, dim3(blocks), dim3(WALK_BLOCK), 0, s, ctx->rows, (const int32_t *)ctx->scal, g->nnz, g->n, C, ctx->list,
                               ctx->off, ctx->coff, ctx->scal, 0, 2);
            GC_LAUNCHED();
            gc_status st = gc_sync_scalars(ctx, s);
            if (st) return st;
            if (!(ctx->hscal[S_ERR] & 4)) break;
        }
        if (per_cu < 1) return gc_fail(ctx, GC_ERR_DEVICE, "walk kernel: no grid was fully resident");
        GC_HIP(hipMemsetAsync(ctx->scal + S_ERR, 0, 8, s));
        ctx->walk_blocks = blocks;
        ctx->walk_blocks_group = G;
    }
    // An ordinary stream-ordered launch whose grid is exactly what the device
    // holds at once: the kernel starts after the previous kernel of the stream
    // has finished, so every workgroup is dispatched at once on an otherwise idle
    // device (kernels of other streams can only delay some workgroups until they
    // finish; the bounded waits keep even that case from hanging).
    const int32_t xcd = ctx->tune.xcd_chunks > 0 ? 1 : 0;
    if (ctx->tune.check_resident) GC_HIP(hipMemsetAsync(ctx->scal + S_TICKET, 0, 8, s));
    // the walk reads col[0] unconditionally (masked afterwards): give it one valid word when the graph has no edges
    const int32_t *col = g->nnz > 0 ? g->col_idx : (const int32_t *)ctx->scal;
    GC_TIMED(GC_K_WALK, s, hipLaunchKernelGGL(f, dim3(ctx->walk_blocks), dim3(WALK_BLOCK), 0, s, ctx->rows, col,
                                              g->nnz, g->n, C, ctx->list, ctx->off, ctx->coff, ctx->scal, xcd,
                                              ctx->tune.check_resident));
    GC_LAUNCHED();
    return GC_OK;
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
    const int G = ctx->tune.group;
    const int32_t deg_wave = ctx->tune.deg_wave;
    const int hist_grid = gc_grid(ctx, n, block) < 2 * ctx->num_cu ? gc_grid(ctx, n, block) : 2 * ctx->num_cu;
    GC_HIP(hipMemsetAsync(ctx->scal + S_MAXC, 0, 8, s));
    GC_HIP(hipMemsetAsync(ctx->scal + S_ERR, 0, 8, s));
    GC_TIMED(GC_K_HIST, s, k_hist<<<hist_grid, block, 0, s>>>(n, colors_in, g->row_ptr, g->nnz, deg_wave, ctx->ccap, ctx->hist,
                                                     ctx->histw, ctx->scal));
    GC_LAUNCHED();
    GC_TIMED(GC_K_ORDER, s, k_class_order<<<1, PERM_THREADS, 0, s>>>(ctx->ccap, perm, gc_stream_value(seed, GC_TAG_PERM, (uint32_t)pass), 64 / G,
                                            ctx->hist, ctx->histw, (int32_t *)ctx->keys, ctx->pi, ctx->rank, ctx->off,
                                            ctx->coff, ctx->cursor, ctx->scal));
    GC_LAUNCHED();
    int64_t tiles = ((int64_t)n + block * SCATTER_ITEMS - 1) / (block * SCATTER_ITEMS);
    GC_TIMED(GC_K_SCATTER, s, k_scatter<<<(unsigned)tiles, block, 0, s>>>(n, colors_in, colors_out, g->row_ptr, g->nnz, deg_wave, ctx->ccap,
                                                ctx->rank, ctx->cursor, ctx->list, ctx->rows, ctx->scal));
    GC_LAUNCHED();
    if (ctx->tune.walk_mode == 0) {
        status = launch_walk_flow(ctx, g, colors_out, s);
        if (status) return status;
    } else {
        status = gc_sync_scalars(ctx, s);
        if (status) return status;
        if (ctx->hscal[S_ERR] & 1) return gc_fail(ctx, GC_ERR_COLORING, "input color outside [1, %d]", ctx->ccap);
        const int32_t k = (int32_t)ctx->hscal[S_K];
        for (int32_t r = 0; r < k; r++) {
            GC_TIMED(GC_K_WALK, s, k_walk_class<<<gc_grid(ctx, n, block), block, 0, s>>>(g->row_ptr, g->col_idx, g->nnz, n, colors_out, ctx->list,
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
        if (ctx->hscal[S_ERR] & 4) return gc_fail(ctx, GC_ERR_DEVICE, "class walk: workgroups were not all resident (grid %d)", ctx->walk_blocks);
        if (ctx->hscal[S_ERR] & 2) return gc_fail(ctx, GC_ERR_DEVICE, "class walk: a dependency wait ran out");
        st->rounds = 0;
        st->losers_total = 0;
        st->k_classes = (int32_t)ctx->hscal[S_K];
        st->num_colors = (int32_t)ctx->hscal[S_NUMC];
        st->max_color = (int32_t)ctx->hscal[S_MAXC];
    }
    return GC_OK;
}
