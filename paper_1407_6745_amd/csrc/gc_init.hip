// gc_init.hip - speculative round-synchronous initial coloring
// (section 2.2 framework, one superstep per round over every uncolored
// vertex; First Fit of section 2.1 or Random-X Fit of section 3.2).
//
// In-place encoding of the colors array C during the rounds:
//   C[v] > 0   committed color (final);
//   C[v] < 0   v is in the current round's set W_r with tentative color -C[v]
//              (or lost the previous round and waits for a new one).
// Readers of the assign step treat every value <= 0 as "no color", which is
// exactly the start-of-round snapshot: a value only becomes positive in the
// detect step.  The detect step compares |C[w]| with v's tentative color: a
// neighbor w with |C[w]| = T_v is necessarily in W_r (T_v avoids every color
// committed before the round), whether w has already flipped its own sign to
// commit or not.  Losers keep -T until the next assign overwrites it, so every
// detect read of the round sees every tentative color.
//
// Work layout: every vertex is handled by a group of G lanes (rows up to
// deg_wave long) or by a whole wavefront (longer rows).  Each round keeps two
// worklists (group bin, wavefront bin); losers are appended through LDS queues
// (one global atomic per flush).
#include "gc_internal.h"

#include <climits>
#include <cstdint>
#include <vector>

#define INIT_BLOCK 256
#define GC_RUN_AHEAD 8       // rounds queued per host read-back,
#define GC_RUN_AHEAD_MAX 32  // growing to r / 4 (at most this many) once the rounds run long
static_assert(S_REC + 2 * GC_RUN_AHEAD_MAX <= S_COUNT, "round records");
// loads in flight per lane: whole-wavefront rows are long, so they keep more
#define ROW_UNROLL(G) ((G) >= 32 ? 8 : GC_UNROLL)
// The round-0 and assign scans keep eight in flight at every group size: a
// 27-point mesh row (26 entries on 4 lanes) then takes one batch of loads
// (mesh initial coloring 0.89 -> 0.85 ms); the detect scan stays at
// ROW_UNROLL, where eight cost more than they save (detect 0.39 -> 0.48 ms).
#define SELECT_UNROLL 8

// Tentative color of w in round 0: 1 + its Random-X offset (no color is held yet).
__device__ inline int32_t round0_color(uint32_t s_color, int32_t w, uint32_t X, bool randx) {
    return randx ? (int32_t)gc_pick(s_color, w, X) + 1 : 1;
}

// Does v (tentative color tv, priority pv) lose against a neighbor?  Group of
// G lanes, result uniform over the group.  ROUND0: neighbor colors come from
// the hash; otherwise |C[w]|.
template <int G, bool ROUND0, int UNR = GC_UNROLL, typename CA = const int32_t *>
__device__ inline bool group_loses(int32_t tv, uint64_t pv, int32_t e0, int32_t e1, const int32_t *__restrict__ col,
                                   CA C, int32_t n, const Prio &pr, uint32_t s_color, uint32_t X,
                                   bool randx) {
    const int l = __lane_id() & (G - 1);
    bool lose = false;
    for (int32_t eb = e0 + l; eb < e1; eb += G * UNR) {
        int32_t w[UNR], t[UNR];
#pragma unroll
        for (int u = 0; u < UNR; u++) {
            const int32_t e = eb + u * G;
            const int32_t wl = col[e < e1 ? e : eb];
            w[u] = e < e1 ? wl : -1;
        }
#pragma unroll
        for (int u = 0; u < UNR; u++) {
            const bool ok = (uint32_t)w[u] < (uint32_t)n;
            if (ROUND0) {
                t[u] = ok ? round0_color(s_color, w[u], X, randx) : 0;
            } else {
                const int32_t cl = (int32_t)C[ok ? w[u] : 0];
                t[u] = ok ? abs(cl) : 0;
            }
        }
#pragma unroll
        for (int u = 0; u < UNR; u++)
            if (t[u] == tv && round_prio(pr, w[u]) > pv) lose = true;
        // one conflict decides: the group reads no more of a loser's row (the
        // ballot sees only the lanes with entries left, which can only delay
        // the exit; a row that fits one batch skips it)
        if (eb + G * UNR < e1 && group_any<G>(lose)) break;
    }
    return group_any<G>(lose);
}

// One wavefront over src[e0, e1): does v (tentative color tv, priority pv)
// lose to a neighbor, and (out != NULL) which entries are still uncolored.
// Every batch of UNR x 64 entries issues all its id loads, then all its color
// loads, and appends its kept entries in order at out[*] with one
// reservation per batch: *cursor (wavefront-private, len == NULL) or an
// atomic add on *len (several wavefronts append to one list).  EARLY stops
// at the first batch that finds a conflict (no kept entries then).
template <int UNR, bool EARLY, typename CA = const int32_t *>
__device__ inline bool wave_loses_keep(int32_t tv, uint64_t pv, int32_t e0, int32_t e1, const int32_t *__restrict__ src,
                                       CA C, int32_t n, const Prio &pr, int32_t *out, int32_t *cursor,
                                       int32_t *len) {
    const int lane = __lane_id();
    bool lose = false;
    for (int32_t eb = e0; eb < e1; eb += 64 * UNR) {
        int32_t w[UNR], c[UNR];
#pragma unroll
        for (int u = 0; u < UNR; u++) {
            const int32_t e = eb + u * 64 + lane;
            const int32_t wl = src[e < e1 ? e : eb];
            w[u] = e < e1 ? wl : -1;
        }
#pragma unroll
        for (int u = 0; u < UNR; u++) {
            const bool ok = (uint32_t)w[u] < (uint32_t)n;
            const int32_t cl = (int32_t)C[ok ? w[u] : 0];
            c[u] = ok ? cl : INT32_MAX;  // an invalid id: neither a conflict nor kept
        }
#pragma unroll
        for (int u = 0; u < UNR; u++)
            if (c[u] != INT32_MAX && abs(c[u]) == tv && round_prio(pr, w[u]) > pv) lose = true;
        if (out) {
            unsigned long long bm[UNR];
            int32_t tot = 0;
#pragma unroll
            for (int u = 0; u < UNR; u++) {
                bm[u] = __ballot(c[u] <= 0);
                tot += (int32_t)__popcll(bm[u]);
            }
            if (tot) {
                int32_t base = 0;
                if (len) {
                    if (lane == 0) base = atomicAdd(len, tot);
                    base = __shfl(base, 0);
                } else {
                    base = *cursor;
                    *cursor += tot;
                }
#pragma unroll
                for (int u = 0; u < UNR; u++) {
                    if (c[u] <= 0) out[base + __popcll(bm[u] & ((1ull << lane) - 1ull))] = w[u];
                    base += (int32_t)__popcll(bm[u]);
                }
            }
        }
        if (EARLY && __ballot(lose)) return true;
    }
    return __ballot(lose) != 0ull;
}

// Committed-color masks of the long rows (more than deg_wave entries): for a
// long row x, fm[longidx[x]] holds which of the colors 1 .. FM_COLORS its
// neighbors have committed so far.  Every vertex that commits ORs its color
// into the masks of its long neighbors, so the assign step of a long row
// reads FM_WORDS words instead of its row (the row is scanned only for colors
// above FM_COLORS).  The masks are off (idx == NULL) for graphs without long
// rows.
#define FM_WORDS 8
#define FM_COLORS (64 * FM_WORDS)

struct LongMasks {
    const int32_t *idx;
    unsigned long long *fm;
};

// Called by the G lanes of the group that committed color c for a row col[e0, e1).
template <int G>
__device__ inline void publish_long(const LongMasks &lm, const int32_t *__restrict__ col, int32_t e0, int32_t e1,
                                   int32_t n, int32_t c) {
    if (!lm.idx || c < 1 || c > FM_COLORS) return;
    const unsigned long long bit = 1ull << ((c - 1) & 63);
    const int w = (c - 1) >> 6;
    constexpr int PU = G >= 32 ? 4 : 1;  // a wavefront's row: four neighbor ids per lane in flight
    for (int32_t e = e0 + (int32_t)(__lane_id() & (G - 1)); e < e1; e += G * PU) {
        int32_t x[PU], li[PU];
#pragma unroll
        for (int u = 0; u < PU; u++) x[u] = e + u * G < e1 ? col[e + u * G] : -1;
#pragma unroll
        for (int u = 0; u < PU; u++) li[u] = (uint32_t)x[u] < (uint32_t)n ? lm.idx[x[u]] : -1;
#pragma unroll
        for (int u = 0; u < PU; u++)
            if (li[u] >= 0) atomicOr(&lm.fm[(size_t)li[u] * FM_WORDS + w], bit);
    }
}

// (j+1)-th smallest color free in a long row's mask, else past FM_COLORS by a
// scan of the row (a wavefront per row).
template <bool COH = false, typename CA = const int32_t *>
__device__ inline int32_t fm_select(const unsigned long long *__restrict__ m, uint32_t j,
                                    const int32_t *__restrict__ col, int32_t e0, int32_t e1, CA C,
                                    int32_t n) {
    const int lane = __lane_id();
    uint64_t word = ~0ull;
    if (lane < FM_WORDS)
        word = COH ? __hip_atomic_load(&m[lane], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) : m[lane];
    const uint32_t t = wave_nth_free(word, j);
    if (t) return (int32_t)t;
    const uint32_t freec = (uint32_t)wave_sum_u64((unsigned long long)__popcll(~word));
    return group_select<64>(col, e0, e1, C, n, j - freec, FM_COLORS);
}

// Active lists of the split rows (rows handled in chunks): from the second
// round on, a split row's detect step reads only the neighbors that were
// still uncolored when the row was last scanned.  Each detect step of a
// split row also writes the entries it finds uncolored into the other buffer
// (same offsets as col, order free), for the next round.  len[li] < 0: the
// row has no list yet (read col).  Committed neighbors leave the lists, so a
// row that stays uncolored for many rounds (the dense core of a skewed graph)
// scans fewer and fewer entries; the assign step never needs them (masks).
struct ActiveLists {
    const int32_t *idx;  // longidx (NULL: lists off)
    const int32_t *cur;  // this round's lists
    const int32_t *len;  // their lengths by long-row index
    int32_t *next;       // next round's lists (written by the detect step)
    int32_t *len_next;
};

// LDS state of a kernel that appends to two worklists.
struct InitQueues {
    int32_t buf[2][GC_QCAP];
    int32_t cnt[2];
    int32_t base[2];
};

__device__ inline void queues_init(InitQueues &q) {
    if (threadIdx.x == 0) { q.cnt[0] = 0; q.cnt[1] = 0; }
    __syncthreads();
}

__device__ inline void queues_flush(InitQueues &q, int32_t *wl_lo, unsigned long long *c_lo, int32_t *wl_hub,
                                    unsigned long long *c_hub, bool force) {
    __syncthreads();
    bq_flush(q.buf[0], &q.cnt[0], &q.base[0], wl_lo, c_lo, force);
    bq_flush(q.buf[1], &q.cnt[1], &q.base[1], wl_hub, c_hub, force);
}

// Round 0, by vertex id (in_list == NULL) or over a list of long rows.  By
// vertex id, rows longer than deg_wave are not processed but appended to the
// second queue (they get their own launch, one wavefront each); over a list,
// rows longer than skip_len are left to the split kernels.  Writes
// C[v] = +T (kept) or -T (lost) and appends losers by bin.
// Compact copy of the colors for the neighbor reads of the rounds, written
// beside C at every change.  CT = int8_t when every color the coloring can
// take fits (the longest row plus X is at most 127); CT = int16_t otherwise,
// saturated at +-C16_SAT (a saturated word sends the reader to C, which
// stays exact); CT = int32_t: no copy, C itself.  Half or a quarter of the
// bytes keep more of the colors in the L2 for graphs whose neighbors lie far
// apart in the vertex order.
// The two-byte copy saturates at +-sat (the compact_sat knob, 32767 by
// default; tests lower it to reach the saturated path on small graphs).
template <typename CT>
struct CompactCopy {
    CT *p;
    int32_t sat;
    __device__ void put(int32_t v, int32_t x) const {
        if (sizeof(CT) == 1) p[v] = (CT)x;
        if (sizeof(CT) == 2) p[v] = (CT)(x > sat ? sat : (x < -sat ? -sat : x));
    }
};

// The copy as the split-row kernels (not instantiated per copy width) see it:
// bytes = 0 (no copy), 1 or 2.
struct CopyRef {
    void *p;
    int32_t bytes, sat;
    __device__ void put(int32_t v, int32_t x) const {
        if (bytes == 1) ((int8_t *)p)[v] = (int8_t)x;
        else if (bytes == 2) ((int16_t *)p)[v] = (int16_t)(x > sat ? sat : (x < -sat ? -sat : x));
    }
};
template <typename CT>
inline CopyRef copy_ref(const CompactCopy<CT> &S) {
    return CopyRef{(void *)S.p, sizeof(CT) < 4 ? (int32_t)sizeof(CT) : 0, S.sat};
}

// Optional per-vertex output: the round in which a vertex's color became final.
struct RoundOut {
    int32_t *p;  // NULL: off
    int32_t r;
    __device__ void put(int32_t v) const {
        if (p) p[v] = r;
    }
};

struct Sat16 {
    const int16_t *s;
    const int32_t *c;
    int32_t sat;
    __device__ int32_t operator[](int64_t i) const {
        const int32_t x = s[i];
        return (x == sat || x == -sat) ? c[i] : x;
    }
};

// The neighbor-color reader of a kernel instantiated for CT.
template <typename CT>
struct CompactRead {
    using R = const CT *;
    __device__ static R of(const CompactCopy<CT> &S, const int32_t *C) {
        return sizeof(CT) < 4 ? S.p : (const CT *)C;
    }
};
template <>
struct CompactRead<int16_t> {
    using R = Sat16;
    __device__ static R of(const CompactCopy<int16_t> &S, const int32_t *C) { return Sat16{S.p, C, S.sat}; }
};

template <int G, typename CT>
__global__ void __launch_bounds__(INIT_BLOCK) k_round0(const int32_t *__restrict__ rp, const int32_t *__restrict__ col,
                                                       int64_t nnz, int32_t n, int32_t *C, CompactCopy<CT> S, int32_t deg_wave,
                                                       int32_t skip_len, const int32_t *__restrict__ in_list,
                                                       const unsigned long long *__restrict__ in_count,
                                                       int32_t *wl_lo, unsigned long long *c_lo, int32_t *wl_hub,
                                                       unsigned long long *c_hub, Prio pr, uint32_t s_color,
                                                       uint32_t X, int randx, LongMasks lm, RoundOut ro) {
    __shared__ InitQueues q;
    queues_init(q);
    const int64_t cnt = in_list ? (int64_t)*in_count : (int64_t)n;
    const int vpi = INIT_BLOCK / G;  // vertices per block iteration
    const int gi = threadIdx.x / G;
    for (int64_t base = (int64_t)blockIdx.x * vpi; base < cnt; base += (int64_t)gridDim.x * vpi) {
        const int64_t i = base + gi;
        int32_t v = -1, e0 = 0, e1 = 0;
        bool forward = false;
        if (i < cnt) {
            v = in_list ? in_list[i] : (int32_t)i;
            row_range(rp, v, nnz, e0, e1);
            if (!in_list && e1 - e0 > deg_wave) forward = true;
            if (in_list && e1 - e0 > skip_len) { v = -1; e0 = e1 = 0; }  // split rows: their own kernels
        }
        const bool hub = e1 - e0 > deg_wave;
        if (forward) e1 = e0;
        const int32_t tv = v >= 0 ? round0_color(s_color, v, X, randx != 0) : 0;
        const uint64_t pv = v >= 0 ? round_prio(pr, v) : 0u;
        const bool lose = group_loses<G, true, SELECT_UNROLL>(tv, pv, e0, e1, col, C, n, pr, s_color, X, randx != 0);
        const bool leader = (__lane_id() & (G - 1)) == 0 && v >= 0;
        if (leader && !forward) {
            C[v] = lose ? -tv : tv;
            S.put(v, lose ? -tv : tv);
            if (!lose) ro.put(v);
        }
        if (v >= 0 && !forward && !lose) publish_long<G>(lm, col, e0, e1, n, tv);
        bq_push(q.buf[0], &q.cnt[0], leader && !forward && lose && !hub, v);
        bq_push(q.buf[1], &q.cnt[1], leader && (forward || (lose && hub)), v);
        queues_flush(q, wl_lo, c_lo, wl_hub, c_hub, false);
    }
    queues_flush(q, wl_lo, c_lo, wl_hub, c_hub, true);
}

// Assign step of round r >= 1: C[v] = -T for every v of the list.
template <int G, typename CT>
__global__ void __launch_bounds__(INIT_BLOCK) k_assign(const int32_t *__restrict__ rp, const int32_t *__restrict__ col,
                                                       int64_t nnz, int32_t n, int32_t *C, CompactCopy<CT> S,
                                                       const int32_t *__restrict__ wl,
                                                       const unsigned long long *__restrict__ wcount, uint32_t s_color,
                                                       uint32_t X, int randx, unsigned long long *degsum,
                                                       int32_t skip_len, LongMasks lm, unsigned long long *zero2,
                                                       unsigned long long *zero1, unsigned long long *rec,
                                                       const unsigned long long *rec_in) {
    __shared__ unsigned long long sdeg;
    __shared__ unsigned long long lmask[INIT_BLOCK];
    unsigned long long *lw = lmask + (threadIdx.x & ~63u);
    if (threadIdx.x == 0) sdeg = 0;
    // counters the detect step appends to next, and the degree sum of the next
    // round (neither is touched by this launch)
    // (a round queued without a host read first records its input size and
    // the previous round's degree sum, which the last slot still holds)
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        if (rec) {
            rec[0] = rec_in[0] + rec_in[1];
            rec[1] = *zero1;
        }
        zero2[0] = 0;
        zero2[1] = 0;
        *zero1 = 0;
    }
    __syncthreads();
    const int64_t cnt = (int64_t)*wcount;
    const int vpi = INIT_BLOCK / G;
    const int gi = threadIdx.x / G;
    unsigned long long degs = 0;
    for (int64_t base = (int64_t)blockIdx.x * vpi; base < cnt; base += (int64_t)gridDim.x * vpi) {
        const int64_t i = base + gi;
        int32_t v = -1, e0 = 0, e1 = 0;
        if (i < cnt) {
            v = wl[i];
            row_range(rp, v, nnz, e0, e1);
            if (e1 - e0 > skip_len) { v = -1; e0 = e1 = 0; }
        }
        const uint32_t j = (v >= 0 && randx) ? gc_pick(s_color, v, X) : 0u;
        int32_t t;
        const int32_t li = (G == 64 && lm.idx && v >= 0) ? lm.idx[v] : -1;  // one row per wavefront: uniform
        if (li >= 0) t = fm_select(lm.fm + (size_t)li * FM_WORDS, j, col, e0, e1, C, n);
        else t = group_select_wide<G, SELECT_UNROLL>(col, e0, e1, CompactRead<CT>::of(S, C), n,
                                                           j, lw);
        if (v >= 0 && (__lane_id() & (G - 1)) == 0) {
            C[v] = -t;
            S.put(v, -t);
            degs += (unsigned long long)(e1 - e0);
        }
    }
    degs = wave_sum_u64(degs);
    if (__lane_id() == 0 && degs) atomicAdd(&sdeg, degs);
    __syncthreads();
    if (threadIdx.x == 0 && sdeg) atomicAdd(degsum, sdeg);
}

// Detect step of round r >= 1: v loses when a neighbor has the same tentative
// color and a larger priority; winners commit (flip the sign), losers go to
// the next worklist of their bin.
// LISTS (G = 64 with active lists): every row is scanned by wave_loses_keep
// (rows without a list keep nothing), so the kernel holds one scan routine.
template <int G, typename CT, bool RO, bool LISTS>
__global__ void __launch_bounds__(INIT_BLOCK) k_detect(const int32_t *__restrict__ rp, const int32_t *__restrict__ col,
                                                       int64_t nnz, int32_t n, int32_t *C, CompactCopy<CT> S, int32_t deg_wave,
                                                       const int32_t *__restrict__ wl,
                                                       const unsigned long long *__restrict__ wcount, int32_t *wl_lo,
                                                       unsigned long long *c_lo, int32_t *wl_hub,
                                                       unsigned long long *c_hub, Prio pr, int32_t skip_len,
                                                       LongMasks lm, ActiveLists al, RoundOut ro) {
    __shared__ InitQueues q;
    queues_init(q);
    const int64_t cnt = (int64_t)*wcount;
    const int vpi = INIT_BLOCK / G;
    const int gi = threadIdx.x / G;
    int32_t iter = 0;
    for (int64_t base = (int64_t)blockIdx.x * vpi; base < cnt; base += (int64_t)gridDim.x * vpi) {
        const int64_t i = base + gi;
        int32_t v = -1, e0 = 0, e1 = 0, t = 0, full = 0, li = -1;
        bool act = false;
        if (i < cnt) {
            v = wl[i];
            row_range(rp, v, nnz, e0, e1);
            full = e1 - e0;
            if (G == 64 && al.idx) {  // a long row reads its active list when it has one
                li = al.idx[v];
                if (li >= 0 && al.len[li] >= 0) {
                    act = true;
                    e1 = e0 + min(al.len[li], full);
                }
            }
            if (e1 - e0 > skip_len) { v = -1; e0 = e1 = 0; }  // long enough for the split kernels
            else t = -C[v];
        }
        const int32_t *src = act ? al.cur : col;
        const uint64_t pv = v >= 0 ? round_prio(pr, v) : 0u;
        bool lose;
        if (LISTS) {
            // one scan decides the conflict and keeps the entries still uncolored:
            // the row's list for the next round (one wavefront, in order)
            const bool keep = v >= 0 && li >= 0;
            int32_t kept = 0;
            lose = wave_loses_keep<ROW_UNROLL(64), false>(t, pv, e0, e1, src, CompactRead<CT>::of(S, C), n, pr,
                                                          keep ? al.next + e0 : nullptr, &kept, nullptr);
            if (keep && __lane_id() == 0) al.len_next[li] = kept;
        } else {
            lose = group_loses<G, false, ROW_UNROLL(G)>(t, pv, e0, e1, src, CompactRead<CT>::of(S, C), n, pr, 0u,
                                                           1u, false);
        }
        const bool leader = (__lane_id() & (G - 1)) == 0 && v >= 0;
        if (leader && !lose) {
            C[v] = t;
            S.put(v, t);
            // (a compile-time switch: the run-time test alone slowed this
            // kernel by a quarter on the mesh)
            if (RO) ro.put(v);
        }
        if (v >= 0 && !lose) publish_long<G>(lm, src, e0, e1, n, t);
        const bool hub = full > deg_wave;  // worklist bins by the full row length
        bq_push(q.buf[0], &q.cnt[0], leader && lose && !hub, v);
        bq_push(q.buf[1], &q.cnt[1], leader && lose && hub, v);
        // wavefront rows push at most four entries an iteration: they check
        // the queues (a block barrier) every 64 iterations only, which still
        // flushes before the buffer can overflow (the trip count is uniform
        // across the block)
        if (G < 64 || ++iter % 64 == 0) queues_flush(q, wl_lo, c_lo, wl_hub, c_hub, false);
    }
    queues_flush(q, wl_lo, c_lo, wl_hub, c_hub, true);
}

// ---------------------------------------------------------------------------
// long rows (longer than deg_wave and deg_split): split_len-entry chunks,
// one wavefront each, several wavefronts per row.  A per-round plan lists
// the long rows of a worklist (hub slot = position in the plan) and the first
// chunk of each.  Partial results meet in the row's hub slot (mask words for
// the assign step, a lose flag for the detect step); the chunk that finishes
// last completes the row and clears the slot.
// ---------------------------------------------------------------------------

// The plan of a round's split rows: slot i holds row hub_v[i], whose chunks
// start at hub_first[i] (increasing with i).  Any number of workgroups: each
// wavefront reserves its rows' slots and chunks with one 64-bit atomic on the
// packed total (rows << 32 | chunks), so slots and first chunks grow in the
// same order.  `next` (the other round's total) is cleared for the next round.
__device__ inline int32_t plan_rows(const unsigned long long *plan) { return (int32_t)(*plan >> 32); }
__device__ inline int32_t plan_chunks(const unsigned long long *plan) { return (int32_t)(*plan & 0xFFFFFFFFull); }

__global__ void __launch_bounds__(256) k_split_plan(const int32_t *__restrict__ rp, int64_t nnz,
                                                    const int32_t *__restrict__ in_list,
                                                    const unsigned long long *__restrict__ in_count, int32_t thresh,
                                                    int32_t split_len, int32_t *__restrict__ hub_v,
                                                    int32_t *__restrict__ hub_first, unsigned long long *plan,
                                                    unsigned long long *next, ActiveLists al) {
    if (blockIdx.x == 0 && threadIdx.x == 0) *next = 0;
    const int64_t cnt = (int64_t)*in_count;
    const int lane = __lane_id();
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t base = (int64_t)blockIdx.x * blockDim.x + (threadIdx.x & ~63u); base < cnt; base += stride) {
        const int64_t i = base + lane;
        int32_t v = -1, len = 0;
        if (i < cnt) {
            v = in_list[i];
            int32_t e0, e1;
            row_range(rp, v, nnz, e0, e1);
            len = e1 - e0;
        }
        // the entries the row's chunks would cover this round: its active list when it has one
        int32_t clen = len, li = -1;
        if (v >= 0 && al.idx) {
            li = al.idx[v];
            if (li >= 0 && al.len[li] >= 0) clen = min(al.len[li], len);
        }
        const bool lg = v >= 0 && clen > thresh;  // longer rows take the split kernels, the others k_detect
        if (lg && li >= 0 && al.len_next) al.len_next[li] = 0;
        const uint32_t nsub = lg ? (clen > 0 ? (uint32_t)((clen + split_len - 1) / split_len) : 1u) : 0u;
        const unsigned long long bm = __ballot(lg);
        if (!bm) continue;
        uint32_t inc = nsub;  // inclusive scan of the chunk counts over the wavefront
        for (int o = 1; o < 64; o <<= 1) {
            const uint32_t y = __shfl_up(inc, o);
            if (lane >= o) inc += y;
        }
        const uint32_t tot = __shfl(inc, 63);
        unsigned long long old = 0;
        if (lane == 0) old = atomicAdd(plan, ((unsigned long long)__popcll(bm) << 32) | tot);
        old = __shfl(old, 0);
        if (lg) {
            const uint32_t slot = (uint32_t)(old >> 32) + (uint32_t)__popcll(bm & ((1ull << lane) - 1ull));
            hub_v[slot] = v;
            hub_first[slot] = (int32_t)((uint32_t)(old & 0xFFFFFFFFull) + inc - nsub);
        }
    }
}

// Chunk c of the plan: its row's slot, vertex, row range and chunk range.

// Chunk c of the plan: its row's slot, vertex, the entries [e0, e1) the row's
// chunks cover this round (its active list when it has one: act = true, read
// from the lists' buffer at the same offsets), the chunk's [a, b), and the
// row's chunk count.
struct SplitChunk {
    int32_t slot, v, e0, e1, a, b, nsub, li;
    bool act;
};

__device__ inline SplitChunk split_chunk(int32_t c, int32_t nrow, int32_t nch, const int32_t *__restrict__ hub_v,
                                         const int32_t *__restrict__ hub_first, const int32_t *__restrict__ rp,
                                         int64_t nnz, int32_t split_len, const ActiveLists &al) {
    int32_t lo = 0, hi = nrow - 1;  // last slot whose first chunk is <= c
    while (lo < hi) {
        const int32_t mid = (lo + hi + 1) >> 1;
        if (hub_first[mid] <= c) lo = mid;
        else hi = mid - 1;
    }
    SplitChunk k;
    k.slot = lo;
    k.v = hub_v[lo];
    row_range(rp, k.v, nnz, k.e0, k.e1);
    k.li = al.idx ? al.idx[k.v] : -1;
    k.act = k.li >= 0 && al.len[k.li] >= 0;
    if (k.act) k.e1 = k.e0 + min(al.len[k.li], k.e1 - k.e0);
    k.nsub = (lo + 1 < nrow ? hub_first[lo + 1] : nch) - hub_first[lo];
    k.a = k.e0 + (c - hub_first[lo]) * split_len;
    k.b = min(k.e1, k.a + split_len);
    return k;
}

// Counts a finished chunk of slot; true (wavefront-uniform) for the last one.
// What the chunks exchange through the slot is written and read with device
// atomics only, so no cache maintenance is needed: the wavefront waits until
// its own atomics on the slot are done before counting itself, and the last
// chunk reads the slot after its count came back.
__device__ inline bool split_last(int32_t *hub_cnt, int32_t slot, int32_t nsub) {
    __builtin_amdgcn_s_waitcnt(0);
    int32_t done = 0;
    if (__lane_id() == 0) done = atomicAdd(&hub_cnt[slot], 1) + 1;
    done = __shfl(done, 0);
    return done == nsub;
}

// Assign step for long rows (rounds >= 1): committed neighbor colors 1..64
// in a register word, 65 .. 64 * hub_words in the wavefront's LDS words,
// merged into the row's hub words; the last chunk takes the (j+1)-th free
// color (past color 64 * hub_words it rescans the row).
__global__ void __launch_bounds__(INIT_BLOCK) k_split_assign(const int32_t *__restrict__ rp,
                                                             const int32_t *__restrict__ col, int64_t nnz, int32_t n,
                                                             int32_t *C, const int32_t *__restrict__ hub_v,
                                                             const int32_t *__restrict__ hub_first,
                                                             const unsigned long long *__restrict__ plan,
                                                             int32_t split_len, int32_t hub_words, uint32_t s_color,
                                                             uint32_t X, int randx, unsigned long long *hub_bits,
                                                             int32_t *hub_cnt, unsigned long long *degsum, CopyRef cr) {
    __shared__ unsigned long long lmask[INIT_BLOCK];
    const ActiveLists al{nullptr, nullptr, nullptr, nullptr, nullptr};  // whole rows (no masks on this path)
    const int lane = __lane_id();
    unsigned long long *lw = lmask + (threadIdx.x & ~63u);
    const int32_t nrow = plan_rows(plan), nch = plan_chunks(plan);
    const int wpb = INIT_BLOCK / 64;
    const int wib = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    for (int32_t c = blockIdx.x * wpb + wib; c < nch; c += gridDim.x * wpb) {
        const SplitChunk k = split_chunk(c, nrow, nch, hub_v, hub_first, rp, nnz, split_len, al);
        unsigned long long *bits = hub_bits + (int64_t)k.slot * GC_HUB_WORDS;
        lw[lane] = 0ull;
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        uint64_t m = 0;
        for (int32_t eb = k.a + lane; __ballot(eb < k.b); eb += 64 * ROW_UNROLL(64)) {
            int32_t w[ROW_UNROLL(64)], x[ROW_UNROLL(64)];
#pragma unroll
            for (int u = 0; u < ROW_UNROLL(64); u++) {
                const int32_t e = eb + u * 64;
                const int32_t wl = col[e < k.b ? e : k.a];
                w[u] = e < k.b ? wl : -1;
            }
#pragma unroll
            for (int u = 0; u < ROW_UNROLL(64); u++) {
                const bool ok = (uint32_t)w[u] < (uint32_t)n;
                const int32_t cl = C[ok ? w[u] : 0];
                x[u] = ok ? cl : 0;
            }
#pragma unroll
            for (int u = 0; u < ROW_UNROLL(64); u++) mask_mark<true>(x[u], 0u, m, lw, 0, hub_words - 1);
        }
        m = group_or_rt(m, 64);
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        const uint64_t lword = lane >= 1 ? lw[lane - 1] : 0ull;
        const uint64_t mine = lane == 0 ? m : lword;
        if (lane < hub_words && mine) atomicOr(&bits[lane], mine);
        if (split_last(hub_cnt, k.slot, k.nsub)) {
            const uint64_t word = lane < hub_words ? atomicOr(&bits[lane], 0ull) : ~0ull;
            const uint32_t j = randx ? gc_pick(s_color, k.v, X) : 0u;
            uint32_t t = wave_nth_free(word, j);
            if (t == 0) t = (uint32_t)group_select<64>(col, k.e0, k.e1, C, n, j);  // beyond color 64 * hub_words
            if (lane < hub_words) atomicExch(&bits[lane], 0ull);
            if (lane == 0) {
                atomicExch(&hub_cnt[k.slot], 0);
                C[k.v] = -(int32_t)t;
                cr.put(k.v, -(int32_t)t);
                atomicAdd(degsum, (unsigned long long)(k.e1 - k.e0));
            }
        }
    }
}

// Detect step for long rows: a chunk that finds a neighbor with the same
// tentative color and a larger priority raises the row's lose flag (hub word
// 0); the last chunk commits the row or appends it to the long-row worklist.
// ROUND0: tentative colors come from the hash and the row's own word is
// written here (+T kept, -T lost).
template <bool ROUND0>
__global__ void __launch_bounds__(INIT_BLOCK) k_split_detect(const int32_t *__restrict__ rp,
                                                             const int32_t *__restrict__ col, int64_t nnz, int32_t n,
                                                             int32_t *C, const int32_t *__restrict__ hub_v,
                                                             const int32_t *__restrict__ hub_first,
                                                             const unsigned long long *__restrict__ plan,
                                                             int32_t split_len, Prio pr, uint32_t s_color,
                                                             uint32_t X, int randx, unsigned long long *hub_bits,
                                                             int32_t *hub_cnt, int32_t *wl_hub, unsigned long long *c_hub,
                                                             ActiveLists al, CopyRef cr, RoundOut ro) {
    const int lane = __lane_id();
    const int32_t nrow = plan_rows(plan), nch = plan_chunks(plan);
    const int wpb = INIT_BLOCK / 64;
    const int wib = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    for (int32_t c = blockIdx.x * wpb + wib; c < nch; c += gridDim.x * wpb) {
        const SplitChunk k = split_chunk(c, nrow, nch, hub_v, hub_first, rp, nnz, split_len, al);
        unsigned long long *flag = hub_bits + (int64_t)k.slot * GC_HUB_WORDS;
        const int32_t t = ROUND0 ? round0_color(s_color, k.v, X, randx != 0) : -C[k.v];
        const uint64_t pv = round_prio(pr, k.v);
        const int32_t *src = k.act ? al.cur : col;
        bool lose;
        if (!ROUND0 && al.next && k.li >= 0)  // the chunk's entries still uncolored go to the row's next list
            lose = wave_loses_keep<ROW_UNROLL(64), false>(t, pv, k.a, k.b, src, C, n, pr, al.next + k.e0, nullptr,
                                                          &al.len_next[k.li]);
        else
            lose = group_loses<64, ROUND0, ROW_UNROLL(64)>(t, pv, k.a, k.b, src, C, n, pr, s_color, X, randx != 0);
        if (lose && lane == 0) atomicOr(flag, 1ull);
        if (split_last(hub_cnt, k.slot, k.nsub)) {
            if (lane == 0) {
                const bool lost = atomicExch(flag, 0ull) != 0ull;
                atomicExch(&hub_cnt[k.slot], 0);
                if (ROUND0) {
                    C[k.v] = lost ? -t : t;
                    cr.put(k.v, lost ? -t : t);
                } else if (!lost) {
                    C[k.v] = t;
                    cr.put(k.v, t);
                }
                if (!lost) ro.put(k.v);
                if (lost) wl_hub[atomicAdd(c_hub, 1ull)] = k.v;
            }
        }
    }
}

// After a long-row detect step: every long row of the plan that committed
// publishes its color, each chunk for its own entries.
__global__ void __launch_bounds__(INIT_BLOCK) k_split_publish(const int32_t *__restrict__ rp,
                                                              const int32_t *__restrict__ col, int64_t nnz, int32_t n,
                                                              const int32_t *C, const int32_t *__restrict__ hub_v,
                                                              const int32_t *__restrict__ hub_first,
                                                              const unsigned long long *__restrict__ plan,
                                                              int32_t split_len, LongMasks lm, ActiveLists al) {
    const int32_t nrow = plan_rows(plan), nch = plan_chunks(plan);
    const int wpb = INIT_BLOCK / 64;
    const int wib = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    for (int32_t c = blockIdx.x * wpb + wib; c < nch; c += gridDim.x * wpb) {
        const SplitChunk k = split_chunk(c, nrow, nch, hub_v, hub_first, rp, nnz, split_len, al);
        const int32_t cv = __builtin_amdgcn_readfirstlane(C[k.v]);
        if (cv > 0) publish_long<64>(lm, k.act ? al.cur : col, k.a, k.b, n, cv);
    }
}

// Mask index of every long row (rows of more than deg_wave entries), -1 for
// the others.  Indexes stop at cap (only reachable with overlapping rows;
// such rows then simply scan their row in the assign step).
__global__ void k_long_index(const int32_t *__restrict__ rp, int32_t n, int64_t nnz, int32_t deg_wave, int64_t cap,
                             int32_t *__restrict__ idx, unsigned long long *count) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        int32_t e0, e1;
        row_range(rp, (int32_t)i, nnz, e0, e1);
        const bool lg = e1 - e0 > deg_wave;
        const unsigned long long b = __ballot(lg);
        unsigned int base = 0;
        const int leader = b ? __ffsll((long long)b) - 1 : 0;
        if (b && __lane_id() == leader) base = (unsigned int)atomicAdd(count, (unsigned long long)__popcll(b));
        base = __shfl(base, leader);
        const int64_t k = (int64_t)base + __popcll(b & ((1ull << __lane_id()) - 1ull));
        idx[i] = (lg && k < cap) ? (int32_t)k : -1;
    }
}

// ---------------------------------------------------------------------------
// Tail of the initial coloring: the remaining (small) rounds in one
// persistent launch, rounds and their assign / detect steps separated by grid
// barriers, so that no round pays for kernel launches and a host read-back.
// One wavefront per vertex, with the per-vertex steps of k_assign<64> /
// k_detect<64> (long-row masks and active lists included); losers go to a
// single worklist.  Every workgroup must be resident for the barriers: the
// workgroups first check in, and unless all of them do within a bounded
// wait the launch decides to do nothing (the host then goes on round by
// round from the same state).  Slots T = scal + S_TAIL: [0] check-in,
// [1] decision (0 open, 1 run, 2 give up), [2] barrier arrivals, [3] barrier
// generation, [4 + (q & 1)] losers of tail round q, [6 + (q & 1)] its degree
// sum, [8] rounds run, [9] status.  Round q's record goes to round_stats.
// ---------------------------------------------------------------------------

#define TAIL_CHECKIN_LIMIT (1u << 14)

__device__ inline int32_t coherent_load(const int32_t *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Grid barrier over every (resident) workgroup; false when a bounded wait ran
// out (recorded as a sticky device error; the launch then stops).  Two
// levels, so that no counter sees more than a few dozen arrivals: workgroup b
// arrives at group counter b % TAIL_GROUPS (each on its own 128-byte line of
// `bar`), the last of each group at the top counter, and the last of those
// bumps the generation T[3] that everyone waits for.
#define TAIL_GROUPS 16
#define TAIL_LINE 16  // 64-bit words per 128-byte line
__device__ inline bool tail_barrier(unsigned long long *T, unsigned long long *bar, uint32_t &gen, uint32_t limit,
                                    unsigned long long *scal, int32_t *lds_flag) {
    // Everything the workgroups exchange inside the launch is written with
    // agent-scope atomics and read with agent-scope atomic loads, so the
    // barrier needs no cache maintenance: each wave waits until its own
    // stores are done, then the workgroup arrives.
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    if (threadIdx.x == 0) {
        bool ok = true;
        const uint32_t groups = gridDim.x < TAIL_GROUPS ? gridDim.x : TAIL_GROUPS;
        const uint32_t grp = blockIdx.x % groups;
        const uint32_t gsize = (gridDim.x - grp + groups - 1) / groups;  // workgroups b with b % groups == grp
        if (atomicAdd(&bar[grp * TAIL_LINE], 1ull) == gsize - 1) {
            atomicExch(&bar[grp * TAIL_LINE], 0ull);
            if (atomicAdd(&bar[TAIL_GROUPS * TAIL_LINE], 1ull) == groups - 1) {
                atomicExch(&bar[TAIL_GROUPS * TAIL_LINE], 0ull);
                atomicExch(&T[3], (unsigned long long)(gen + 1));
            }
        }
        uint32_t it = 0;
        while ((uint32_t)__hip_atomic_load(&T[3], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == gen) {
            if (++it > limit) {
                ok = false;
                atomicOr(&scal[S_ERR], 2ull);
                atomicOr(&scal[S_STICKY], 2ull);
                break;
            }
            __builtin_amdgcn_s_sleep(2);
        }
        *lds_flag = ok ? 1 : 0;
    }
    gen++;
    __syncthreads();
    return *lds_flag != 0;
}

template <int UNR, typename CT>
__global__ void __launch_bounds__(INIT_BLOCK) k_tail_rounds(
    const int32_t *__restrict__ rp, const int32_t *__restrict__ col, int64_t nnz, int32_t n, int32_t *C, CompactCopy<CT> S,
    const int32_t *__restrict__ lo_in, const int32_t *__restrict__ hub_in, const unsigned long long *c_lo_in,
    const unsigned long long *c_hub_in, int32_t *buf0, int32_t *buf1, int32_t r0, int32_t max_rounds, uint64_t seed,
    int fixed_prio, Prio pbase, int randx, uint32_t X, LongMasks lm, ActiveLists al, long long *round_stats,
    unsigned long long *T, unsigned long long *bar, unsigned long long *scal, uint32_t limit, int32_t *vround) {
    __shared__ unsigned long long lmask[INIT_BLOCK];
    __shared__ int32_t sh[4];
    unsigned long long *lw = lmask + (threadIdx.x & ~63u);
    const int lane = __lane_id();
    // check in; run only if every workgroup is resident
    if (threadIdx.x == 0) {
        int32_t d = (int32_t)__hip_atomic_load(&T[1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (d == 0) {
            atomicAdd(&T[0], 1ull);
            for (uint32_t it = 0;; it++) {
                d = (int32_t)__hip_atomic_load(&T[1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                if (d != 0) break;
                if (__hip_atomic_load(&T[0], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) >= gridDim.x)
                    atomicCAS(&T[1], 0ull, 1ull);
                else if (it > TAIL_CHECKIN_LIMIT)
                    atomicCAS(&T[1], 0ull, 2ull);
                __builtin_amdgcn_s_sleep(1);
            }
        }
        __threadfence();
        sh[0] = d;
    }
    __syncthreads();
    if (sh[0] != 1) return;
    const int wpb = INIT_BLOCK / 64;
    const int64_t wave = (int64_t)blockIdx.x * wpb + (threadIdx.x >> 6);
    const int64_t waves = (int64_t)gridDim.x * wpb;
    uint32_t gen = 0;
    int32_t status = GC_OK;
    int32_t q = 0;
    for (;; q++) {
        const int32_t R = r0 + q;
        int64_t cnt_a, cnt_b = 0;
        const int32_t *A, *B = hub_in;
        if (q == 0) {
            A = lo_in;
            cnt_a = (int64_t)__hip_atomic_load(c_lo_in, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            cnt_b = (int64_t)__hip_atomic_load(c_hub_in, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        } else {
            A = (q - 1) & 1 ? buf1 : buf0;
            cnt_a = (int64_t)__hip_atomic_load(&T[4 + ((q - 1) & 1)], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
        const int64_t cnt = cnt_a + cnt_b;
        if (blockIdx.x == 0 && threadIdx.x == 0) {
            if (q > 0) {  // the previous round's record
                round_stats[2 * (int64_t)(R - 1)] = (long long)
                    (q == 1 ? (int64_t)__hip_atomic_load(c_lo_in, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) +
                                  (int64_t)__hip_atomic_load(c_hub_in, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)
                            : (int64_t)__hip_atomic_load(&T[4 + ((q - 2) & 1)], __ATOMIC_RELAXED,
                                                         __HIP_MEMORY_SCOPE_AGENT));
                round_stats[2 * (int64_t)(R - 1) + 1] =
                    (long long)__hip_atomic_load(&T[6 + ((q - 1) & 1)], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                // the degree-sum slot of round q - 1 is round q + 1's: clear it now
                // (round q accumulates in the other one, cleared at the top of round q - 1)
                atomicExch(&T[6 + ((q - 1) & 1)], 0ull);
            }
            // this round's loser count starts at 0 (the slot of round q - 2, recorded above)
            if (q >= 2) atomicExch(&T[4 + (q & 1)], 0ull);
        }
        if (cnt == 0) break;
        if (max_rounds > 0 && R >= max_rounds) {
            status = GC_ERR_NOT_CONVERGED;
            break;
        }
        // assign: the (j+1)-th color free among the neighbors' committed colors
        const uint32_t sc = gc_stream_value(seed, GC_TAG_COLOR, (uint32_t)R);
        unsigned long long degs = 0;
        const CoherentColors cc{C};
        for (int64_t i = wave; i < cnt; i += waves) {
            const int32_t v = i < cnt_a ? coherent_load(&A[i]) : coherent_load(&B[i - cnt_a]);
            int32_t e0, e1;
            row_range(rp, v, nnz, e0, e1);
            const uint32_t j = randx ? gc_pick(sc, v, X) : 0u;
            const int32_t li = lm.idx ? lm.idx[v] : -1;
            int32_t t;
            if (li >= 0) t = fm_select<true>(lm.fm + (size_t)li * FM_WORDS, j, col, e0, e1, cc, n);
            else t = group_select_wide<64, UNR>(col, e0, e1, cc, n, j, lw);
            if (lane == 0) {
                __hip_atomic_store(&C[v], -t, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                degs += (unsigned long long)(e1 - e0);
            }
        }
        if (lane == 0 && degs) atomicAdd(&T[6 + (q & 1)], degs);
        if (!tail_barrier(T, bar, gen, limit, scal, &sh[1])) return;
        // detect: v loses to a neighbor of the same tentative color and larger
        // priority.  The scan stops at the first batch with a conflict, and the
        // active lists are read as they are (no compaction): an entry committed
        // since is never a conflict (its color was excluded by the assign step).
        Prio pr = pbase;
        pr.s_prio = gc_stream_value(seed, GC_TAG_PRIO, fixed_prio ? 0u : (uint32_t)R);
        int32_t *out = q & 1 ? buf1 : buf0;
        for (int64_t i = wave; i < cnt; i += waves) {
            const int32_t v = i < cnt_a ? coherent_load(&A[i]) : coherent_load(&B[i - cnt_a]);
            int32_t e0, e1;
            row_range(rp, v, nnz, e0, e1);
            const int32_t full = e1 - e0;
            int32_t li = -1;
            bool act = false;
            if (al.idx) {
                li = al.idx[v];
                if (li >= 0 && al.len[li] >= 0) {
                    act = true;
                    e1 = e0 + min(al.len[li], full);
                }
            }
            const int32_t t = -cc[v];
            const int32_t *src = act ? al.cur : col;
            const bool lose =
                wave_loses_keep<UNR, true>(t, round_prio(pr, v), e0, e1, src, cc, n, pr, nullptr, nullptr, nullptr);
            if (!lose) {
                if (lane == 0) __hip_atomic_store(&C[v], t, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                if (lane == 0 && vround) vround[v] = R;
                publish_long<64>(lm, src, e0, e1, n, t);
            }
            if (lose && lane == 0)
                __hip_atomic_store(&out[atomicAdd(&T[4 + (q & 1)], 1ull)], v, __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_AGENT);
        }
        if (!tail_barrier(T, bar, gen, limit, scal, &sh[1])) return;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        T[8] = (unsigned long long)q;
        T[9] = (unsigned long long)status;
    }
}

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------

template <int G, typename CT>
static void launch_round0(int grid, hipStream_t s, const gc_csr *g, int32_t *C, CompactCopy<CT> S, int32_t deg_wave, int32_t skip_len,
                          const int32_t *in_list,
                          const unsigned long long *in_count, int32_t *wl_lo, unsigned long long *c_lo,
                          int32_t *wl_hub, unsigned long long *c_hub, Prio pr, uint32_t sc, uint32_t X, int randx,
                          LongMasks lm, RoundOut ro) {
    k_round0<G, CT><<<grid, INIT_BLOCK, 0, s>>>(g->row_ptr, g->col_idx, g->nnz, g->n, C, S, deg_wave, skip_len, in_list, in_count, wl_lo,
                                            c_lo, wl_hub, c_hub, pr, sc, X, randx, lm, ro);
}

template <int G, typename CT>
static void launch_assign(int grid, hipStream_t s, const gc_csr *g, int32_t *C, CompactCopy<CT> S, const int32_t *wl,
                          const unsigned long long *wc, uint32_t sc, uint32_t X, int randx, unsigned long long *degsum,
                          int32_t skip_len, LongMasks lm, unsigned long long *zero2, unsigned long long *zero1,
                          unsigned long long *rec, const unsigned long long *rec_in) {
    k_assign<G, CT><<<grid, INIT_BLOCK, 0, s>>>(g->row_ptr, g->col_idx, g->nnz, g->n, C, S, wl, wc, sc, X, randx, degsum,
                                            skip_len, lm, zero2, zero1, rec, rec_in);
}

template <int G, typename CT>
static void launch_detect(int grid, hipStream_t s, const gc_csr *g, int32_t *C, CompactCopy<CT> S, int32_t deg_wave, const int32_t *wl,
                          const unsigned long long *wc, int32_t *wl_lo, unsigned long long *c_lo, int32_t *wl_hub,
                          unsigned long long *c_hub, Prio pr, int32_t skip_len, LongMasks lm,
                          ActiveLists al, RoundOut ro) {
    constexpr bool L = G == 64;  // the list variants exist for wavefront rows only
    if (L && al.next) {
        if (ro.p)
            k_detect<G, CT, true, L><<<grid, INIT_BLOCK, 0, s>>>(g->row_ptr, g->col_idx, g->nnz, g->n, C, S, deg_wave, wl,
                                                             wc, wl_lo, c_lo, wl_hub, c_hub, pr, skip_len, lm, al, ro);
        else
            k_detect<G, CT, false, L><<<grid, INIT_BLOCK, 0, s>>>(g->row_ptr, g->col_idx, g->nnz, g->n, C, S, deg_wave, wl,
                                                              wc, wl_lo, c_lo, wl_hub, c_hub, pr, skip_len, lm, al, ro);
    } else if (ro.p) {
        k_detect<G, CT, true, false><<<grid, INIT_BLOCK, 0, s>>>(g->row_ptr, g->col_idx, g->nnz, g->n, C, S, deg_wave, wl,
                                                             wc, wl_lo, c_lo, wl_hub, c_hub, pr, skip_len, lm, al, ro);
    } else {
        k_detect<G, CT, false, false><<<grid, INIT_BLOCK, 0, s>>>(g->row_ptr, g->col_idx, g->nnz, g->n, C, S, deg_wave, wl,
                                                              wc, wl_lo, c_lo, wl_hub, c_hub, pr, skip_len, lm, al, ro);
    }
}

#define GC_DISPATCH_G(G, ...)                                   \
    switch (G) {                                                \
        case 1: { constexpr int GG = 1; __VA_ARGS__; } break;   \
        case 2: { constexpr int GG = 2; __VA_ARGS__; } break;   \
        case 4: { constexpr int GG = 4; __VA_ARGS__; } break;   \
        case 8: { constexpr int GG = 8; __VA_ARGS__; } break;   \
        case 16: { constexpr int GG = 16; __VA_ARGS__; } break; \
        case 32: { constexpr int GG = 32; __VA_ARGS__; } break; \
        default: { constexpr int GG = 64; __VA_ARGS__; } break; \
    }

// Speculative rounds over every vertex (arguments already checked, n > 0).
// prank == NULL: the initial coloring with hash priorities; otherwise a
// per-vertex class rank that decides conflicts (asynchronous recoloring).
template <typename CT>
static gc_status spec_rounds_t(gc_ctx *ctx, const gc_csr *g, int32_t select, int32_t X, uint64_t seed,
                               int32_t max_rounds, uint32_t flags, int32_t *colors, gc_stats *st, hipStream_t s,
                               const int32_t *prank, CompactCopy<CT> S) {
    gc_status status = GC_OK;
    int32_t *vround = prank ? nullptr : ctx->vround;  // each vertex's commit round, when asked for
    if (select == GC_FIRST_FIT) X = 1;
    const int randx = select == GC_RANDOM_X ? 1 : 0;
    const int32_t n = g->n;
    // conflict priority of round r
    const int pmode = prank ? PRIO_RANK
                            : (flags & GC_FLAG_PRIO_LF) ? PRIO_LF : (flags & GC_FLAG_PRIO_NATURAL) ? PRIO_NATURAL : PRIO_HASH;
    auto prio_of = [&](int32_t r) {
        const bool fixed = (flags & (GC_FLAG_FIXED_PRIORITY | GC_FLAG_PRIO_LF)) != 0;
        return Prio{pmode, gc_stream_value(seed, GC_TAG_PRIO, fixed ? 0u : (uint32_t)r), prank, g->row_ptr};
    };
    const int G = ctx->tune.group;
    const int32_t deg_wave = ctx->tune.deg_wave;
    const int cap = ctx->num_cu * ctx->tune.grid_per_cu;
    auto grid_for = [&](int64_t items, int gsz) {
        int64_t per = INIT_BLOCK / gsz;
        int64_t want = (items + per - 1) / per;
        return (int)(want < 1 ? 1 : (want > cap ? cap : want));
    };
    // Worklists wl[2 * buf + bin] (bin 0: lane groups, bin 1: wavefronts),
    // counts in scal[S_WL + 2 * buf + bin]; scal[S_WL + 4 + (r & 1)] holds the
    // degree sum of round r.  Round 0 uses wl[3] for the long rows it
    // forwards to its second launch.
    unsigned long long *cnt = ctx->scal + S_WL;
    std::vector<int64_t> sizes, degsum;
    sizes.push_back(n);
    degsum.push_back(g->nnz);
    GC_HIP(hipMemsetAsync(cnt, 0, 6 * 8, s));
    // Long rows (longer than deg_wave and deg_split) go to the split kernels;
    // the others skip them.
    int32_t maxdeg = 0;
    status = gc_graph_max_degree(ctx, g, s, &maxdeg);
    if (status) return status;
    const int32_t thresh = deg_wave > ctx->tune.deg_split ? deg_wave : ctx->tune.deg_split;
    // split kernels only when some row is long enough (without them every row is handled by the others)
    const bool split = ctx->tune.deg_split > 0 && maxdeg > thresh;
    const int32_t skip = split ? thresh : INT32_MAX;
    const int32_t split_len = ctx->tune.split_len;
    if (split) {
        status = gc_ensure_hub_slots(ctx, g->nnz, ctx->tune.deg_split, s);
        if (status) return status;
    }
    // committed-color masks for the long rows (graphs that have any)
    LongMasks lm{nullptr, nullptr};
    if (maxdeg > deg_wave) {
        const int64_t fm_need = g->nnz / ((int64_t)deg_wave + 1) + 1;  // long rows are at most this many
        if (fm_need * FM_WORDS * 8 <= (2LL << 30)) {
            if (!ctx->longidx && hipMalloc((void **)&ctx->longidx, (size_t)ctx->max_n * 4) != hipSuccess) {
                ctx->longidx = nullptr;
                return gc_fail(ctx, GC_ERR_OOM, "long-row mask index");
            }
            if (fm_need > ctx->fm_cap) {
                GC_HIP(hipStreamSynchronize(s));
                if (ctx->fm) { GC_HIP(hipFree(ctx->fm)); ctx->fm = nullptr; ctx->fm_cap = 0; }
                if (hipMalloc((void **)&ctx->fm, (size_t)fm_need * FM_WORDS * 8) != hipSuccess)
                    return gc_fail(ctx, GC_ERR_OOM, "long-row masks (%lld)", (long long)fm_need);
                ctx->fm_cap = fm_need;
            }
            GC_HIP(hipMemsetAsync(ctx->fm, 0, (size_t)fm_need * FM_WORDS * 8, s));
            GC_HIP(hipMemsetAsync(ctx->scal + S_NLONG, 0, 8, s));
            GC_TIMED(GC_K_OTHER, s, k_long_index<<<gc_grid(ctx, n, 256), 256, 0, s>>>(g->row_ptr, n, g->nnz, deg_wave,
                                                                                    fm_need, ctx->longidx,
                                                                                    ctx->scal + S_NLONG));
            GC_LAUNCHED();
            lm = LongMasks{ctx->longidx, ctx->fm};
        }
    }
    const bool masks = lm.idx != nullptr;
    // active lists of the split rows (with the masks): two buffers, swapped
    // after every round that has split rows
    const bool lists = masks;
    int acur = 0;
    if (lists) {
        const int64_t fm_need = g->nnz / ((int64_t)deg_wave + 1) + 1;
        if (2 * g->nnz > ctx->act_cap || 2 * fm_need > ctx->alen_cap) {
            GC_HIP(hipStreamSynchronize(s));
            if (ctx->act) { GC_HIP(hipFree(ctx->act)); ctx->act = nullptr; ctx->act_cap = 0; }
            if (ctx->alen) { GC_HIP(hipFree(ctx->alen)); ctx->alen = nullptr; ctx->alen_cap = 0; }
            if (hipMalloc((void **)&ctx->act, (size_t)(2 * g->nnz) * 4) != hipSuccess ||
                hipMalloc((void **)&ctx->alen, (size_t)(2 * fm_need) * 4) != hipSuccess)
                return gc_fail(ctx, GC_ERR_OOM, "split-row active lists (%lld entries)", (long long)g->nnz);
            ctx->act_cap = 2 * g->nnz;
            ctx->alen_cap = 2 * fm_need;
        }
        GC_HIP(hipMemsetAsync(ctx->alen, 0xFF, (size_t)(ctx->alen_cap / 2) * 4, s));  // no lists yet: -1
    }
    auto lists_of = [&](bool with_next) {
        if (!lists) return ActiveLists{nullptr, nullptr, nullptr, nullptr, nullptr};
        const int64_t half_a = ctx->act_cap / 2, half_l = ctx->alen_cap / 2;
        int32_t *a0 = ctx->act + acur * half_a, *a1 = ctx->act + (acur ^ 1) * half_a;
        int32_t *l0 = ctx->alen + acur * half_l, *l1 = ctx->alen + (acur ^ 1) * half_l;
        return ActiveLists{ctx->longidx, a0, l0, with_next ? a1 : nullptr, with_next ? l1 : nullptr};
    };
    // round r's plan total is scal[S_PLAN + (r & 1)]; its plan launch clears the other
    unsigned long long *plan0 = ctx->scal + S_PLAN;
    if (split) GC_HIP(hipMemsetAsync(plan0, 0, 2 * 8, s));
    auto split_plan = [&](int32_t rr, const int32_t *list, const unsigned long long *count, int64_t items,
                          const ActiveLists &al) {
        const int64_t want = (items + 255) / 256;
        const int grid = (int)(want < 1 ? 1 : (want > cap ? cap : want));
        k_split_plan<<<grid, 256, 0, s>>>(g->row_ptr, g->nnz, list, count, thresh, split_len, ctx->hub_v,
                                          ctx->hub_first, plan0 + (rr & 1), plan0 + ((rr + 1) & 1), al);
    };
    unsigned long long *plan = plan0;  // the current round's plan total
    const Prio sp0 = prio_of(0);
    const uint32_t sc0 = gc_stream_value(seed, GC_TAG_COLOR, 0);
    GC_TIMED(GC_K_ROUND0, s, GC_DISPATCH_G(G, launch_round0<GG, CT>(grid_for(n, GG), s, g, colors, S, deg_wave, skip, nullptr,
                                                                nullptr, ctx->wl[0], cnt + 0, ctx->wl[3], cnt + 3, sp0,
                                                                sc0, (uint32_t)X, randx, lm, RoundOut{vround, 0})));
    GC_LAUNCHED();
    GC_TIMED(GC_K_ROUND0, s, launch_round0<64, CT>(cap, s, g, colors, S, deg_wave, skip, ctx->wl[3], cnt + 3, ctx->wl[0], cnt + 0,
                                               ctx->wl[1], cnt + 1, sp0, sc0, (uint32_t)X, randx, lm, RoundOut{vround, 0}));
    GC_LAUNCHED();
    if (split) {
        const ActiveLists al0 = lists_of(false);  // round 0 reads whole rows and writes no lists
        GC_TIMED(GC_K_OTHER, s, split_plan(0, ctx->wl[3], cnt + 3, (int64_t)cap * 256, al0));
        GC_LAUNCHED();
        GC_TIMED(GC_K_ROUND0, s, k_split_detect<true><<<cap, INIT_BLOCK, 0, s>>>(
                                     g->row_ptr, g->col_idx, g->nnz, n, colors, ctx->hub_v, ctx->hub_first, plan,
                                     split_len, sp0, sc0, (uint32_t)X, randx, ctx->hub_bits, ctx->hub_cnt, ctx->wl[1],
                                     cnt + 1, al0, copy_ref(S), RoundOut{vround, 0}));
        GC_LAUNCHED();
        if (masks) {
            GC_TIMED(GC_K_ROUND0, s, k_split_publish<<<cap, INIT_BLOCK, 0, s>>>(g->row_ptr, g->col_idx, g->nnz, n, colors,
                                                                              ctx->hub_v, ctx->hub_first, plan,
                                                                              split_len, lm, al0));
            GC_LAUNCHED();
        }
    }
    int32_t r = 1, cur = 0;
    // Split rows stay on the split path while their active list is longer than
    // the threshold; lists only shrink, so once a round plans no split row the
    // later rounds skip the split kernels.
    bool split_live = split, planned = split;
    // No launch of a round depends on a value the host must read: the
    // kernels take the worklist counts from the device, each bin's list only
    // shrinks (a vertex keeps its bin, so the last counts read bound the
    // grids, and a bin read empty stays empty), a round whose list is empty
    // does nothing, the split kernels take their rows from the round's plan
    // on the device (an empty plan does nothing), and the active lists swap
    // buffers every round that has long rows.  The host therefore queues up
    // to GC_RUN_AHEAD rounds per read-back, with or without split rows
    // (RMAT-22: 38.4 -> 37.0 ms against one read-back per round while split
    // rows last), and r / 4 rounds (at most GC_RUN_AHEAD_MAX) from round 32
    // on, so a long tail of small rounds pays for few read-backs while a
    // short coloring queues few empty rounds past its end (RMAT-22:
    // 37.0 -> 36.4 ms; the mesh's 8 rounds are unchanged).  Every queued
    // round after the first records its input size and the previous round's
    // degree sum in scal[S_REC + 2q ..], so the statistics stay exact.
    int32_t batch = 0;  // rounds queued since the last read-back
    // Rounds of at most tail_max vertices run in one persistent launch
    // (k_tail_rounds) once no row needs the split kernels.
    bool tail_on = ctx->tune.tail_max > 0;
    const int64_t tail_max = ctx->tune.tail_max;
    int tail_per_cu = 0;  // one workgroup per compute unit, when the kernel fits at all
    GC_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(
        &tail_per_cu, reinterpret_cast<const void *>(k_tail_rounds<ROW_UNROLL(64), CT>), INIT_BLOCK, 0));
    if (tail_per_cu < 1) tail_on = false;
    const int tail_grid = ctx->num_cu;
    for (;;) {
        gc_status ss = gc_sync_scalars(ctx, s);
        if (ss) return ss;
        bool ended = false;
        for (int32_t q = 1; q < batch && !ended; q++) {
            degsum.push_back((int64_t)ctx->hscal[S_REC + 2 * q + 1]);
            const int64_t sz = (int64_t)ctx->hscal[S_REC + 2 * q];
            if (sz == 0) ended = true;  // the queued rounds from this one on were empty
            else sizes.push_back(sz);
        }
        if (ended) break;
        if (planned && lists && (ctx->hscal[S_PLAN + ((r - 1) & 1)] >> 32) == 0) split_live = false;
        const int64_t nlo = (int64_t)ctx->hscal[S_WL + 2 * cur], nhub = (int64_t)ctx->hscal[S_WL + 2 * cur + 1];
        if (r > 1) degsum.push_back((int64_t)ctx->hscal[S_WL + 4 + ((r - 1) & 1)]);
        const int64_t tot = nlo + nhub;
        if (tot == 0) break;
        if (max_rounds > 0 && r == max_rounds) { status = GC_ERR_NOT_CONVERGED; break; }
        if (r > n) return gc_fail(ctx, GC_ERR_DEVICE, "no progress after %d rounds", r);  // each round commits >= 1 vertex
        if (tail_on && !split_live && tot <= tail_max) {
            // the remaining rounds in one persistent launch
            unsigned long long *T = ctx->scal + S_TAIL;
            GC_HIP(hipMemsetAsync(T, 0, 10 * 8, s));
            GC_HIP(hipMemsetAsync(ctx->sync, 0, GC_SYNC_BYTES, s));
            const int nxt = cur ^ 1;
            const ActiveLists al = lists_of(false);  // read as they are
            const bool fixed = (flags & (GC_FLAG_FIXED_PRIORITY | GC_FLAG_PRIO_LF)) != 0;
            const uint32_t limit = ctx->tune.spin_limit > 0 ? (uint32_t)ctx->tune.spin_limit : (1u << 20);
            GC_TIMED(GC_K_DETECT, s, k_tail_rounds<ROW_UNROLL(64), CT><<<tail_grid, INIT_BLOCK, 0, s>>>(
                                         g->row_ptr, g->col_idx, g->nnz, n, colors, S, ctx->wl[2 * cur],
                                         ctx->wl[2 * cur + 1],
                                         cnt + 2 * cur, cnt + 2 * cur + 1, ctx->wl[2 * nxt], ctx->wl[2 * cur], r,
                                         max_rounds, seed, fixed ? 1 : 0, prio_of(0), randx, (uint32_t)X, lm, al,
                                         (long long *)ctx->round_stats, T, ctx->sync, ctx->scal, limit, vround));
            GC_LAUNCHED();
            ss = gc_sync_scalars(ctx, s);
            if (ss) return ss;
            if (ctx->hscal[S_TAIL + 1] == 1) {
                const int32_t q = (int32_t)ctx->hscal[S_TAIL + 8];
                if (q > 0) {
                    std::vector<long long> rec((size_t)2 * q);
                    GC_HIP(hipMemcpyAsync(rec.data(), ctx->round_stats + 2 * (int64_t)r, rec.size() * 8,
                                          hipMemcpyDeviceToHost, s));
                    GC_HIP(hipStreamSynchronize(s));
                    for (int32_t i = 0; i < q; i++) {
                        sizes.push_back(rec[2 * i]);
                        degsum.push_back(rec[2 * i + 1]);
                    }
                }
                r += q;
                // (a barrier that ran out is a sticky device error, reported by the entry point)
                if (ctx->hscal[S_TAIL + 9] == GC_ERR_NOT_CONVERGED) status = GC_ERR_NOT_CONVERGED;
                break;
            }
            tail_on = false;  // not every workgroup was resident: go on round by round
        }
        sizes.push_back(tot);
        batch = r / 4 > GC_RUN_AHEAD ? (r / 4 < GC_RUN_AHEAD_MAX ? r / 4 : GC_RUN_AHEAD_MAX) : GC_RUN_AHEAD;
        if (max_rounds > 0 && max_rounds - r < batch) batch = max_rounds - r;
        for (int32_t q = 0; q < batch; q++) {
            unsigned long long *rec = q > 0 ? ctx->scal + S_REC + 2 * q : nullptr;
            const int nxt = cur ^ 1;
            int32_t *lo_in = ctx->wl[2 * cur], *hub_in = ctx->wl[2 * cur + 1];
            int32_t *lo_out = ctx->wl[2 * nxt], *hub_out = ctx->wl[2 * nxt + 1];
            unsigned long long *c_lo_in = cnt + 2 * cur, *c_hub_in = cnt + 2 * cur + 1;
            unsigned long long *c_lo_out = cnt + 2 * nxt, *c_hub_out = cnt + 2 * nxt + 1;
            // this round's degree sum goes to slot 4 + (r & 1); the assign launches
            // clear c_*_out and the other slot (no memset launches per round)
            unsigned long long *dsum = cnt + 4 + (r & 1), *dsum_next = cnt + 4 + ((r + 1) & 1);
            const uint32_t sc = gc_stream_value(seed, GC_TAG_COLOR, (uint32_t)r);
            const Prio sp = prio_of(r);
            const bool split_round = split_live && nhub > 0;
            planned = split_round;
            const ActiveLists al = lists_of(true);
            plan = plan0 + (r & 1);
            if (split_round) {
                GC_TIMED(GC_K_OTHER, s, split_plan(r, hub_in, c_hub_in, nhub, al));
                GC_LAUNCHED();
            }
            if (nlo) {
                GC_TIMED(GC_K_ASSIGN, s, GC_DISPATCH_G(G, launch_assign<GG, CT>(grid_for(nlo, GG), s, g, colors, S, lo_in, c_lo_in,
                                                                            sc, (uint32_t)X, randx, dsum, skip, lm, c_lo_out,
                                                                            dsum_next, rec, c_lo_in)));
                GC_LAUNCHED();
            }
            if (nhub) {
                // with the masks, long rows of every length take their color here
                GC_TIMED(GC_K_ASSIGN, s, launch_assign<64, CT>(grid_for(nhub, 64), s, g, colors, S, hub_in, c_hub_in, sc, (uint32_t)X,
                                                           randx, dsum, masks ? INT32_MAX : skip, lm, c_lo_out, dsum_next,
                                                           nlo ? nullptr : rec, c_lo_in));
                GC_LAUNCHED();
            }
            if (split_round && !masks) {
                GC_TIMED(GC_K_ASSIGN, s, k_split_assign<<<cap, INIT_BLOCK, 0, s>>>(
                                             g->row_ptr, g->col_idx, g->nnz, n, colors, ctx->hub_v, ctx->hub_first, plan,
                                             split_len, ctx->tune.hub_words, sc, (uint32_t)X, randx, ctx->hub_bits,
                                             ctx->hub_cnt, dsum, copy_ref(S)));
                GC_LAUNCHED();
            }
            if (nlo) {
                GC_TIMED(GC_K_DETECT, s, GC_DISPATCH_G(G, launch_detect<GG, CT>(grid_for(nlo, GG), s, g, colors, S, deg_wave, lo_in,
                                                                            c_lo_in, lo_out, c_lo_out, hub_out, c_hub_out,
                                                                            sp, skip, lm, al, RoundOut{vround, r})));
                GC_LAUNCHED();
            }
            if (nhub) {
                GC_TIMED(GC_K_DETECT, s, launch_detect<64, CT>(grid_for(nhub, 64), s, g, colors, S, deg_wave, hub_in, c_hub_in, lo_out,
                                                           c_lo_out, hub_out, c_hub_out, sp, skip, lm, al, RoundOut{vround, r}));
                GC_LAUNCHED();
            }
            if (split_round) {
                GC_TIMED(GC_K_DETECT, s, k_split_detect<false><<<cap, INIT_BLOCK, 0, s>>>(
                                             g->row_ptr, g->col_idx, g->nnz, n, colors, ctx->hub_v, ctx->hub_first, plan,
                                             split_len, sp, 0u, 1u, 0, ctx->hub_bits, ctx->hub_cnt, hub_out, c_hub_out,
                                             al, copy_ref(S), RoundOut{vround, r}));
                GC_LAUNCHED();
                if (masks) {
                    GC_TIMED(GC_K_DETECT, s, k_split_publish<<<cap, INIT_BLOCK, 0, s>>>(g->row_ptr, g->col_idx, g->nnz, n,
                                                                                      colors, ctx->hub_v, ctx->hub_first,
                                                                                      plan, split_len, lm, al));
                    GC_LAUNCHED();
                }
            }
            if (lists && nhub > 0) acur ^= 1;  // this round's surviving entries are the next round's lists
            cur = nxt;
            r++;
        }
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

gc_status gc_spec_rounds(gc_ctx *ctx, const gc_csr *g, int32_t select, int32_t X, uint64_t seed, int32_t max_rounds,
                         uint32_t flags, int32_t *colors, gc_stats *st, hipStream_t s, const int32_t *prank) {
    // Neighbor reads through a compact copy of the colors: one byte when no
    // color can exceed 127 (a color is at most the row length plus X), else
    // two.  compact_init 1: always; -1: the one-byte copy when most adjacency
    // entries point far away in the vertex order (there the int32 colors'
    // cache lines are rarely shared by neighbors, and a quarter of the bytes
    // keeps more of them in the L2: a random graph of 4 M vertices, 8.5 ->
    // 4.8 ms).  With near neighbors the copy's stores cost more than it
    // saves (the 27-point mesh), and the two-byte copy measured slower on
    // RMAT-22 (46.2 against 42.6 ms), so neither is taken by default.
    int32_t maxdeg = 0;
    gc_status status = gc_graph_max_degree(ctx, g, s, &maxdeg);
    if (status) return status;
    double far = 0.0;
    status = gc_graph_far_fraction(ctx, g, s, &far);
    if (status) return status;
    const int32_t xw = select == GC_FIRST_FIT ? 1 : X;
    const bool fits8 = (int64_t)maxdeg + xw <= 127;
    const bool compact = ctx->tune.compact_init == 1 || (ctx->tune.compact_init == -1 && far > 0.5 && fits8);
    const int32_t sat = ctx->tune.compact_sat > 0 ? ctx->tune.compact_sat : 32767;
    if (compact && fits8)
        return spec_rounds_t<int8_t>(ctx, g, select, X, seed, max_rounds, flags, colors, st, s, prank,
                                     CompactCopy<int8_t>{(int8_t *)ctx->shadow, 127});
    if (compact)
        return spec_rounds_t<int16_t>(ctx, g, select, X, seed, max_rounds, flags, colors, st, s, prank,
                                      CompactCopy<int16_t>{(int16_t *)ctx->shadow, sat});
    return spec_rounds_t<int32_t>(ctx, g, select, X, seed, max_rounds, flags, colors, st, s, prank,
                                  CompactCopy<int32_t>{colors, 0});
}

static gc_status gc_init_color_impl(gc_ctx *ctx, const gc_csr *g, int32_t select, int32_t X, uint64_t seed,
                                   int32_t max_rounds, uint32_t flags, int32_t *colors, gc_stats *st, void *stream) {
    gc_status status = gc_check_graph_args(ctx, g);
    if (status) return status;
    if (select != GC_FIRST_FIT && select != GC_RANDOM_X) return gc_fail(ctx, GC_ERR_ARG, "select must be GC_FIRST_FIT or GC_RANDOM_X");
    if (select == GC_RANDOM_X && (X < 1 || X > GC_MAX_X)) return gc_fail(ctx, GC_ERR_ARG, "X must be in [1, %d]", GC_MAX_X);
    if (max_rounds < 0) return gc_fail(ctx, GC_ERR_ARG, "max_rounds must be >= 0");
    if (g->n > 0 && !colors) return gc_fail(ctx, GC_ERR_ARG, "colors is NULL");
    if ((flags & GC_FLAG_PRIO_LF) && (flags & GC_FLAG_PRIO_NATURAL))
        return gc_fail(ctx, GC_ERR_ARG, "GC_FLAG_PRIO_LF and GC_FLAG_PRIO_NATURAL exclude each other");
    const bool d2 = (flags & GC_FLAG_DISTANCE2) != 0;
    if (d2 && (flags & GC_FLAG_PRIO_LF))
        return gc_fail(ctx, GC_ERR_ARG, "GC_FLAG_PRIO_LF is not available with GC_FLAG_DISTANCE2");
    if (flags & ~(GC_FLAG_FIXED_PRIORITY | GC_FLAG_PRIO_LF | GC_FLAG_PRIO_NATURAL | GC_FLAG_DISTANCE2))
        return gc_fail(ctx, GC_ERR_ARG, "unknown flags 0x%x", flags);
    GC_HIP(hipSetDevice(ctx->device));
    if (g->n == 0) {
        if (st) { st->rounds = 0; st->num_colors = 0; st->max_color = 0; st->k_classes = 0; st->losers_total = 0; }
        return GC_OK;
    }
    if (d2) {
        int32_t maxdeg = 0;
        status = gc_graph_max_degree(ctx, g, (hipStream_t)stream, &maxdeg);
        if (status) return status;
        if (maxdeg >= GC_D2_MAX_DEGREE)
            return gc_fail(ctx, GC_ERR_ARG, "distance-2 coloring takes rows below %d entries", GC_D2_MAX_DEGREE);
        return gc_spec_rounds_d2(ctx, g, select, X, seed, max_rounds, flags, colors, st, (hipStream_t)stream);
    }
    return gc_spec_rounds(ctx, g, select, X, seed, max_rounds, flags, colors, st, (hipStream_t)stream, nullptr);
}

// Public entry points: the implementations above, with any sticky device
// failure harvested on the way reported in the returned status.
extern "C" gc_status gc_init_color(gc_ctx *ctx, const gc_csr *g, int32_t select, int32_t X, uint64_t seed,
                                   int32_t max_rounds, uint32_t flags, int32_t *colors, gc_stats *st, void *stream) {
    return gc_report(ctx, gc_init_color_impl(ctx, g, select, X, seed, max_rounds, flags, colors, st, stream));
}

static gc_status gc_init_color_rounds_impl(gc_ctx *ctx, const gc_csr *g, int32_t select, int32_t X, uint64_t seed,
                                           int32_t max_rounds, uint32_t flags, int32_t *colors,
                                           int32_t *vertex_round, gc_stats *st, void *stream) {
    if (!ctx) return GC_ERR_ARG;
    gc_status status = gc_check_graph_args(ctx, g);
    if (status) return status;
    if (g->n > 0 && !vertex_round) return gc_fail(ctx, GC_ERR_ARG, "vertex_round is NULL");
    if (flags & GC_FLAG_DISTANCE2)
        return gc_fail(ctx, GC_ERR_ARG, "commit rounds are not recorded for GC_FLAG_DISTANCE2");
    if (g->n > 0) {
        GC_HIP(hipSetDevice(ctx->device));
        GC_HIP(hipMemsetAsync(vertex_round, 0xFF, (size_t)g->n * 4, (hipStream_t)stream));  // -1: not committed
    }
    ctx->vround = vertex_round;
    status = gc_init_color_impl(ctx, g, select, X, seed, max_rounds, flags, colors, st, stream);
    ctx->vround = nullptr;
    return status;
}

extern "C" gc_status gc_init_color_rounds(gc_ctx *ctx, const gc_csr *g, int32_t select, int32_t X, uint64_t seed,
                                          int32_t max_rounds, uint32_t flags, int32_t *colors, int32_t *vertex_round,
                                          gc_stats *st, void *stream) {
    return gc_report(ctx, gc_init_color_rounds_impl(ctx, g, select, X, seed, max_rounds, flags, colors, vertex_round,
                                                    st, stream));
}
