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
// Color masks.  M[u] (D2_MW words) holds the colors 1 .. D2_MCOLORS settled
// in N(u) u {u}: colors committed by the rounds so far, or the new colors of
// the recoloring pass so far.  The OR of M[u] over u in N(v) is then exactly
// the set of settled colors of N2(v) in that range, so the selections read
// deg(v) masks instead of the sum of the neighbors' degrees; a vertex that
// settles ORs its color into the masks of N(v) u {v}.  Selections run with
// G lanes per vertex; a vertex whose (j+1)-th free color lies above
// D2_MCOLORS scans N2(v) itself, window by window.  In a recoloring pass
// two vertices of one class are never within two edges, so no vertex reads
// a mask that another vertex of its class is writing.
//
// Encoding of C during the rounds is the distance-1 one: C[v] > 0 committed,
// C[v] < 0 tentative (or a loser waiting for the next round).  A tentative
// color T_v avoids every color committed in N2(v) before the round, so a w in
// N2(v) with |C[w]| = T_v belongs to the same round, whether it has already
// committed in this detect step or not.
#include "gc_internal.h"

#include <vector>

#define D2_BLOCK 256
#define D2_UNROLL 4
#define D2_ROW_UNROLL 4  // neighbor ids per lane in flight in the mask scans of a row (mesh 128^3 step 25.7 -> 22.8 ms)
#define D2_MW 2                    // mask words per vertex
#define D2_MCOLORS (64 * D2_MW)    // colors tracked by the masks

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

// Losers of a round collect in LDS and go to the next worklist with one
// global atomic per flush: per wavefront (64 slots) in the wavefront-per-vertex
// kernels, whose vertices finish at different times; per workgroup in the
// group kernels (loops workgroup-uniform around the push and flush calls).
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

struct LoserQueue {
    int32_t buf[GC_QCAP];
    int32_t cnt, base;
};

// ORs color c into M[u] for u in N(v) u {v} (colors above D2_MCOLORS are
// not tracked).  G lanes, gl = lane in the group.  ATOMIC = false when no
// other vertex can write the same masks during the launch: in a recoloring
// pass, N(u) u {u} holds at most one vertex of each class of the (distance-2)
// input coloring, so one class launch has a single writer per mask.
template <int G, bool ATOMIC>
__device__ inline void d2_publish(const int32_t *__restrict__ col, int32_t e0, int32_t e1, int32_t n,
                                  unsigned long long *M, int32_t v, int32_t c, int gl) {
    if (c < 1 || c > D2_MCOLORS) return;
    const unsigned long long bit = 1ull << ((c - 1) & 63);
    const int w_ = (c - 1) >> 6;
    auto put = [&](int32_t u) {
        unsigned long long *p = &M[(size_t)D2_MW * u + w_];
        if (ATOMIC) atomicOr(p, bit);
        else *p |= bit;
    };
    if (gl == 0) put(v);
    // a batch's neighbor ids first, then all its atomics, or (one writer per
    // mask) all its mask loads before its stores: a row takes one round trip
    // per batch instead of one per entry (two entries of a batch naming the
    // same u set the same bit)
    for (int32_t eb = e0 + gl; eb < e1; eb += G * D2_ROW_UNROLL) {
        int32_t w[D2_ROW_UNROLL];
#pragma unroll
        for (int k = 0; k < D2_ROW_UNROLL; k++) {
            const int32_t e = eb + k * G;
            const int32_t x = col[e < e1 ? e : eb];
            w[k] = e < e1 && (uint32_t)x < (uint32_t)n ? x : -1;
        }
        if (ATOMIC) {
#pragma unroll
            for (int k = 0; k < D2_ROW_UNROLL; k++)
                if (w[k] >= 0) put(w[k]);
        } else {
            unsigned long long old[D2_ROW_UNROLL];
#pragma unroll
            for (int k = 0; k < D2_ROW_UNROLL; k++) old[k] = M[(size_t)D2_MW * (w[k] >= 0 ? w[k] : v) + w_];
#pragma unroll
            for (int k = 0; k < D2_ROW_UNROLL; k++)
                if (w[k] >= 0) M[(size_t)D2_MW * w[k] + w_] = old[k] | bit;
        }
    }
}

// (j+1)-th smallest color free in the OR of M[u] over u in N(v), among
// 1 .. D2_MCOLORS; 0 when there are not that many (then *jrem = j minus the
// free colors of that range).  G lanes, same result in each.
template <int G>
__device__ inline int32_t d2_mask_select(const int32_t *__restrict__ col, int32_t e0, int32_t e1, int32_t n,
                                         const unsigned long long *__restrict__ M, uint32_t j, int gl,
                                         uint32_t *jrem) {
    static_assert(D2_MW == 2, "two mask words");
    unsigned long long f0 = 0, f1 = 0;
    // a batch's neighbor ids, then all its mask loads (an invalid id reads
    // vertex 0's masks and drops them)
    for (int32_t eb = e0 + gl; eb < e1; eb += G * D2_ROW_UNROLL) {
        int32_t w[D2_ROW_UNROLL];
#pragma unroll
        for (int k = 0; k < D2_ROW_UNROLL; k++) {
            const int32_t e = eb + k * G;
            const int32_t x = col[e < e1 ? e : eb];
            w[k] = e < e1 && (uint32_t)x < (uint32_t)n ? x : -1;
        }
#pragma unroll
        for (int k = 0; k < D2_ROW_UNROLL; k++) {
            const ulonglong2 m = *reinterpret_cast<const ulonglong2 *>(M + (size_t)D2_MW * (w[k] >= 0 ? w[k] : 0));
            f0 |= w[k] >= 0 ? m.x : 0ull;
            f1 |= w[k] >= 0 ? m.y : 0ull;
        }
    }
    f0 = ~group_or_u64<G>(f0);
    f1 = ~group_or_u64<G>(f1);
    const uint32_t c0 = (uint32_t)__popcll(f0);
    if (j < c0) return 1 + (int32_t)nth_set_bit(f0, j);
    j -= c0;
    const uint32_t c1 = (uint32_t)__popcll(f1);
    if (j < c1) return 65 + (int32_t)nth_set_bit(f1, j);
    *jrem = j - c1;
    return 0;
}

// (j+1)-th smallest color >= base held by no w in N2(v) as a positive value
// of C, by scanning N2(v) (each lane walks the rows of its neighbors), 64
// colors per window.  G lanes, same result in each.
template <int G>
__device__ inline int32_t d2_scan_select(const int32_t *__restrict__ rp, const int32_t *__restrict__ col, int64_t nnz,
                                         int32_t n, const int32_t *C, int32_t v, int32_t e0, int32_t e1,
                                         uint32_t base, uint32_t j, int gl) {
    auto mark = [&](unsigned long long &m, int32_t c) {
        const uint32_t d = (uint32_t)c - base;
        if (c > 0 && d < 64u) m |= 1ull << d;
    };
    for (;;) {
        unsigned long long m = 0;
        for (int32_t e = e0 + gl; e < e1; e += G) {
            const int32_t u = col[e];
            if ((uint32_t)u >= (uint32_t)n) continue;
            mark(m, C[u]);
            int32_t a, b;
            row_range(rp, u, nnz, a, b);
            for (int32_t f = a; f < b; f++) {
                const int32_t w = col[f];
                if (w != v && (uint32_t)w < (uint32_t)n) mark(m, C[w]);
            }
        }
        const unsigned long long fr = ~group_or_u64<G>(m);
        const uint32_t cnt = (uint32_t)__popcll(fr);
        if (j < cnt) return (int32_t)(base + nth_set_bit(fr, j));
        j -= cnt;
        base += 64u;
    }
}

__device__ inline int32_t d2_round0_color(uint32_t s_color, int32_t w, uint32_t X, int randx) {
    return randx ? (int32_t)gc_pick(s_color, w, X) + 1 : 1;
}

// Round 0: every vertex's tentative color follows from the hash alone (no
// color is held yet), so assign and detect fuse: v keeps T_v unless a
// vertex of N2(v) with the same T has a larger key.
__global__ void __launch_bounds__(D2_BLOCK) k_d2_round0(const int32_t *__restrict__ rp,
                                                        const int32_t *__restrict__ col, int64_t nnz, int32_t n,
                                                        int32_t *C, unsigned long long *M, Prio pr, uint32_t s_color,
                                                        uint32_t X, int randx, int32_t *wl_out,
                                                        unsigned long long *c_out) {
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
        else d2_publish<64, true>(col, e0, e1, n, M, v, T, __lane_id());
    }
    lq.flush(wl_out, c_out);
}

// Rounds >= 1, assign step: every vertex of the worklist takes the (j+1)-th
// smallest color free in N2(v) among the colors committed before the round
// (G lanes per vertex, from the masks).
template <int G>
__global__ void __launch_bounds__(D2_BLOCK) k_d2_assign(const int32_t *__restrict__ rp,
                                                        const int32_t *__restrict__ col, int64_t nnz, int32_t n,
                                                        int32_t *C, const unsigned long long *__restrict__ M,
                                                        const int32_t *__restrict__ wl,
                                                        const unsigned long long *__restrict__ wc, uint32_t s_color,
                                                        uint32_t X, int randx) {
    const int gpb = D2_BLOCK / G;
    const int gl = threadIdx.x & (G - 1);
    const int64_t cnt = (int64_t)*wc;
    for (int64_t i = (int64_t)blockIdx.x * gpb + threadIdx.x / G; i < cnt; i += (int64_t)gridDim.x * gpb) {
        const int32_t v = wl[i];
        int32_t e0, e1;
        row_range(rp, v, nnz, e0, e1);
        const uint32_t j = randx ? gc_pick(s_color, v, X) : 0u;
        uint32_t jr = 0;
        int32_t c = d2_mask_select<G>(col, e0, e1, n, M, j, gl, &jr);
        if (c == 0) c = d2_scan_select<G>(rp, col, nnz, n, C, v, e0, e1, D2_MCOLORS + 1, jr, gl);
        if (gl == 0) C[v] = -c;
    }
}

// Rounds >= 1, detect step: v loses iff some w in N2(v) holds the same
// tentative color (|C[w]| = T_v) with a larger key; winners commit.
__global__ void __launch_bounds__(D2_BLOCK) k_d2_detect(const int32_t *__restrict__ rp,
                                                        const int32_t *__restrict__ col, int64_t nnz, int32_t n,
                                                        int32_t *C, const int32_t *__restrict__ wl,
                                                        const unsigned long long *__restrict__ wc,
                                                        unsigned long long *M, Prio pr, int32_t *wl_out,
                                                        unsigned long long *c_out) {
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
        else d2_publish<64, true>(col, e0, e1, n, M, v, T, __lane_id());
    }
    lq.flush(wl_out, c_out);
}

// One class of a recoloring pass: every vertex of the class takes the
// smallest color free among the new colors of N2(v) (G lanes per vertex, from
// the masks) and publishes it.
template <int G>
__global__ void __launch_bounds__(D2_BLOCK) k_d2_class(const int32_t *__restrict__ rp, const int32_t *__restrict__ col,
                                                       int64_t nnz, int32_t n, int32_t *C, unsigned long long *M,
                                                       const int32_t *__restrict__ list, int32_t a, int32_t b) {
    const int gpb = D2_BLOCK / G;
    const int gl = threadIdx.x & (G - 1);
    for (int32_t i = a + blockIdx.x * gpb + (int32_t)threadIdx.x / G; i < b; i += gridDim.x * gpb) {
        const int32_t v = list[i];
        int32_t e0, e1;
        row_range(rp, v, nnz, e0, e1);
        uint32_t jr = 0;
        int32_t c = d2_mask_select<G>(col, e0, e1, n, M, 0u, gl, &jr);
        if (c == 0) c = d2_scan_select<G>(rp, col, nnz, n, C, v, e0, e1, D2_MCOLORS + 1, jr, gl);
        if (gl == 0) C[v] = c;
        d2_publish<G, false>(col, e0, e1, n, M, v, c, gl);
    }
}

// Detect step of a large round (rows of at most D2_STAR_ROW entries), in two
// launches.  v loses iff, for some u in N(v) u {v}, another member of
// S(u) = N(u) u {u} holds v's tentative color with a larger key (every w of
// N2(v) lies in such an S(u) together with v).  k_d2_mark: one group per
// vertex u stages (color, key) of the tentative members of S(u) in LDS and
// marks the members so dominated (1).  A row longer than D2_STAR_ROW does
// not fit the stage: its tentative members are marked for a recheck (2)
// instead.  k_d2_commit: unmarked vertices of the round commit and publish,
// marked ones clear the mark and go to the next round, and those marked for
// a recheck scan N2(v) themselves.  Marks may overwrite each other: a 1 is
// only ever written for a vertex that loses, and a 2 leads to the exact scan.
#define D2_STAR_ROW 64

// Does some w in N2(v) hold |C[w]| = T with a larger key than pv?  Each lane
// walks the rows of its neighbors; G lanes, same result in each.
template <int G>
__device__ inline bool d2_scan_conflict(const int32_t *__restrict__ rp, const int32_t *__restrict__ col, int64_t nnz,
                                        int32_t n, const int32_t *C, const Prio &pr, int32_t v, int32_t e0,
                                        int32_t e1, int32_t T, uint64_t pv, int gl) {
    auto hit = [&](int32_t w) {
        const int32_t c = C[w];
        return (c == T || c == -T) && round_prio(pr, w) > pv;
    };
    bool found = false;
    for (int32_t e = e0 + gl; e < e1 && !found; e += G) {
        const int32_t u = col[e];
        if ((uint32_t)u >= (uint32_t)n) continue;
        found = hit(u);
        int32_t a, b;
        row_range(rp, u, nnz, a, b);
        for (int32_t f = a; f < b && !found; f++) {
            const int32_t w = col[f];
            if (w != v && (uint32_t)w < (uint32_t)n) found = hit(w);
        }
    }
    return group_or_u64<G>(found ? 1ull : 0ull) != 0;
}

template <int G>
__global__ void __launch_bounds__(D2_BLOCK) k_d2_mark(const int32_t *__restrict__ rp, const int32_t *__restrict__ col,
                                                      int64_t nnz, int32_t n, const int32_t *__restrict__ C, Prio pr,
                                                      uint8_t *lost) {
    __shared__ unsigned long long tab[D2_BLOCK / G][D2_STAR_ROW + 1];
    const int gpb = D2_BLOCK / G;
    const int gid = threadIdx.x / G, gl = threadIdx.x & (G - 1);
    unsigned long long *t = tab[gid];
    for (int32_t u = blockIdx.x * gpb + gid; u < n; u += gridDim.x * gpb) {
        int32_t e0, e1;
        row_range(rp, u, nnz, e0, e1);
        if (e1 - e0 > D2_STAR_ROW) {
            for (int32_t i = gl; i <= e1 - e0; i += G) {
                const int32_t x = i == 0 ? u : col[e0 + i - 1];
                if ((uint32_t)x < (uint32_t)n && C[x] < 0) lost[x] = 2;
            }
            continue;
        }
        const int32_t sz = e1 - e0 + 1;
        // a batch of member ids, then all their colors, then the stage
        for (int32_t ib = gl; ib < sz; ib += G * D2_ROW_UNROLL) {
            int32_t x[D2_ROW_UNROLL], c[D2_ROW_UNROLL];
#pragma unroll
            for (int k = 0; k < D2_ROW_UNROLL; k++) {
                const int32_t i = ib + k * G < sz ? ib + k * G : ib;
                const int32_t y = i == 0 ? u : col[e0 + i - 1];
                x[k] = ib + k * G < sz && (uint32_t)y < (uint32_t)n ? y : -1;
            }
#pragma unroll
            for (int k = 0; k < D2_ROW_UNROLL; k++) c[k] = C[x[k] >= 0 ? x[k] : u];
#pragma unroll
            for (int k = 0; k < D2_ROW_UNROLL; k++) {
                uint32_t T = 0, key = 0;  // T = 0: not tentative (never matches)
                if (x[k] >= 0 && c[k] < 0) {
                    T = (uint32_t)(-c[k]);
                    key = (uint32_t)round_prio(pr, x[k]);
                }
                if (ib + k * G < sz) t[ib + k * G] = ((unsigned long long)T << 32) | key;
            }
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        for (int32_t i = gl; i < sz; i += G) {
            const unsigned long long me = t[i];
            const uint32_t T = (uint32_t)(me >> 32);
            if (T == 0) continue;
            bool dom = false;
            // unrolled: the stage reads pipeline (mesh 128^3 step 22.6 -> 21.8 ms)
#pragma unroll 8
            for (int32_t q = 0; q < sz; q++) {
                const unsigned long long o = t[q];
                dom |= (uint32_t)(o >> 32) == T && (uint32_t)o > (uint32_t)me;
            }
            if (dom) lost[i == 0 ? u : col[e0 + i - 1]] = 1;
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
    }
}

template <int G>
__global__ void __launch_bounds__(D2_BLOCK) k_d2_commit(const int32_t *__restrict__ rp,
                                                        const int32_t *__restrict__ col, int64_t nnz, int32_t n,
                                                        int32_t *C, unsigned long long *M, uint8_t *lost, Prio pr,
                                                        const int32_t *__restrict__ wl,
                                                        const unsigned long long *__restrict__ wc, int32_t *wl_out,
                                                        unsigned long long *c_out) {
    __shared__ LoserQueue q;
    if (threadIdx.x == 0) q.cnt = 0;
    __syncthreads();
    const int gpb = D2_BLOCK / G;
    const int gl = threadIdx.x & (G - 1);
    const int64_t cnt = (int64_t)*wc;
    for (int64_t b = (int64_t)blockIdx.x * gpb; b < cnt; b += (int64_t)gridDim.x * gpb) {
        const int64_t i = b + threadIdx.x / G;
        bool lose = false;
        int32_t v = -1;
        if (i < cnt) {
            v = wl[i];
            const int32_t T = -C[v];
            int32_t e0, e1;
            row_range(rp, v, nnz, e0, e1);
            const uint8_t mark = lost[v];
            lose = mark == 1;
            if (mark == 2) lose = d2_scan_conflict<G>(rp, col, nnz, n, C, pr, v, e0, e1, T, round_prio(pr, v), gl);
            if (mark && gl == 0) lost[v] = 0;
            if (!lose) {
                if (gl == 0) C[v] = T;
                d2_publish<G, true>(col, e0, e1, n, M, v, T, gl);
            }
        }
        bq_push(q.buf, &q.cnt, lose && gl == 0, v);
        __syncthreads();
        bq_flush(q.buf, &q.cnt, &q.base, wl_out, c_out, false);
    }
    __syncthreads();
    bq_flush(q.buf, &q.cnt, &q.base, wl_out, c_out, true);
}

// Vertices sharing their positive color with a vertex of N2(v), and vertices
// with color <= 0.
// Distance-2 check, phase 1: uncolored vertices, and the vertices that share
// their color with some vertex of N2(v) (early exit at the first), appended
// to `bad` for phase 2.
__global__ void __launch_bounds__(D2_BLOCK) k_d2_validate(const int32_t *__restrict__ rp,
                                                          const int32_t *__restrict__ col, int64_t nnz, int32_t n,
                                                          const int32_t *__restrict__ C, unsigned long long *nbad,
                                                          unsigned long long *uncolored, int32_t *__restrict__ bad) {
    const int wpb = D2_BLOCK / 64;
    const int wib = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    unsigned long long nu = 0;
    for (int32_t v = blockIdx.x * wpb + wib; v < n; v += gridDim.x * wpb) {
        const int32_t cv = __builtin_amdgcn_readfirstlane(C[v]);
        if (cv <= 0) {
            nu++;
            continue;
        }
        int32_t e0, e1;
        row_range(rp, v, nnz, e0, e1);
        if (d2_visit(rp, col, nnz, n, v, e0, e1, [&](int32_t w) { return C[w] == cv; }) && __lane_id() == 0)
            bad[atomicAdd(nbad, 1ull)] = v;
    }
    if (__lane_id() == 0 && nu) atomicAdd(uncolored, nu);
}

#define D2_SET 2048             // LDS hash-set slots per wavefront
#define D2_SET_FILL (D2_SET / 2)  // keys one sweep may hold: probes always meet an empty slot

// Distance-2 check, phase 2 (vertices of phase 1 only): for each such v, the
// number of DISTINCT w > v in N2(v) with C[w] = C[v]; the visit reaches a w
// once per path, so the partners are deduplicated in an LDS hash set.  A
// first sweep counts partner visits (with repeats), an upper bound of the
// distinct partners; the partners are split over that bound / D2_SET_FILL
// sweeps by a hash of w, each deduplicated on its own.  A sweep whose part
// would overfill the set (an uneven split) stops inserting, and the vertex
// starts over with twice the sweeps, so every probe sequence ends.
__global__ void __launch_bounds__(D2_BLOCK) k_d2_pairs(const int32_t *__restrict__ rp, const int32_t *__restrict__ col,
                                                       int64_t nnz, int32_t n, const int32_t *__restrict__ C,
                                                       const int32_t *__restrict__ bad,
                                                       const unsigned long long *__restrict__ nbad,
                                                       unsigned long long *pairs) {
    __shared__ int32_t set_all[(D2_BLOCK / 64) * D2_SET];
    __shared__ int32_t fill_all[D2_BLOCK / 64];
    const int wpb = D2_BLOCK / 64;
    const int wib = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int lane = __lane_id();
    int32_t *set = set_all + wib * D2_SET;
    int32_t *fill = fill_all + wib;
    const int64_t nb = (int64_t)*nbad;
    unsigned long long total = 0;
    for (int64_t i = (int64_t)blockIdx.x * wpb + wib; i < nb; i += (int64_t)gridDim.x * wpb) {
        const int32_t v = __builtin_amdgcn_readfirstlane(bad[i]);
        const int32_t cv = __builtin_amdgcn_readfirstlane(C[v]);
        int32_t e0, e1;
        row_range(rp, v, nnz, e0, e1);
        unsigned long long visits = 0;
        (void)d2_visit(rp, col, nnz, n, v, e0, e1, [&](int32_t w) {
            if (w > v && C[w] == cv) visits++;
            return false;
        });
        for (int o = 32; o >= 1; o >>= 1) visits += __shfl_xor(visits, o);
        uint64_t sweeps = (visits + D2_SET_FILL - 1) / D2_SET_FILL;
        unsigned long long found = 0;
        for (uint64_t r = 0; r < sweeps; r++) {
            for (int j = lane; j < D2_SET; j += 64) set[j] = -1;
            if (lane == 0) *fill = 0;
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            bool over = false;
            (void)d2_visit(rp, col, nnz, n, v, e0, e1, [&](int32_t w) {
                if (w > v && C[w] == cv) {
                    const uint32_t h = (uint32_t)w * 0x9E3779B1u;
                    if (sweeps == 1 || (uint64_t)(h >> 8) % sweeps == r) {
                        for (uint32_t k = h & (D2_SET - 1);; k = (k + 1) & (D2_SET - 1)) {
                            const int32_t cur = atomicAdd(&set[k], 0);
                            if (cur == w) break;
                            if (cur != -1) continue;
                            // reserve room first: the set never holds more than D2_SET_FILL keys
                            if (atomicAdd(fill, 1) >= D2_SET_FILL) {
                                over = true;
                                break;
                            }
                            const int32_t old = atomicCAS(&set[k], -1, w);
                            if (old == -1) {
                                found++;
                                break;
                            }
                            atomicSub(fill, 1);
                            if (old == w) break;
                        }
                    }
                }
                return false;
            });
            __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
            __builtin_amdgcn_wave_barrier();
            if (__ballot(over)) {  // uneven split: start this vertex over with twice the sweeps
                sweeps *= 2;
                r = (uint64_t)-1;
                found = 0;
            }
        }
        total += found;
    }
    for (int o = 32; o >= 1; o >>= 1) total += __shfl_xor(total, o);
    if (lane == 0 && total) atomicAdd(pairs, total);
}

// workgroups for `items` vertices at `per_vertex` lanes each
static int d2_grid(const gc_ctx *ctx, int64_t items, int per_vertex = 64) {
    const int64_t cap = (int64_t)ctx->num_cu * ctx->tune.grid_per_cu;
    const int64_t per = D2_BLOCK / per_vertex;
    const int64_t want = (items + per - 1) / per;
    return (int)(want < 1 ? 1 : (want > cap ? cap : want));
}

// Lanes per vertex of the mask selections: 8, or a wavefront when some row is
// longer than 64 entries.
static int d2_group(int32_t maxdeg) { return maxdeg > 64 ? 64 : 8; }

// The masks (max_n * D2_MW words) followed by the detect marks (max_n bytes).
static uint8_t *d2_lost(gc_ctx *ctx) { return (uint8_t *)(ctx->d2mask + (size_t)ctx->max_n * D2_MW); }

static gc_status d2_masks(gc_ctx *ctx, int32_t n, hipStream_t s) {
    if (!ctx->d2mask) {
        GC_HIP(hipStreamSynchronize(s));
        if (hipMalloc((void **)&ctx->d2mask, (size_t)ctx->max_n * (D2_MW * 8 + 1) + 256) != hipSuccess) {
            ctx->d2mask = nullptr;
            return gc_fail(ctx, GC_ERR_OOM, "distance-2 color masks (%lld vertices)", (long long)ctx->max_n);
        }
    }
    GC_HIP(hipMemsetAsync(ctx->d2mask, 0, (size_t)n * D2_MW * 8, s));
    return GC_OK;
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
    int32_t maxdeg = 0;
    status = gc_graph_max_degree(ctx, g, s, &maxdeg);
    if (status) return status;
    const int G = d2_group(maxdeg);
    status = d2_masks(ctx, n, s);
    if (status) return status;
    unsigned long long *M = ctx->d2mask;
    uint8_t *lost = d2_lost(ctx);
    GC_HIP(hipMemsetAsync(lost, 0, (size_t)n, s));
    GC_HIP(hipMemsetAsync(cnt, 0, 2 * 8, s));
    GC_TIMED(GC_K_ROUND0, s, k_d2_round0<<<d2_grid(ctx, n), D2_BLOCK, 0, s>>>(
                                 g->row_ptr, g->col_idx, g->nnz, n, colors, M, prio_of(0),
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
        const uint32_t sc = gc_stream_value(seed, GC_TAG_COLOR, (uint32_t)r);
        if (G == 8)
            GC_TIMED(GC_K_ASSIGN, s, k_d2_assign<8><<<d2_grid(ctx, tot, 8), D2_BLOCK, 0, s>>>(
                                         g->row_ptr, g->col_idx, g->nnz, n, colors, M, ctx->wl[cur], cnt + cur, sc,
                                         (uint32_t)X, randx));
        else
            GC_TIMED(GC_K_ASSIGN, s, k_d2_assign<64><<<d2_grid(ctx, tot, 64), D2_BLOCK, 0, s>>>(
                                         g->row_ptr, g->col_idx, g->nnz, n, colors, M, ctx->wl[cur], cnt + cur, sc,
                                         (uint32_t)X, randx));
        GC_LAUNCHED();
        const int star = ctx->tune.d2_star;  // the marking kernels stay exact for any row length
        if (star == 1 || (star == 0 && maxdeg <= D2_STAR_ROW && tot > n / 8)) {
            // large round: star marking over every vertex, then commit
            GC_TIMED(GC_K_DETECT, s, k_d2_mark<8><<<d2_grid(ctx, n, 8), D2_BLOCK, 0, s>>>(
                                         g->row_ptr, g->col_idx, g->nnz, n, colors, prio_of(r), lost));
            GC_LAUNCHED();
            GC_TIMED(GC_K_DETECT, s, k_d2_commit<8><<<d2_grid(ctx, tot, 8), D2_BLOCK, 0, s>>>(
                                         g->row_ptr, g->col_idx, g->nnz, n, colors, M, lost, prio_of(r),
                                         ctx->wl[cur], cnt + cur, ctx->wl[nxt], cnt + nxt));
        } else {
            GC_TIMED(GC_K_DETECT, s, k_d2_detect<<<d2_grid(ctx, tot), D2_BLOCK, 0, s>>>(
                                         g->row_ptr, g->col_idx, g->nnz, n, colors, ctx->wl[cur], cnt + cur, M,
                                         prio_of(r), ctx->wl[nxt], cnt + nxt));
        }
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
    int32_t maxdeg = 0;
    gc_status status = gc_graph_max_degree(ctx, g, s, &maxdeg);
    if (status) return status;
    const int G = d2_group(maxdeg);
    status = d2_masks(ctx, g->n, s);
    if (status) return status;
    unsigned long long *M = ctx->d2mask;
    for (int32_t r = 0; r < k; r++) {
        const int32_t a = off_host[seg_per_rank * r], b = off_host[seg_per_rank * r + seg_per_rank];
        if (b <= a) continue;
        if (G == 8)
            GC_TIMED(GC_K_WALK, s, k_d2_class<8><<<d2_grid(ctx, b - a, 8), D2_BLOCK, 0, s>>>(
                                       g->row_ptr, g->col_idx, g->nnz, g->n, C, M, ctx->list, a, b));
        else
            GC_TIMED(GC_K_WALK, s, k_d2_class<64><<<d2_grid(ctx, b - a, 64), D2_BLOCK, 0, s>>>(
                                       g->row_ptr, g->col_idx, g->nnz, g->n, C, M, ctx->list, a, b));
        GC_LAUNCHED();
    }
    return GC_OK;
}

gc_status gc_validate_d2_impl(gc_ctx *ctx, const gc_csr *g, const int32_t *colors, int64_t *conflict_pairs,
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
        // S_CONFLICTS: vertices with a conflict (phase 1), S_UNCOLORED, S_DONE: pairs (phase 2)
        static_assert(S_UNCOLORED == S_CONFLICTS + 1, "adjacent validation slots");
        GC_HIP(hipMemsetAsync(ctx->scal + S_CONFLICTS, 0, 2 * 8, s));
        GC_HIP(hipMemsetAsync(ctx->scal + S_DONE, 0, 8, s));
        int32_t *bad = ctx->wl[0];  // free outside the initial coloring's rounds
        GC_TIMED(GC_K_OTHER, s, k_d2_validate<<<d2_grid(ctx, g->n), D2_BLOCK, 0, s>>>(
                                    g->row_ptr, g->col_idx, g->nnz, g->n, colors, ctx->scal + S_CONFLICTS,
                                    ctx->scal + S_UNCOLORED, bad));
        GC_LAUNCHED();
        status = gc_sync_scalars(ctx, s);
        if (status) return status;
        const int64_t nbad = (int64_t)ctx->hscal[S_CONFLICTS];
        nu = (int64_t)ctx->hscal[S_UNCOLORED];
        if (nbad > 0) {
            GC_TIMED(GC_K_OTHER, s, k_d2_pairs<<<d2_grid(ctx, nbad), D2_BLOCK, 0, s>>>(
                                        g->row_ptr, g->col_idx, g->nnz, g->n, colors, bad, ctx->scal + S_CONFLICTS,
                                        ctx->scal + S_DONE));
            GC_LAUNCHED();
            status = gc_sync_scalars(ctx, s);
            if (status) return status;
            nc = (int64_t)ctx->hscal[S_DONE];
        }
    }
    if (conflict_pairs) *conflict_pairs = nc;
    if (uncolored) *uncolored = nu;
    return GC_OK;
}

// Public entry points: the implementations above, with any sticky device
// failure harvested on the way reported in the returned status.
extern "C" gc_status gc_validate_d2(gc_ctx *ctx, const gc_csr *g, const int32_t *colors, int64_t *conflict_pairs,
                                    int64_t *uncolored, void *stream) {
    return gc_report(ctx, gc_validate_d2_impl(ctx, g, colors, conflict_pairs, uncolored, stream));
}
