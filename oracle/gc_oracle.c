/*
 * gc_oracle.c - plain, single-threaded CPU oracle for speculative distance-1
 * coloring with iterated (Culberson) recoloring, and the square graph that
 * turns distance-2 coloring into distance-1 coloring.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may include, link,
 * load or call this file: only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg use it.  It shares no code, header, table or
 * constant generator with the HIP implementation; both are written from the
 * paper's description and from the published definitions of the two hash
 * mixers named below.
 *
 * Paper: Sariyuce, Saule, Catalyurek, "On Distributed Graph Coloring with
 * Iterative Recoloring" (arXiv 1407.6745).
 *
 * Conventions (the paper's problem statement, section 1): colours are
 * positive integers, 0 means "not coloured", a colouring is proper when no
 * edge joins two equal colours.  Graphs are int32 CSR, symmetric, no
 * self-loops.
 *
 * Each function is a direct transcription of the definition it cites, with no
 * blocking, fusion or reordering.  Where the paper leaves a choice open the
 * reading taken is stated at the function.
 *
 * Parity status: every function is pinned by tests against closed forms,
 * brute force or published values except the exact vertex colours of the
 * speculative initial colouring on general graphs, which have no closed form
 * ("parity unpinned beyond invariants": properness, the Grundy bound, the
 * X = 1 reduction, the K_n / star / edgeless special cases and schedule
 * independence pin it).  The square graph is pinned against shortest-path
 * distances from an independent library; the distance-2 colourings built on it
 * by closed forms (path, star, 27-point mesh), brute force and invariants.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* status codes (same numeric meaning as the library's, defined independently) */
enum { ORC_OK = 0, ORC_ERR_ARG = 1, ORC_ERR_GRAPH = 2, ORC_ERR_COLORING = 3, ORC_ERR_OOM = 4,
       ORC_ERR_NOT_CONVERGED = 6 };
enum { ORC_FIRST_FIT = 0, ORC_RANDOM_X = 1 };
enum { ORC_PERM_REVERSE = 0, ORC_PERM_NONINC = 1, ORC_PERM_NONDEC = 2, ORC_PERM_RANDOM = 3 };
enum { ORC_FLAG_FIXED_PRIORITY = 1, ORC_FLAG_PRIO_LF = 2, ORC_FLAG_PRIO_NATURAL = 4 };
enum { ORC_TAG_PRIO = 1, ORC_TAG_COLOR = 2, ORC_TAG_PERM = 3, ORC_TAG_GRAPH = 4 };

typedef struct {
    int32_t rounds;
    int32_t num_colors;
    int32_t max_color;
    int32_t _pad;
    int64_t losers_total;
} orc_stats;

/* ------------------------------------------------------------------ */
/* Hash: counter-based randomness for priorities, Random-X picks and    */
/* random class permutations.                                           */
/* ------------------------------------------------------------------ */

/* SplitMix64 output function (Steele, Lea, Flood 2014; Stafford's Mix13 constants). */
uint64_t orc_mix64(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

/* MurmurHash3 32-bit finalizer (Appleby); a bijection on uint32. */
uint32_t orc_fmix32(uint32_t h) {
    h ^= h >> 16;
    h *= 0x85EBCA6BU;
    h ^= h >> 13;
    h *= 0xC2B2AE35U;
    h ^= h >> 16;
    return h;
}

#define ORC_GOLDEN 0x9E3779B97F4A7C15ULL

/* One 32-bit value per (seed, tag, counter): high half of mix64(seed + golden * (tag << 32 | counter)). */
uint32_t orc_stream(uint64_t seed, uint32_t tag, uint32_t counter) {
    uint64_t x = seed + ORC_GOLDEN * (((uint64_t)tag << 32) | counter);
    return (uint32_t)(orc_mix64(x) >> 32);
}

/*
 * Priority of v in round r (section 2.2: ties between conflicting vertices
 * are broken by a random total order).  The total order is the 64-bit key
 * (prio << 32 | v); the larger key keeps its colour.  prio is a bijection of
 * v for a fixed round, so keys never tie.
 */
uint32_t orc_prio(uint64_t seed, uint32_t r, uint32_t v) {
    return orc_fmix32(orc_stream(seed, ORC_TAG_PRIO, r) ^ v);
}
uint64_t orc_key(uint64_t seed, uint32_t r, uint32_t v) {
    return ((uint64_t)orc_prio(seed, r, v) << 32) | v;
}

/* Random-X offset j in [0, X) for v in round r (section 3.2): multiply-shift of a 32-bit hash. */
uint32_t orc_pick(uint64_t seed, uint32_t r, uint32_t v, uint32_t X) {
    uint32_t h = orc_fmix32(orc_stream(seed, ORC_TAG_COLOR, r) ^ v);
    return (uint32_t)(((uint64_t)h * X) >> 32);
}

/* Uniform-ish index in [0, m) for swap step i of pass p's Knuth shuffle. */
uint32_t orc_bounded(uint64_t seed, uint32_t p, uint32_t i, uint32_t m) {
    uint32_t h = orc_fmix32(orc_stream(seed, ORC_TAG_PERM, p) ^ i);
    return (uint32_t)(((uint64_t)h * m) >> 32);
}

/* Seed of graph g in a batch. */
uint64_t orc_graph_seed(uint64_t base, uint32_t g) {
    return orc_mix64(base + ORC_GOLDEN * (((uint64_t)ORC_TAG_GRAPH << 32) | g));
}

/* ------------------------------------------------------------------ */
/* Section 2.1, Algorithm 1: sequential greedy colouring.               */
/* ------------------------------------------------------------------ */

/*
 * Visits vertices in `order` (natural order when NULL).  For each v the
 * colours of its neighbours are stamped with v in forbiddenColors, and v
 * takes the smallest i > 0 whose stamp is not v.  Vertices not yet visited
 * have colour 0, which is never a candidate.  Entries of `color` for
 * vertices absent from `order` stay 0.
 */
int orc_greedy_seq(int32_t n, const int32_t *rp, const int32_t *col, const int32_t *order, int32_t *color) {
    if (n < 0) return ORC_ERR_ARG;
    int32_t maxd = 0;
    for (int32_t v = 0; v < n; v++)
        if (rp[v + 1] - rp[v] > maxd) maxd = rp[v + 1] - rp[v];
    int64_t *forbidden = (int64_t *)malloc(((size_t)maxd + 2) * sizeof(int64_t));
    if (!forbidden) return ORC_ERR_OOM;
    for (int32_t i = 0; i < maxd + 2; i++) forbidden[i] = -1;
    for (int32_t v = 0; v < n; v++) color[v] = 0;
    for (int32_t t = 0; t < n; t++) {
        int32_t v = order ? order[t] : t;
        for (int32_t e = rp[v]; e < rp[v + 1]; e++) {
            int32_t c = color[col[e]];
            if (c <= maxd + 1) forbidden[c] = v; /* colours above deg+1 cannot be the minimum */
        }
        int32_t i = 1;
        while (forbidden[i] == v) i++;
        color[v] = i;
    }
    free(forbidden);
    return ORC_OK;
}

/* ------------------------------------------------------------------ */
/* COUNT and VALIDATE (section 1: a colouring maps V to positive        */
/* integers with different colours on the two ends of every edge).      */
/* ------------------------------------------------------------------ */

static int cmp_i32(const void *a, const void *b) {
    int32_t x = *(const int32_t *)a, y = *(const int32_t *)b;
    return (x > y) - (x < y);
}

/* Number of distinct positive colours (independent sets) and the largest colour. */
int orc_count(int32_t n, const int32_t *color, int32_t *num_colors, int32_t *max_color) {
    int32_t *s = (int32_t *)malloc(((size_t)n + 1) * sizeof(int32_t));
    if (!s) return ORC_ERR_OOM;
    memcpy(s, color, (size_t)n * sizeof(int32_t));
    qsort(s, (size_t)n, sizeof(int32_t), cmp_i32);
    int32_t num = 0, mx = 0;
    for (int32_t i = 0; i < n; i++) {
        if (s[i] <= 0) continue;
        if (i == 0 || s[i] != s[i - 1]) num++;
        mx = s[i];
    }
    free(s);
    *num_colors = num;
    *max_color = mx;
    return ORC_OK;
}

/*
 * conflicts = number of adjacency entries (u, w) with u < w and
 * color[u] == color[w] > 0 (each undirected edge once);
 * uncolored = number of v with color[v] <= 0.
 */
int orc_validate(int32_t n, const int32_t *rp, const int32_t *col, const int32_t *color,
                 int64_t *conflicts, int64_t *uncolored) {
    int64_t cf = 0, un = 0;
    for (int32_t u = 0; u < n; u++) {
        if (color[u] <= 0) { un++; continue; }
        for (int32_t e = rp[u]; e < rp[u + 1]; e++) {
            int32_t w = col[e];
            if (u < w && color[w] == color[u]) cf++;
        }
    }
    *conflicts = cf;
    *uncolored = un;
    return ORC_OK;
}

/* CSR precondition check: ids in range, no self-loops, symmetric (with multiplicity). */
int orc_check_csr(int32_t n, const int32_t *rp, const int32_t *col) {
    if (n < 0 || rp[0] != 0) return ORC_ERR_GRAPH;
    for (int32_t v = 0; v < n; v++)
        if (rp[v + 1] < rp[v]) return ORC_ERR_GRAPH;
    for (int32_t v = 0; v < n; v++)
        for (int32_t e = rp[v]; e < rp[v + 1]; e++) {
            int32_t w = col[e];
            if (w < 0 || w >= n || w == v) return ORC_ERR_GRAPH;
            int32_t fwd = 0, back = 0;
            for (int32_t f = rp[v]; f < rp[v + 1]; f++) fwd += col[f] == w;
            for (int32_t f = rp[w]; f < rp[w + 1]; f++) back += col[f] == v;
            if (fwd != back) return ORC_ERR_GRAPH;
        }
    return ORC_OK;
}

/* ------------------------------------------------------------------ */
/* Speculative initial colouring (section 2.2 framework; colour         */
/* selection First Fit of section 2.1 or Random-X Fit of section 3.2).  */
/* ------------------------------------------------------------------ */

/*
 * Conflict key of v in round r (the larger key keeps its colour):
 *   default: orc_key(seed, r, v), a random order redrawn every round
 *            (round 0's order in every round with ORC_FLAG_FIXED_PRIORITY);
 *   ORC_FLAG_PRIO_LF: Largest First (section 2.1's vertex-visit orderings) --
 *            larger degree first, ties by round 0's random order;
 *   ORC_FLAG_PRIO_NATURAL: natural order -- smaller vertex id first.
 */
static uint64_t init_key(uint32_t flags, uint64_t seed, uint32_t r, const int32_t *rp, int32_t v) {
    if (flags & ORC_FLAG_PRIO_LF)
        return ((uint64_t)(uint32_t)(rp[v + 1] - rp[v]) << 32) | orc_prio(seed, 0u, (uint32_t)v);
    if (flags & ORC_FLAG_PRIO_NATURAL) return (uint64_t)(0xFFFFFFFFu - (uint32_t)v);
    return orc_key(seed, (flags & ORC_FLAG_FIXED_PRIORITY) ? 0u : r, (uint32_t)v);
}

/*
 * Rounds: every uncoloured vertex is tentatively coloured from the colours its
 * neighbours held at the start of the round (all vertices of a round read the
 * same snapshot: one superstep covering every uncoloured vertex).  Then each
 * tentatively coloured v that shares its tentative colour with a neighbour w
 * of the same round whose key is larger loses: it becomes uncoloured and joins
 * the next round.  All tentative colours of the round count in that test,
 * including those of vertices that lose themselves.  Winners keep their
 * colours.  Stops when a round leaves no loser.
 *
 * Selection: the (j+1)-th smallest positive colour no neighbour holds, with
 * j = 0 for First Fit and j = orc_pick(seed, r, v, X) for Random-X Fit
 * (uniform among the first X permissible colours).
 *
 * w_sizes[r] = |W_r| and w_degsum[r] = sum of degrees over W_r for the first
 * w_cap rounds (either pointer may be NULL).  commit_round (may be NULL):
 * for every vertex, the round in which it kept its colour, -1 if none.
 */
int orc_init_color_rounds(int32_t n, const int32_t *rp, const int32_t *col, int32_t sel, int32_t X, uint64_t seed,
                          int32_t max_rounds, uint32_t flags, int32_t *C, orc_stats *st,
                          int64_t *w_sizes, int64_t *w_degsum, int32_t w_cap, int32_t *commit_round) {
    if (n < 0 || (sel != ORC_FIRST_FIT && sel != ORC_RANDOM_X) || (sel == ORC_RANDOM_X && X < 1) || max_rounds < 0)
        return ORC_ERR_ARG;
    if ((flags & ORC_FLAG_PRIO_LF) && (flags & ORC_FLAG_PRIO_NATURAL)) return ORC_ERR_ARG;
    if (sel == ORC_FIRST_FIT) X = 1;
    int32_t maxd = 0;
    for (int32_t v = 0; v < n; v++)
        if (rp[v + 1] - rp[v] > maxd) maxd = rp[v + 1] - rp[v];
    int64_t fcap = (int64_t)maxd + X + 2;
    int64_t *forbidden = (int64_t *)malloc((size_t)fcap * sizeof(int64_t));
    int32_t *T = (int32_t *)malloc(((size_t)n + 1) * sizeof(int32_t));
    int32_t *inW = (int32_t *)malloc(((size_t)n + 1) * sizeof(int32_t));
    int32_t *W = (int32_t *)malloc(((size_t)n + 1) * sizeof(int32_t));
    int32_t *L = (int32_t *)malloc(((size_t)n + 1) * sizeof(int32_t));
    uint8_t *lost = (uint8_t *)malloc((size_t)n + 1);
    if (!forbidden || !T || !inW || !W || !L || !lost) {
        free(forbidden); free(T); free(inW); free(W); free(L); free(lost);
        return ORC_ERR_OOM;
    }
    for (int64_t i = 0; i < fcap; i++) forbidden[i] = -1;
    for (int32_t v = 0; v < n; v++) { C[v] = 0; inW[v] = -1; W[v] = v; }
    if (commit_round)
        for (int32_t v = 0; v < n; v++) commit_round[v] = -1;
    int64_t stamp = 0, visited = 0;
    int32_t nW = n, r = 0, status = ORC_OK;
    while (nW > 0) {
        if (max_rounds > 0 && r == max_rounds) { status = ORC_ERR_NOT_CONVERGED; break; }
        int64_t degsum = 0;
        /* tentative colouring from the start-of-round snapshot C (C is not written here) */
        for (int32_t i = 0; i < nW; i++) {
            int32_t v = W[i];
            int32_t d = rp[v + 1] - rp[v];
            degsum += d;
            stamp++;
            for (int32_t e = rp[v]; e < rp[v + 1]; e++) {
                int32_t c = C[col[e]];
                if (c > 0 && (int64_t)c < fcap) forbidden[c] = stamp;
            }
            uint32_t j = (sel == ORC_FIRST_FIT) ? 0u : orc_pick(seed, (uint32_t)r, (uint32_t)v, (uint32_t)X);
            int32_t c = 0;
            uint32_t seen = 0;
            for (c = 1;; c++) {
                if (forbidden[c] == stamp) continue;
                if (seen == j) break;
                seen++;
            }
            T[v] = c;
            inW[v] = r;
        }
        if (w_sizes && r < w_cap) w_sizes[r] = nW;
        if (w_degsum && r < w_cap) w_degsum[r] = degsum;
        visited += nW;
        /* conflict detection against every tentative colour of this round */
        int32_t nL = 0;
        for (int32_t i = 0; i < nW; i++) {
            int32_t v = W[i];
            uint64_t kv = init_key(flags, seed, (uint32_t)r, rp, v);
            lost[i] = 0;
            for (int32_t e = rp[v]; e < rp[v + 1]; e++) {
                int32_t w = col[e];
                if (inW[w] == r && T[w] == T[v] && init_key(flags, seed, (uint32_t)r, rp, w) > kv) { lost[i] = 1; break; }
            }
        }
        /* winners keep their colour, losers form the next round */
        for (int32_t i = 0; i < nW; i++) {
            int32_t v = W[i];
            if (lost[i]) L[nL++] = v;
            else {
                C[v] = T[v];
                if (commit_round) commit_round[v] = r;
            }
        }
        int32_t *tmp = W; W = L; L = tmp;
        nW = nL;
        r++;
    }
    if (st) {
        st->rounds = r;
        st->losers_total = visited - n;
        orc_count(n, C, &st->num_colors, &st->max_color);
    }
    free(forbidden); free(T); free(inW); free(W); free(L); free(lost);
    return status;
}

int orc_init_color(int32_t n, const int32_t *rp, const int32_t *col, int32_t sel, int32_t X, uint64_t seed,
                   int32_t max_rounds, uint32_t flags, int32_t *C, orc_stats *st,
                   int64_t *w_sizes, int64_t *w_degsum, int32_t w_cap) {
    return orc_init_color_rounds(n, rp, col, sel, X, seed, max_rounds, flags, C, st, w_sizes, w_degsum, w_cap, NULL);
}

/* ------------------------------------------------------------------ */
/* Recolouring pass (section 2.1, Culberson's Iterated Greedy; section  */
/* 3, synchronous recolouring RC and the RV / NI / ND / RAND class      */
/* permutations).                                                       */
/* ------------------------------------------------------------------ */

static const int64_t *g_size; /* class sizes seen by the comparators below */

static int cmp_noninc(const void *a, const void *b) {
    int32_t x = *(const int32_t *)a, y = *(const int32_t *)b;
    if (g_size[x] != g_size[y]) return g_size[x] > g_size[y] ? -1 : 1;
    return (x > y) - (x < y);
}
static int cmp_nondec(const void *a, const void *b) {
    int32_t x = *(const int32_t *)a, y = *(const int32_t *)b;
    if (g_size[x] != g_size[y]) return g_size[x] < g_size[y] ? -1 : 1;
    return (x > y) - (x < y);
}

/*
 * The class order pi of one pass over the non-empty colour classes of c_old
 * (ascending colour list K, class sizes size[c]):
 *   RV:   colours in decreasing order;
 *   NI:   non-increasing class size, ties by increasing colour;
 *   ND:   non-decreasing class size, ties by increasing colour;
 *   RAND: Knuth shuffle of K: for i = k-1 down to 1 swap K[i] with
 *         K[orc_bounded(seed, pass, i, i+1)].
 * Writes pi[0..k-1]; returns k.
 */
int32_t orc_class_order(int32_t maxc, const int64_t *size, int32_t perm, uint64_t seed, int32_t pass, int32_t *pi) {
    int32_t k = 0;
    for (int32_t c = 1; c <= maxc; c++)
        if (size[c] > 0) pi[k++] = c;
    if (perm == ORC_PERM_REVERSE) {
        for (int32_t i = 0; i < k / 2; i++) { int32_t t = pi[i]; pi[i] = pi[k - 1 - i]; pi[k - 1 - i] = t; }
    } else if (perm == ORC_PERM_NONINC || perm == ORC_PERM_NONDEC) {
        g_size = size;
        qsort(pi, (size_t)k, sizeof(int32_t), perm == ORC_PERM_NONINC ? cmp_noninc : cmp_nondec);
    } else {
        for (int32_t i = k - 1; i >= 1; i--) {
            uint32_t j = orc_bounded(seed, (uint32_t)pass, (uint32_t)i, (uint32_t)i + 1);
            int32_t t = pi[i]; pi[i] = pi[j]; pi[j] = t;
        }
    }
    return k;
}

/*
 * One recolouring pass.  The classes of c_old are visited in the order pi;
 * every vertex of the current class takes the smallest positive colour not
 * held by a neighbour already recoloured in this pass (First Fit, as in
 * Algorithm 1; neighbours not yet recoloured in this pass hold no colour).
 * Vertices of one class are independent, so their order inside the class
 * does not matter; here they go by increasing id.
 *
 * c_old must be a proper colouring with every colour >= 1 (else
 * ORC_ERR_COLORING).  pi_out (capacity max colour) and k_out may be NULL.
 */
int orc_recolor(int32_t n, const int32_t *rp, const int32_t *col, int32_t perm, uint64_t seed, int32_t pass,
                const int32_t *c_old, int32_t *c_new, int32_t *pi_out, int32_t *k_out, orc_stats *st) {
    if (n < 0 || perm < 0 || perm > 3) return ORC_ERR_ARG;
    int32_t maxc = 0;
    for (int32_t v = 0; v < n; v++) {
        if (c_old[v] <= 0) return ORC_ERR_COLORING;
        if (c_old[v] > maxc) maxc = c_old[v];
    }
    int64_t conflicts = 0, unc = 0;
    orc_validate(n, rp, col, c_old, &conflicts, &unc);
    if (conflicts) return ORC_ERR_COLORING;
    int64_t *size = (int64_t *)calloc((size_t)maxc + 1, sizeof(int64_t));
    int32_t *pi = (int32_t *)malloc(((size_t)maxc + 1) * sizeof(int32_t));
    int32_t *rank = (int32_t *)malloc(((size_t)maxc + 1) * sizeof(int32_t));
    int32_t *order = (int32_t *)malloc(((size_t)n + 1) * sizeof(int32_t));
    int64_t *start = (int64_t *)calloc((size_t)maxc + 2, sizeof(int64_t));
    if (!size || !pi || !rank || !order || !start) {
        free(size); free(pi); free(rank); free(order); free(start);
        return ORC_ERR_OOM;
    }
    for (int32_t v = 0; v < n; v++) size[c_old[v]]++;
    int32_t k = orc_class_order(maxc, size, perm, seed, pass, pi);
    for (int32_t s = 0; s < k; s++) rank[pi[s]] = s;
    /* vertices grouped by the rank of their old class, increasing id inside a class */
    for (int32_t s = 0; s < k; s++) start[s + 1] = start[s] + size[pi[s]];
    for (int32_t v = 0; v < n; v++) order[start[rank[c_old[v]]]++] = v;
    /* Algorithm 1 over that order: neighbours outside the visited prefix hold 0 */
    int rc = orc_greedy_seq(n, rp, col, order, c_new);
    if (pi_out) memcpy(pi_out, pi, (size_t)k * sizeof(int32_t));
    if (k_out) *k_out = k;
    if (st) {
        st->rounds = 0;
        st->losers_total = 0;
        orc_count(n, c_new, &st->num_colors, &st->max_color);
    }
    free(size); free(pi); free(rank); free(order); free(start);
    return rc;
}

/*
 * Asynchronous recolouring aRC (section 3): the vertex-visit order taken from
 * the previous colouring (classes in the order pi) drives a second
 * speculative parallel colouring with conflict-resolution rounds.  Reading
 * for one device and Jacobi rounds: the visit order acts as the conflict
 * priority, i.e. of two neighbours with the same tentative colour the one
 * whose old class comes earlier in pi keeps it (two neighbours always have
 * different old classes, so this decides every conflict).  Every round,
 * each vertex still uncoloured takes First Fit over the colours committed
 * before the round; winners commit, losers go to the next round.
 *
 * c_old as for orc_recolor.  rounds_out (may be NULL) receives the rounds.
 */
int orc_arc_recolor(int32_t n, const int32_t *rp, const int32_t *col, int32_t perm, uint64_t seed, int32_t pass,
                    const int32_t *c_old, int32_t *c_new, int32_t *rounds_out, orc_stats *st) {
    if (n < 0 || perm < 0 || perm > 3) return ORC_ERR_ARG;
    int32_t maxc = 0;
    for (int32_t v = 0; v < n; v++) {
        if (c_old[v] <= 0) return ORC_ERR_COLORING;
        if (c_old[v] > maxc) maxc = c_old[v];
    }
    int64_t conflicts = 0, unc = 0;
    orc_validate(n, rp, col, c_old, &conflicts, &unc);
    if (conflicts) return ORC_ERR_COLORING;
    int32_t maxd = 0;
    for (int32_t v = 0; v < n; v++)
        if (rp[v + 1] - rp[v] > maxd) maxd = rp[v + 1] - rp[v];
    int64_t *size = (int64_t *)calloc((size_t)maxc + 1, sizeof(int64_t));
    int32_t *pi = (int32_t *)malloc(((size_t)maxc + 1) * sizeof(int32_t));
    int32_t *rank = (int32_t *)malloc(((size_t)maxc + 1) * sizeof(int32_t));
    int32_t *T = (int32_t *)malloc(((size_t)n + 1) * sizeof(int32_t));
    int32_t *W = (int32_t *)malloc(((size_t)n + 1) * sizeof(int32_t));
    int32_t *L = (int32_t *)malloc(((size_t)n + 1) * sizeof(int32_t));
    int32_t *round_of = (int32_t *)malloc(((size_t)n + 1) * sizeof(int32_t));
    int64_t *forbidden = (int64_t *)malloc(((size_t)maxd + 2) * sizeof(int64_t));
    uint8_t *lost = (uint8_t *)malloc((size_t)n + 1);
    if (!size || !pi || !rank || !T || !W || !L || !round_of || !forbidden || !lost) {
        free(size); free(pi); free(rank); free(T); free(W); free(L); free(round_of); free(forbidden); free(lost);
        return ORC_ERR_OOM;
    }
    for (int32_t v = 0; v < n; v++) size[c_old[v]]++;
    int32_t k = orc_class_order(maxc, size, perm, seed, pass, pi);
    for (int32_t s = 0; s < k; s++) rank[pi[s]] = s;
    for (int32_t i = 0; i < maxd + 2; i++) forbidden[i] = -1;
    for (int32_t v = 0; v < n; v++) { c_new[v] = 0; W[v] = v; round_of[v] = -1; }
    int32_t nW = n, r = 0;
    int64_t stamp = 0;
    while (nW > 0) {
        /* First Fit from the colours committed before the round */
        for (int32_t i = 0; i < nW; i++) {
            int32_t v = W[i];
            stamp++;
            for (int32_t e = rp[v]; e < rp[v + 1]; e++) {
                int32_t c = c_new[col[e]];
                if (c > 0 && c <= maxd + 1) forbidden[c] = stamp;
            }
            int32_t c = 1;
            while (forbidden[c] == stamp) c++;
            T[v] = c;
            round_of[v] = r;
        }
        /* v loses to a neighbour of this round with the same colour and an earlier old class */
        int32_t nL = 0;
        for (int32_t i = 0; i < nW; i++) {
            int32_t v = W[i];
            lost[i] = 0;
            for (int32_t e = rp[v]; e < rp[v + 1]; e++) {
                int32_t w = col[e];
                if (round_of[w] == r && T[w] == T[v] && rank[c_old[w]] < rank[c_old[v]]) { lost[i] = 1; break; }
            }
        }
        for (int32_t i = 0; i < nW; i++) {
            int32_t v = W[i];
            if (lost[i]) L[nL++] = v;
            else c_new[v] = T[v];
        }
        int32_t *tmp = W; W = L; L = tmp;
        nW = nL;
        r++;
    }
    if (rounds_out) *rounds_out = r;
    if (st) {
        st->rounds = r;
        st->losers_total = 0;
        orc_count(n, c_new, &st->num_colors, &st->max_color);
    }
    free(size); free(pi); free(rank); free(T); free(W); free(L); free(round_of); free(forbidden); free(lost);
    return ORC_OK;
}

/*
 * Hybrid class-order schedules (section 4.2.1): iteration t counts from 1.
 *   kind 0: the fixed permutation `base` at every iteration;
 *   kind 1 (ND-RAND%x): RAND when t is a multiple of x, ND otherwise;
 *   kind 2 (ND-RAND%2^i): RAND at t = 2, 4, 8, 16, ..., ND otherwise.
 */
int32_t orc_schedule_perm(int32_t kind, int32_t base, int32_t x, int32_t t) {
    if (kind == 1) return (x > 0 && t % x == 0) ? ORC_PERM_RANDOM : ORC_PERM_NONDEC;
    if (kind == 2) return (t >= 2 && (t & (t - 1)) == 0) ? ORC_PERM_RANDOM : ORC_PERM_NONDEC;
    return base;
}

/* ------------------------------------------------------------------ */
/* Brute force on tiny graphs (test pins).                              */
/* ------------------------------------------------------------------ */

static int bt_color(int32_t v, int32_t n, const int32_t *rp, const int32_t *col, int32_t k, int32_t *c) {
    if (v == n) return 1;
    /* symmetry breaking: v may use at most one colour above the largest used so far */
    int32_t used = 0;
    for (int32_t u = 0; u < v; u++) if (c[u] > used) used = c[u];
    int32_t lim = used + 1 < k ? used + 1 : k;
    for (int32_t x = 1; x <= lim; x++) {
        int ok = 1;
        for (int32_t e = rp[v]; e < rp[v + 1]; e++)
            if (col[e] >= 0 && col[e] < v && c[col[e]] == x) { ok = 0; break; }
        if (!ok) continue;
        c[v] = x;
        if (bt_color(v + 1, n, rp, col, k, c)) return 1;
    }
    c[v] = 0;
    return 0;
}

/* Chromatic number by exhaustive backtracking (n <= 20 or so); -1 on error. */
int32_t orc_chromatic(int32_t n, const int32_t *rp, const int32_t *col) {
    if (n <= 0) return 0;
    int32_t *c = (int32_t *)calloc((size_t)n, sizeof(int32_t));
    if (!c) return -1;
    int32_t k;
    for (k = 1; k <= n; k++) {
        memset(c, 0, (size_t)n * sizeof(int32_t));
        if (bt_color(0, n, rp, col, k, c)) break;
    }
    free(c);
    return k;
}

/* ------------------------------------------------------------------ */
/* Distance-2 colouring (section 1: the distance-k problem asks that    */
/* vertices joined by a path of at most k edges get different colours; */
/* the paper expects its techniques to carry over to such variants).    */
/* ------------------------------------------------------------------ */

/*
 * The square G^2 of G: u and w (u != w) are adjacent in G^2 iff G joins them
 * by a path of one or two edges.  A distance-2 colouring of G is by
 * definition a distance-1 colouring of G^2, so the distance-2 initial
 * colouring, recolouring and validation are the distance-1 routines above
 * applied to G^2 (the binding composes them).
 *
 * orc_square_count fills rp2[0..n] (rows of G^2, each sorted and free of
 * duplicates) and returns nnz(G^2), or -1 when it exceeds int32 or memory
 * runs out; orc_square_fill then writes col2[0..nnz(G^2)).
 */
static int64_t square_rows(int32_t n, const int32_t *rp, const int32_t *col, int32_t *rp2, int32_t *col2) {
    int32_t *mark = (int32_t *)malloc(((size_t)n + 1) * sizeof(int32_t));
    int32_t *row = (int32_t *)malloc(((size_t)n + 1) * sizeof(int32_t));
    if (!mark || !row) { free(mark); free(row); return -1; }
    for (int32_t v = 0; v < n; v++) mark[v] = -1;
    int64_t total = 0;
    if (rp2) rp2[0] = 0;
    for (int32_t v = 0; v < n; v++) {
        int32_t len = 0;
        mark[v] = v; /* v itself is not its own neighbour */
        for (int32_t e = rp[v]; e < rp[v + 1]; e++) {
            int32_t u = col[e];
            if (mark[u] != v) { mark[u] = v; row[len++] = u; }
            for (int32_t f = rp[u]; f < rp[u + 1]; f++) {
                int32_t w = col[f];
                if (mark[w] != v) { mark[w] = v; row[len++] = w; }
            }
        }
        if (col2) {
            qsort(row, (size_t)len, sizeof(int32_t), cmp_i32);
            memcpy(col2 + total, row, (size_t)len * sizeof(int32_t));
        }
        total += len;
        if (total > INT32_MAX) { free(mark); free(row); return -1; }
        if (rp2) rp2[v + 1] = (int32_t)total;
    }
    free(mark);
    free(row);
    return total;
}

int64_t orc_square_count(int32_t n, const int32_t *rp, const int32_t *col, int32_t *rp2) {
    if (n < 0) return -1;
    return square_rows(n, rp, col, rp2, NULL);
}

int orc_square_fill(int32_t n, const int32_t *rp, const int32_t *col, int32_t *col2) {
    if (n < 0) return ORC_ERR_ARG;
    return square_rows(n, rp, col, NULL, col2) < 0 ? ORC_ERR_OOM : ORC_OK;
}
