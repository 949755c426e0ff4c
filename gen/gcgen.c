/*
 * gcgen.c - seeded synthetic graph generators (host, C, OpenMP).
 *
 * Input construction only: this file holds none of the coloring method's
 * arithmetic.  Every generator is a pure function of its parameters and seed
 * (thread count never changes the output: rows are sorted and de-duplicated
 * after construction).  Output is an int32 CSR (row_ptr[n+1], col[nnz]) that
 * is symmetric, has no self-loops and no duplicate entries, with each row
 * sorted ascending.
 *
 * Random numbers come from a counter-based SplitMix64 stream
 * (Steele, Lea, Flood, "Fast splittable pseudorandom number generators",
 * OOPSLA 2014): value(i) = mix64(base + GOLDEN * (i + 1)), where base is
 * derived from the seed and a per-family tag.  The generator never uses the
 * C library's RNG or any implementation-defined distribution.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <math.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define GEN_GOLDEN 0x9E3779B97F4A7C15ULL
#define GEN_TAG 5ULL /* generator tag: keeps these streams apart from any other use of the seed */

enum { FAM_ER = 1, FAM_RMAT = 2, FAM_RGG = 3, FAM_RGG_BATCH = 4, FAM_POOL = 5 };

static inline uint64_t g_mix64(uint64_t z) {
    z ^= z >> 30; z *= 0xBF58476D1CE4E5B9ULL;
    z ^= z >> 27; z *= 0x94D049BB133111EBULL;
    z ^= z >> 31;
    return z;
}
static inline uint64_t g_base(uint64_t seed, uint64_t family, uint64_t sub) {
    return g_mix64(seed + GEN_GOLDEN * ((GEN_TAG << 32) | family)) ^ g_mix64(sub + GEN_GOLDEN);
}
static inline uint64_t g_val(uint64_t base, uint64_t i) { return g_mix64(base + GEN_GOLDEN * (i + 1)); }
/* uniform integer in [0, m) by multiply-shift of a 32-bit value (m < 2^32) */
static inline uint32_t g_below(uint32_t r, uint32_t m) { return (uint32_t)(((uint64_t)r * m) >> 32); }

typedef struct {
    int64_t n;
    int64_t nnz;
    int32_t *row_ptr; /* n + 1 */
    int32_t *col;     /* nnz */
    int32_t max_deg;
    int32_t status;   /* 0 ok, 1 out of memory, 2 too large for int32 CSR */
} gen_graph;

static gen_graph *g_alloc(void) { return (gen_graph *)calloc(1, sizeof(gen_graph)); }

void gen_free(gen_graph *g) {
    if (!g) return;
    free(g->row_ptr);
    free(g->col);
    free(g);
}

static int cmp_i32(const void *a, const void *b) {
    int32_t x = *(const int32_t *)a, y = *(const int32_t *)b;
    return (x > y) - (x < y);
}

static void sort_row(int32_t *a, int64_t len) {
    if (len < 32) {
        for (int64_t i = 1; i < len; i++) {
            int32_t x = a[i];
            int64_t j = i - 1;
            while (j >= 0 && a[j] > x) { a[j + 1] = a[j]; j--; }
            a[j + 1] = x;
        }
    } else {
        qsort(a, (size_t)len, sizeof(int32_t), cmp_i32);
    }
}

/*
 * Build a symmetric CSR from undirected pairs (u[i], v[i]).  Self-loops are
 * dropped, both directions are inserted, each row is sorted and duplicates
 * removed.  Frees nothing it was given.
 */
static gen_graph *csr_from_pairs(int64_t n, int64_t np, const int32_t *u, const int32_t *v) {
    gen_graph *g = g_alloc();
    if (!g) return NULL;
    g->n = n;
    int64_t *deg = (int64_t *)calloc((size_t)n + 1, sizeof(int64_t));
    if (!deg) { g->status = 1; return g; }
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < np; i++) {
        if (u[i] == v[i]) continue;
#pragma omp atomic
        deg[u[i]]++;
#pragma omp atomic
        deg[v[i]]++;
    }
    int64_t *start = (int64_t *)malloc(((size_t)n + 1) * sizeof(int64_t));
    if (!start) { free(deg); g->status = 1; return g; }
    start[0] = 0;
    for (int64_t i = 0; i < n; i++) start[i + 1] = start[i] + deg[i];
    int64_t total = start[n];
    int32_t *tmp = (int32_t *)malloc((size_t)(total > 0 ? total : 1) * sizeof(int32_t));
    int64_t *fill = (int64_t *)malloc(((size_t)n + 1) * sizeof(int64_t));
    if (!tmp || !fill) { free(deg); free(start); free(tmp); free(fill); g->status = 1; return g; }
    memcpy(fill, start, ((size_t)n + 1) * sizeof(int64_t));
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < np; i++) {
        if (u[i] == v[i]) continue;
        int64_t pu, pv;
#pragma omp atomic capture
        pu = fill[u[i]]++;
#pragma omp atomic capture
        pv = fill[v[i]]++;
        tmp[pu] = v[i];
        tmp[pv] = u[i];
    }
    free(fill);
    /* sort + dedup each row in place; new degree into deg[] */
#pragma omp parallel for schedule(dynamic, 1024)
    for (int64_t r = 0; r < n; r++) {
        int32_t *a = tmp + start[r];
        int64_t len = start[r + 1] - start[r];
        sort_row(a, len);
        int64_t w = 0;
        for (int64_t i = 0; i < len; i++)
            if (w == 0 || a[i] != a[w - 1]) a[w++] = a[i];
        deg[r] = w;
    }
    int64_t nnz = 0;
    for (int64_t r = 0; r < n; r++) nnz += deg[r];
    if (nnz >= 2147483647LL) { free(deg); free(start); free(tmp); g->status = 2; return g; }
    g->row_ptr = (int32_t *)malloc(((size_t)n + 1) * sizeof(int32_t));
    g->col = (int32_t *)malloc((size_t)(nnz > 0 ? nnz : 1) * sizeof(int32_t));
    if (!g->row_ptr || !g->col) { free(deg); free(start); free(tmp); g->status = 1; return g; }
    int64_t acc = 0;
    int32_t md = 0;
    for (int64_t r = 0; r < n; r++) {
        g->row_ptr[r] = (int32_t)acc;
        acc += deg[r];
        if (deg[r] > md) md = (int32_t)deg[r];
    }
    g->row_ptr[n] = (int32_t)acc;
#pragma omp parallel for schedule(dynamic, 4096)
    for (int64_t r = 0; r < n; r++)
        memcpy(g->col + g->row_ptr[r], tmp + start[r], (size_t)deg[r] * sizeof(int32_t));
    g->nnz = nnz;
    g->max_deg = md;
    free(deg); free(start); free(tmp);
    return g;
}

/* Build from arbitrary (possibly duplicated / self-loop) undirected pairs given by the caller. */
gen_graph *gen_from_pairs(int64_t n, int64_t np, const int32_t *u, const int32_t *v) {
    for (int64_t i = 0; i < np; i++)
        if (u[i] < 0 || u[i] >= n || v[i] < 0 || v[i] >= n) {
            gen_graph *g = g_alloc();
            if (g) { g->n = n; g->status = 3; }
            return g;
        }
    return csr_from_pairs(n, np, u, v);
}

/*
 * 3D 27-point stencil on an N x N x N box: id = x + N*(y + N*z); v is adjacent
 * to every in-bounds w with max(|dx|,|dy|,|dz|) = 1.  Rows come out sorted.
 * nnz = (3N-2)^3 - N^3.
 */
gen_graph *gen_mesh27(int32_t N) {
    gen_graph *g = g_alloc();
    if (!g) return NULL;
    int64_t n = (int64_t)N * N * N;
    int64_t t = 3LL * N - 2;
    int64_t nnz = N > 0 ? t * t * t - n : 0;
    g->n = n;
    if (nnz >= 2147483647LL) { g->status = 2; return g; }
    g->row_ptr = (int32_t *)malloc(((size_t)n + 1) * sizeof(int32_t));
    g->col = (int32_t *)malloc((size_t)(nnz > 0 ? nnz : 1) * sizeof(int32_t));
    if (!g->row_ptr || !g->col) { g->status = 1; return g; }
    /* row lengths are known per vertex: product of per-axis neighbour counts minus 1 */
    g->row_ptr[0] = 0;
    for (int64_t id = 0; id < n; id++) {
        int32_t x = (int32_t)(id % N), y = (int32_t)((id / N) % N), z = (int32_t)(id / ((int64_t)N * N));
        int32_t cx = 1 + (x > 0) + (x < N - 1), cy = 1 + (y > 0) + (y < N - 1), cz = 1 + (z > 0) + (z < N - 1);
        g->row_ptr[id + 1] = g->row_ptr[id] + cx * cy * cz - 1;
    }
#pragma omp parallel for schedule(static)
    for (int64_t id = 0; id < n; id++) {
        int32_t x = (int32_t)(id % N), y = (int32_t)((id / N) % N), z = (int32_t)(id / ((int64_t)N * N));
        int32_t *o = g->col + g->row_ptr[id];
        for (int dz = -1; dz <= 1; dz++)
            for (int dy = -1; dy <= 1; dy++)
                for (int dx = -1; dx <= 1; dx++) {
                    if (!dx && !dy && !dz) continue;
                    int32_t X = x + dx, Y = y + dy, Z = z + dz;
                    if (X < 0 || Y < 0 || Z < 0 || X >= N || Y >= N || Z >= N) continue;
                    *o++ = (int32_t)(X + (int64_t)N * (Y + (int64_t)N * Z));
                }
    }
    g->nnz = nnz;
    g->max_deg = n > 1 ? (int32_t)((N >= 3 ? 27 : (N == 2 ? 8 : 1)) - 1) : 0;
    return g;
}

/* 2D 5-point grid on Nx x Ny: id = x + Nx*y; nnz = 4*Nx*Ny - 2*Nx - 2*Ny. */
gen_graph *gen_grid5(int32_t Nx, int32_t Ny) {
    gen_graph *g = g_alloc();
    if (!g) return NULL;
    int64_t n = (int64_t)Nx * Ny;
    int64_t nnz = n > 0 ? 4 * n - 2LL * Nx - 2LL * Ny : 0;
    g->n = n;
    if (nnz >= 2147483647LL) { g->status = 2; return g; }
    g->row_ptr = (int32_t *)malloc(((size_t)n + 1) * sizeof(int32_t));
    g->col = (int32_t *)malloc((size_t)(nnz > 0 ? nnz : 1) * sizeof(int32_t));
    if (!g->row_ptr || !g->col) { g->status = 1; return g; }
    g->row_ptr[0] = 0;
    for (int64_t id = 0; id < n; id++) {
        int32_t x = (int32_t)(id % Nx), y = (int32_t)(id / Nx);
        g->row_ptr[id + 1] = g->row_ptr[id] + (y > 0) + (x > 0) + (x < Nx - 1) + (y < Ny - 1);
    }
#pragma omp parallel for schedule(static)
    for (int64_t id = 0; id < n; id++) {
        int32_t x = (int32_t)(id % Nx), y = (int32_t)(id / Nx);
        int32_t *o = g->col + g->row_ptr[id];
        if (y > 0) *o++ = (int32_t)(id - Nx);
        if (x > 0) *o++ = (int32_t)(id - 1);
        if (x < Nx - 1) *o++ = (int32_t)(id + 1);
        if (y < Ny - 1) *o++ = (int32_t)(id + Nx);
    }
    g->nnz = nnz;
    int32_t md = 0;
    for (int64_t id = 0; id < n; id++) {
        int32_t d = g->row_ptr[id + 1] - g->row_ptr[id];
        if (d > md) md = d;
    }
    g->max_deg = md;
    return g;
}

/*
 * Erdos-Renyi G(n, m): the first m distinct unordered pairs {u, v}, u != v,
 * drawn in counter order from the seeded stream (each candidate takes the two
 * 32-bit halves of one 64-bit value, mapped to [0, n) by multiply-shift).
 */
gen_graph *gen_er(int64_t n, int64_t m, uint64_t seed) {
    if (n < 2 || n > 2147483647LL || m < 0 || m > n * (n - 1) / 2) {
        gen_graph *g = g_alloc();
        if (g) { g->n = n; g->status = (n < 2 && m == 0) ? 0 : 3; }
        if (g && g->status == 0) {
            g->row_ptr = (int32_t *)calloc((size_t)(n > 0 ? n : 0) + 1, sizeof(int32_t));
            g->col = (int32_t *)malloc(sizeof(int32_t));
        }
        return g;
    }
    uint64_t cap = 16;
    while (cap < (uint64_t)m * 2 + 16) cap <<= 1;
    uint64_t *tab = (uint64_t *)malloc(cap * sizeof(uint64_t));
    int32_t *u = (int32_t *)malloc((size_t)(m > 0 ? m : 1) * sizeof(int32_t));
    int32_t *v = (int32_t *)malloc((size_t)(m > 0 ? m : 1) * sizeof(int32_t));
    if (!tab || !u || !v) { free(tab); free(u); free(v); gen_graph *g = g_alloc(); if (g) g->status = 1; return g; }
    memset(tab, 0xff, cap * sizeof(uint64_t));
    uint64_t base = g_base(seed, FAM_ER, (uint64_t)n);
    int64_t got = 0;
    for (uint64_t i = 0; got < m; i++) {
        uint64_t h = g_val(base, i);
        uint32_t a = g_below((uint32_t)h, (uint32_t)n), b = g_below((uint32_t)(h >> 32), (uint32_t)n);
        if (a == b) continue;
        if (a > b) { uint32_t t = a; a = b; b = t; }
        uint64_t key = ((uint64_t)a << 32) | b;
        uint64_t slot = g_mix64(key) & (cap - 1);
        int dup = 0;
        while (tab[slot] != ~0ULL) {
            if (tab[slot] == key) { dup = 1; break; }
            slot = (slot + 1) & (cap - 1);
        }
        if (dup) continue;
        tab[slot] = key;
        u[got] = (int32_t)a;
        v[got] = (int32_t)b;
        got++;
    }
    free(tab);
    gen_graph *g = csr_from_pairs(n, m, u, v);
    free(u); free(v);
    return g;
}

/*
 * Graph500-style RMAT: ef * 2^scale tuples; for each tuple and each of the
 * `scale` levels (most significant bit first) one 32-bit value picks a
 * quadrant by comparison with the integer thresholds t1 < t2 < t3
 * (floor(a*2^32), floor((a+b)*2^32), floor((a+b+c)*2^32)):
 *   r < t1 -> (0,0), r < t2 -> (0,1), r < t3 -> (1,0), else (1,1).
 * No noise and no vertex relabeling.  Self-loops and duplicates are dropped
 * and the result symmetrised; isolated vertices stay in n = 2^scale.
 */
gen_graph *gen_rmat(int32_t scale, int32_t ef, double a, double b, double c, uint64_t seed) {
    if (scale < 1 || scale > 30 || ef < 1) { gen_graph *g = g_alloc(); if (g) g->status = 3; return g; }
    int64_t n = 1LL << scale;
    int64_t nt = n * ef;
    uint32_t t1 = (uint32_t)floor(a * 4294967296.0);
    uint32_t t2 = (uint32_t)floor((a + b) * 4294967296.0);
    uint32_t t3 = (uint32_t)floor((a + b + c) * 4294967296.0);
    int32_t *u = (int32_t *)malloc((size_t)nt * sizeof(int32_t));
    int32_t *v = (int32_t *)malloc((size_t)nt * sizeof(int32_t));
    if (!u || !v) { free(u); free(v); gen_graph *g = g_alloc(); if (g) g->status = 1; return g; }
    uint64_t base = g_base(seed, FAM_RMAT, ((uint64_t)scale << 32) | (uint32_t)ef);
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < nt; i++) {
        uint32_t uu = 0, vv = 0;
        for (int32_t l = 0; l < scale; l += 2) {
            uint64_t h = g_val(base, (uint64_t)i * 16 + (uint64_t)(l >> 1));
            for (int32_t k = 0; k < 2 && l + k < scale; k++) {
                uint32_t r = k ? (uint32_t)(h >> 32) : (uint32_t)h;
                uint32_t ub = r >= t2, vb = (r >= t1 && r < t2) || r >= t3;
                uu = (uu << 1) | ub;
                vv = (vv << 1) | vb;
            }
        }
        u[i] = (int32_t)uu;
        v[i] = (int32_t)vv;
    }
    gen_graph *g = csr_from_pairs(n, nt, u, v);
    free(u); free(v);
    return g;
}

/* ---------------- random geometric graphs ---------------- */

#define RGG_BITS 20
#define RGG_SIDE (1 << RGG_BITS)

/* r_int = floor(r * 2^20); u ~ v iff dx^2 + dy^2 <= r_int^2 on integer coordinates in [0, 2^20)^2, no wrap. */
static void rgg_points(uint64_t base, int64_t n, int32_t *px, int32_t *py) {
    for (int64_t i = 0; i < n; i++) {
        uint64_t h = g_val(base, (uint64_t)i);
        px[i] = (int32_t)((uint32_t)h >> (32 - RGG_BITS));
        py[i] = (int32_t)((uint32_t)(h >> 32) >> (32 - RGG_BITS));
    }
}

/*
 * Bucket points in a grid of cells of side >= r_int; calls emit(u, v) for each
 * ordered pair u != v in range.  When deg != NULL only counts degrees; when
 * out != NULL writes each row (already positioned by rp) sorted ascending.
 */
static int rgg_scan(int64_t n, const int32_t *px, const int32_t *py, int64_t rint,
                    int64_t *deg, const int64_t *rp, int32_t *out) {
    int64_t cell = rint > 0 ? rint : 1;
    int64_t gs = RGG_SIDE / cell; /* floor, so that the cell side below is >= rint */
    if (gs < 1) gs = 1;
    if (gs > 4096) gs = 4096;
    int64_t csz = (RGG_SIDE + gs - 1) / gs; /* >= RGG_SIDE / gs >= rint */
    int64_t ncell = gs * gs;
    int64_t *cstart = (int64_t *)calloc((size_t)ncell + 1, sizeof(int64_t));
    int32_t *ord = (int32_t *)malloc((size_t)(n > 0 ? n : 1) * sizeof(int32_t));
    if (!cstart || !ord) { free(cstart); free(ord); return 1; }
    for (int64_t i = 0; i < n; i++) cstart[(py[i] / csz) * gs + px[i] / csz + 1]++;
    for (int64_t c = 0; c < ncell; c++) cstart[c + 1] += cstart[c];
    int64_t *cf = (int64_t *)malloc((size_t)ncell * sizeof(int64_t));
    if (!cf) { free(cstart); free(ord); return 1; }
    memcpy(cf, cstart, (size_t)ncell * sizeof(int64_t));
    for (int64_t i = 0; i < n; i++) ord[cf[(py[i] / csz) * gs + px[i] / csz]++] = (int32_t)i;
    free(cf);
    int64_t r2 = rint * rint;
    for (int64_t i = 0; i < n; i++) {
        int64_t cx = px[i] / csz, cy = py[i] / csz;
        int64_t cnt = 0;
        int32_t *o = out ? out + rp[i] : NULL;
        for (int64_t yy = cy - 1; yy <= cy + 1; yy++) {
            if (yy < 0 || yy >= gs) continue;
            for (int64_t xx = cx - 1; xx <= cx + 1; xx++) {
                if (xx < 0 || xx >= gs) continue;
                int64_t c = yy * gs + xx;
                for (int64_t q = cstart[c]; q < cstart[c + 1]; q++) {
                    int32_t j = ord[q];
                    if (j == i) continue;
                    int64_t dx = px[i] - px[j], dy = py[i] - py[j];
                    if (dx * dx + dy * dy <= r2) {
                        if (o) o[cnt] = j;
                        cnt++;
                    }
                }
            }
        }
        if (deg) deg[i] = cnt;
        if (o) sort_row(o, cnt);
    }
    free(cstart);
    free(ord);
    return 0;
}

/* Single random geometric graph with n points and radius r (unit square). */
gen_graph *gen_rgg(int64_t n, double r, uint64_t seed) {
    gen_graph *g = g_alloc();
    if (!g) return NULL;
    g->n = n;
    if (n < 0 || n > 2147483647LL) { g->status = 3; return g; }
    int32_t *px = (int32_t *)malloc((size_t)(n > 0 ? n : 1) * sizeof(int32_t));
    int32_t *py = (int32_t *)malloc((size_t)(n > 0 ? n : 1) * sizeof(int32_t));
    int64_t *deg = (int64_t *)malloc((size_t)(n > 0 ? n : 1) * sizeof(int64_t));
    int64_t *rp = (int64_t *)malloc(((size_t)n + 1) * sizeof(int64_t));
    if (!px || !py || !deg || !rp) { free(px); free(py); free(deg); free(rp); g->status = 1; return g; }
    int64_t rint = (int64_t)floor(r * (double)RGG_SIDE);
    rgg_points(g_base(seed, FAM_RGG, (uint64_t)n), n, px, py);
    if (rgg_scan(n, px, py, rint, deg, NULL, NULL)) { g->status = 1; goto done; }
    rp[0] = 0;
    for (int64_t i = 0; i < n; i++) rp[i + 1] = rp[i] + deg[i];
    if (rp[n] >= 2147483647LL) { g->status = 2; goto done; }
    g->row_ptr = (int32_t *)malloc(((size_t)n + 1) * sizeof(int32_t));
    g->col = (int32_t *)malloc((size_t)(rp[n] > 0 ? rp[n] : 1) * sizeof(int32_t));
    if (!g->row_ptr || !g->col) { g->status = 1; goto done; }
    if (rgg_scan(n, px, py, rint, NULL, rp, g->col)) { g->status = 1; goto done; }
    int32_t md = 0;
    for (int64_t i = 0; i <= n; i++) g->row_ptr[i] = (int32_t)rp[i];
    for (int64_t i = 0; i < n; i++) if (deg[i] > md) md = (int32_t)deg[i];
    g->nnz = rp[n];
    g->max_deg = md;
done:
    free(px); free(py); free(deg); free(rp);
    return g;
}

/*
 * Batch of G random geometric graphs.  Graph g: n_g uniform integer in
 * [n_lo, n_hi], target average degree d_g uniform real in [d_lo, d_hi],
 * radius r_g = sqrt(d_g / (pi * n_g)) (no wrap, so border vertices have
 * fewer neighbours).  Parameters come from the seeded stream; point sets
 * from per-graph sub-streams, so graph g does not depend on G.
 */
void gen_rgg_batch_params(int32_t G, uint64_t seed, int32_t n_lo, int32_t n_hi, double d_lo, double d_hi,
                          int64_t *n_out, double *r_out) {
    uint64_t base = g_base(seed, FAM_RGG_BATCH, 0);
    for (int32_t gi = 0; gi < G; gi++) {
        uint64_t h = g_val(base, (uint64_t)gi);
        int64_t n = n_lo + (int64_t)g_below((uint32_t)h, (uint32_t)(n_hi - n_lo + 1));
        double d = d_lo + (d_hi - d_lo) * ((double)(uint32_t)(h >> 32) / 4294967296.0);
        n_out[gi] = n;
        r_out[gi] = sqrt(d / (M_PI * (double)n));
    }
}

/*
 * Packed batch CSR.  Pass 1 (out_col == NULL): writes per-graph nnz into
 * nnz_out[G].  Pass 2: with vtx_off / edge_off (int64, G+1 each, from the
 * caller's prefix sums of n_g and nnz_g) fills the local int32 row_ptr of graph
 * g (n_g + 1 entries at out_rp + vtx_off[g] + g) and its local col_idx (ids in
 * [0, n_g), at out_col + edge_off[g]).  Returns 0 on success.
 */
int gen_rgg_batch_fill(int32_t G, uint64_t seed, const int64_t *n_in, const double *r_in,
                       int64_t *nnz_out, const int64_t *vtx_off, const int64_t *edge_off,
                       int32_t *out_rp, int32_t *out_col) {
    int err = 0;
#pragma omp parallel for schedule(dynamic, 1) reduction(| : err)
    for (int32_t gi = 0; gi < G; gi++) {
        int64_t n = n_in[gi];
        int32_t *px = (int32_t *)malloc((size_t)n * sizeof(int32_t));
        int32_t *py = (int32_t *)malloc((size_t)n * sizeof(int32_t));
        int64_t *deg = (int64_t *)malloc((size_t)n * sizeof(int64_t));
        int64_t *rp = (int64_t *)malloc(((size_t)n + 1) * sizeof(int64_t));
        if (!px || !py || !deg || !rp) { err |= 1; free(px); free(py); free(deg); free(rp); continue; }
        int64_t rint = (int64_t)floor(r_in[gi] * (double)RGG_SIDE);
        rgg_points(g_base(seed, FAM_RGG_BATCH, (uint64_t)gi + 1), n, px, py);
        err |= rgg_scan(n, px, py, rint, deg, NULL, NULL);
        rp[0] = 0;
        for (int64_t i = 0; i < n; i++) rp[i + 1] = rp[i] + deg[i];
        if (!out_col) {
            nnz_out[gi] = rp[n];
        } else {
            if (edge_off[gi + 1] - edge_off[gi] != rp[n] || vtx_off[gi + 1] - vtx_off[gi] != n) err |= 2;
            else {
                int32_t *lrp = out_rp + vtx_off[gi] + gi;
                for (int64_t i = 0; i <= n; i++) lrp[i] = (int32_t)rp[i];
                err |= rgg_scan(n, px, py, rint, NULL, rp, out_col + edge_off[gi]);
            }
        }
        free(px); free(py); free(deg); free(rp);
    }
    return err;
}

/* number of OpenMP threads the generators will use (1 without OpenMP) */
int gen_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Graph gi of the batch alone (same parameters and points as in the packed batch). */
gen_graph *gen_rgg_batch_one(int32_t gi, uint64_t seed, int32_t n_lo, int32_t n_hi, double d_lo, double d_hi) {
    gen_graph *g = g_alloc();
    if (!g) return NULL;
    uint64_t base = g_base(seed, FAM_RGG_BATCH, 0);
    uint64_t h = g_val(base, (uint64_t)gi);
    int64_t n = n_lo + (int64_t)g_below((uint32_t)h, (uint32_t)(n_hi - n_lo + 1));
    double d = d_lo + (d_hi - d_lo) * ((double)(uint32_t)(h >> 32) / 4294967296.0);
    double r = sqrt(d / (M_PI * (double)n));
    g->n = n;
    int32_t *px = NULL, *py = NULL;
    int64_t *deg = NULL, *rp = NULL;
    px = (int32_t *)malloc((size_t)n * sizeof(int32_t));
    py = (int32_t *)malloc((size_t)n * sizeof(int32_t));
    deg = (int64_t *)malloc((size_t)n * sizeof(int64_t));
    rp = (int64_t *)malloc(((size_t)n + 1) * sizeof(int64_t));
    if (!px || !py || !deg || !rp) { g->status = 1; goto done; }
    int64_t rint = (int64_t)floor(r * (double)RGG_SIDE);
    rgg_points(g_base(seed, FAM_RGG_BATCH, (uint64_t)gi + 1), n, px, py);
    if (rgg_scan(n, px, py, rint, deg, NULL, NULL)) { g->status = 1; goto done; }
    rp[0] = 0;
    for (int64_t i = 0; i < n; i++) rp[i + 1] = rp[i] + deg[i];
    g->row_ptr = (int32_t *)malloc(((size_t)n + 1) * sizeof(int32_t));
    g->col = (int32_t *)malloc((size_t)(rp[n] > 0 ? rp[n] : 1) * sizeof(int32_t));
    if (!g->row_ptr || !g->col) { g->status = 1; goto done; }
    if (rgg_scan(n, px, py, rint, NULL, rp, g->col)) { g->status = 1; goto done; }
    for (int64_t i = 0; i <= n; i++) g->row_ptr[i] = (int32_t)rp[i];
    g->nnz = rp[n];
    int32_t md = 0;
    for (int64_t i = 0; i < n; i++) if (deg[i] > md) md = (int32_t)deg[i];
    g->max_deg = md;
done:
    free(px); free(py); free(deg); free(rp);
    return g;
}
