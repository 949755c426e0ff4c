/*
 * gc.h - C ABI of libgc.so: speculative distance-1 graph coloring with
 * iterated recoloring on AMD MI355X (gfx950), after Sariyuce, Saule and
 * Catalyurek, "On Distributed Graph Coloring with Iterative Recoloring".
 *
 * Problem (paper, section 1): a distance-1 coloring maps every vertex to a
 * positive integer so that the two ends of every edge differ.  Here colors
 * are int32, 1-based; 0 means "not colored".
 *
 * Graphs are int32 CSR in device memory: row_ptr[n+1] (row_ptr[0] = 0,
 * non-decreasing, row_ptr[n] = nnz) and col_idx[nnz] with ids in [0, n).
 * The CSR must be symmetric (every entry (u, w) has a matching (w, u)) with
 * no self-loops; duplicate entries and the order inside a row do not change
 * any result.  gc_check_csr verifies these preconditions; the other calls do
 * not, but every kernel clamps row ranges to [0, nnz] and ignores neighbor ids
 * outside [0, n), so a malformed graph gives wrong colors, never an
 * out-of-bounds access.
 *
 * Ownership: every graph and color pointer is a DEVICE pointer owned by the
 * caller, which keeps it alive until the work queued on `stream` is done.
 * The library keeps no pointer after a call returns.  A gc_ctx owns all
 * device workspace (sized at creation) and must not be used by two host
 * threads at once; use one context per concurrent stream.
 *
 * Streams: `stream` is a hipStream_t passed as void* (NULL = the default
 * stream).  Calls enqueue their kernels on it.  Calls whose results are host
 * values (gc_validate, gc_count_colors, gc_check_csr, and any call given a
 * non-NULL gc_stats) synchronize that stream before returning.
 *
 * Errors: every call returns a gc_status; nothing aborts and no C++
 * exception crosses the ABI.  gc_ctx_last_error gives a message for the last
 * failure on a context.  Device-side failures of asynchronous work (a bounded
 * wait of the persistent recoloring walk that gave up, or a walk whose
 * workgroups were not all resident with check_resident on) are sticky: the
 * kernel records them in the context, and the next call on that context that
 * synchronizes (any call with host results, any call given a gc_stats, or
 * gc_ctx_status) returns GC_ERR_DEVICE and clears the record.  The colors
 * written by the failed pass are then unspecified.
 */
#ifndef GC_H
#define GC_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum gc_status {
    GC_OK = 0,
    GC_ERR_ARG = 1,            /* bad argument (NULL pointer, size above the context's capacity, ...) */
    GC_ERR_GRAPH = 2,          /* gc_check_csr: the CSR breaks a precondition */
    GC_ERR_COLORING = 3,       /* gc_recolor: input coloring has a color <= 0 or above the capacity, or (with
                                  the check_input knob) is not a proper coloring */
    GC_ERR_OOM = 4,            /* device or host allocation failed */
    GC_ERR_DEVICE = 5,         /* a HIP runtime call failed, or a kernel's bounded wait ran out */
    GC_ERR_NOT_CONVERGED = 6   /* gc_init_color stopped at max_rounds with vertices still uncolored */
} gc_status;

/* Color selection of the initial coloring. */
typedef enum gc_select {
    GC_FIRST_FIT = 0,  /* smallest permissible color (section 2.1, First Fit) */
    GC_RANDOM_X = 1    /* uniform among the first X permissible colors (section 3.2, Random-X Fit) */
} gc_select;

/* Order in which a recoloring pass visits the color classes (section 3). */
typedef enum gc_perm {
    GC_PERM_REVERSE = 0,  /* RV: decreasing color */
    GC_PERM_NONINC = 1,   /* NI: non-increasing class size, ties by increasing color */
    GC_PERM_NONDEC = 2,   /* ND: non-decreasing class size, ties by increasing color */
    GC_PERM_RANDOM = 3    /* RAND: Knuth shuffle of the increasing color list */
} gc_perm;

/* gc_init_color flags */
#define GC_FLAG_FIXED_PRIORITY 1u /* one random total order for all rounds (round 0's keys) */
#define GC_FLAG_PRIO_LF 2u        /* Largest First: larger degree wins a conflict, ties by round 0's keys */
#define GC_FLAG_PRIO_NATURAL 4u   /* natural order: the smaller vertex id wins a conflict */
#define GC_FLAG_DISTANCE2 8u      /* distance-2 coloring: neighborhoods are the vertices within two edges */

/* Largest X accepted by GC_RANDOM_X. */
#define GC_MAX_X 1024

typedef struct gc_ctx gc_ctx;

typedef struct gc_csr {
    int32_t n;                /* vertices */
    int32_t reserved;         /* set to 0 */
    int64_t nnz;              /* adjacency entries (2 x undirected edges); must be < 2^31 */
    const int32_t *row_ptr;   /* device, n + 1 */
    const int32_t *col_idx;   /* device, nnz */
} gc_csr;

/*
 * Statistics of one call (host struct).  round_sizes / round_degsum are
 * optional host arrays of round_cap entries: |W_r| (vertices colored
 * tentatively in round r) and the sum of their degrees.
 */
typedef struct gc_stats {
    int32_t rounds;        /* init: rounds run (1 = no conflict; 0 iff n = 0); recolor: 0 */
    int32_t num_colors;    /* distinct colors in the output */
    int32_t max_color;     /* largest color in the output */
    int32_t k_classes;     /* recolor: non-empty classes of the input coloring; init: 0 */
    int64_t losers_total;  /* init: sum over rounds of |W_r|, minus n */
    int64_t *round_sizes;  /* host, round_cap entries, or NULL */
    int64_t *round_degsum; /* host, round_cap entries, or NULL */
    int32_t round_cap;
    int32_t reserved;
} gc_stats;

/* Tuning knobs.  No knob changes any result, only the speed (spin_limit aside, whose failures are
   reported as a device error). */
typedef struct gc_tuning {
    int32_t block;         /* threads per workgroup of the streaming kernels (64..1024, multiple of 64) */
    int32_t deg_wave;      /* rows with more than deg_wave entries get a whole wavefront per vertex (default 64) */
    int32_t group;         /* lanes per vertex for rows of at most deg_wave entries in the initial coloring
                              (and in the walk when walk_group says so; power of two, 1..64) */
    int32_t grid_per_cu;   /* workgroups per compute unit for grid-stride kernels (1..64) */
    int32_t walk_mode;     /* recoloring class walk: 0 = one persistent launch, waits per dependency;
                              1 = one launch per class (host reads the class count) */
    int32_t xcd_chunks;    /* persistent walk: 1 = every class's chunks cut into 8 consecutive parts, part x
                              taken by the workgroups the hardware places on XCD x, so a region of the vertex
                              order stays in one XCD's L2 across classes; 0 = round robin; -1 (default) = the
                              parts when at most half the adjacency entries join vertices 32,768 or more apart
                              in the vertex order (their neighbors share an XCD's L2), else round robin */
    int32_t check_resident;/* persistent walk: verify at start that every workgroup is resident (diagnostic;
                              a failed check makes the call return GC_ERR_DEVICE when it synchronizes) */
    int32_t deg_split;     /* rows longer than both deg_wave and deg_split (0 = never) are scanned by
                              several wavefronts at once, split_len entries each, in the initial coloring's
                              rounds and in the recoloring walk (graphs whose longest row is under 64 use a
                              walk without this path) */
    int32_t split_len;     /* entries per wavefront for split rows (>= 64) */
    int32_t hub_words;     /* 64-bit mask words per split row (1..64): colors up to 64 * hub_words are merged
                              across wavefronts; larger colors rescan the row, and recoloring ranks of
                              64 * hub_words and above keep their long rows on one wavefront */
    int32_t walk_group;    /* lanes per vertex in the recoloring walk (power of two, 1..64); 0 = automatic:
                              8 when every row is shorter than 64 entries, else 2 */
    int32_t d2_star;       /* distance-2 detect step: 0 = automatic (per-neighborhood marking for rounds
                              of more than n / 8 vertices when no row exceeds 64 entries, else a scan of
                              each vertex's distance-2 neighborhood), 1 = marking in every round, -1 = the
                              scan in every round; results are the same */
    int32_t batch_wg_per_cu; /* gc_batch_color: workgroups per compute unit (0 = 4; at most 5 fit) */
    int32_t batch_order;   /* gc_batch_color: 0 = graphs taken in id order, 1 = largest (most entries) first
                              (batches of at most 8192 graphs; larger ones keep id order) */
    int32_t spin_limit;    /* persistent walk: polls of one bounded dependency wait before it gives up
                              (0 = 2^20, about a second).  A wait that gives up leaves a wrong color and
                              raises the context's sticky device error (see gc_ctx_status); a small value
                              only serves to test that error path */
    int32_t check_input;   /* 1 = gc_recolor, gc_recolor_d2 and gc_arc_recolor first check that colors_in is
                              a proper coloring (distance 2 for gc_recolor_d2) with every color >= 1, and
                              return GC_ERR_COLORING otherwise (one validation sweep; synchronizes) */
    int32_t trace;         /* 1 = the persistent walk records when each class finishes (profiling aid, see
                              gc_ctx_get_trace; device atomics per wavefront and class) */
    int32_t tail_max;      /* initial coloring: > 0 = once a round has at most tail_max vertices and no row
                              needs the split kernels, the remaining rounds run in one persistent launch with
                              grid barriers (no host read-back per round); 0 (default) or -1 = never (the
                              per-round launches measured faster on every workload tried) */
    int32_t walk_flags;    /* persistent walk, bit mask: 1 = inside a class, split rows are taken first, then
                              wavefront rows, then group rows; 2 = a split-row sub-chunk still waiting when all
                              the row's other sub-chunks are done takes their mask words and publishes the color
                              itself; 4 = a row waits for a pending lower-rank neighbor where its scan meets
                              it (default: the scan of the whole row goes on, and the pending words are
                              waited for together at its end) */
    int32_t cu_count;      /* compute units the context's streams may use (0 = all of the device): sizes the
                              grids, and the persistent launches measure their co-resident grid on it; for
                              streams created with a compute-unit mask (as the request server does) */
    int32_t compact_init;  /* initial coloring: neighbor colors read from a compact copy of the colors, one byte
                              when no color can exceed 127 (longest row + X <= 127), else two bytes saturated at
                              compact_sat; 1 = always, 0 = never (read the int32 colors), -1 (default) = the
                              one-byte copy when it fits and more than half of the adjacency entries (u, w) have
                              |u - w| >= 32768 (neighbors far apart in the vertex order, where the narrower copy
                              keeps more of the colors in the L2; with near neighbors its extra stores cost more
                              than it saves) */
    int32_t compact_sat;   /* two-byte copy: words saturate at +-compact_sat (1..32767, 0 = 32767), and a
                              saturated word is read from the colors instead; a small value only serves to test
                              that path */
} gc_tuning;

const char *gc_status_string(gc_status s);

/*
 * Create a context on HIP device `device` able to color graphs with up to
 * max_n vertices and max_nnz adjacency entries.  Allocates every workspace
 * buffer once (roughly 40 bytes per vertex).  *out is NULL on failure.
 */
gc_status gc_ctx_create(int device, int64_t max_n, int64_t max_nnz, gc_ctx **out);
void gc_ctx_destroy(gc_ctx *ctx);
const char *gc_ctx_last_error(const gc_ctx *ctx);

/*
 * Synchronizes `stream` and reports the context's sticky device error: GC_OK
 * if no asynchronous work since the last report failed on the device, else
 * GC_ERR_DEVICE (message in gc_ctx_last_error), after which the record is
 * clear.  For callers that queue passes without gc_stats.
 */
gc_status gc_ctx_status(gc_ctx *ctx, void *stream);
gc_status gc_ctx_get_tuning(const gc_ctx *ctx, gc_tuning *t);
gc_status gc_ctx_set_tuning(gc_ctx *ctx, const gc_tuning *t);

/*
 * Launch facts of a context (host values): info[0] = compute units,
 * info[1] = workgroups of the persistent recoloring walk for the current
 * group size (0 until first used), info[2] = its workgroups per compute unit,
 * info[3] = the longest row of the graph a call on this context analysed last
 * (-1 before any), info[4] = that graph's adjacency entries (u, w) with
 * |u - w| >= 32768 (-1 before any; the far entries pick the default color
 * copy of the initial coloring).  Fills min(cap, 5) entries.
 */
gc_status gc_ctx_get_info(gc_ctx *ctx, int64_t *info, int cap);

/*
 * Kernel timing (profiling aid).  When enabled, the library records a pair of
 * HIP events on the launch stream around every kernel of the selected kinds
 * and sums the elapsed times per kind.  enable: 0 = off, -1 = every kind,
 * otherwise a bit mask (bit k selects kind k).  gc_ctx_get_timing
 * synchronizes the device, fills launches[kind] and ms[kind] for kind <
 * min(cap, GC_KERNEL_KINDS) and returns GC_OK.  Enabling (or re-enabling)
 * clears the sums.  Timing adds event records between launches; select only
 * the kinds a measurement needs.
 */
enum {
    GC_K_ROUND0 = 0, GC_K_ASSIGN = 1, GC_K_DETECT = 2, GC_K_HIST = 3, GC_K_ORDER = 4, GC_K_SCATTER = 5,
    GC_K_WALK = 6, GC_K_COUNT = 7, GC_K_BATCH = 8, GC_K_OTHER = 9, GC_KERNEL_KINDS = 10
};
gc_status gc_ctx_set_timing(gc_ctx *ctx, int enable);

/*
 * Class-completion trace of the last persistent recoloring walk run with the
 * trace knob (profiling aid for the dependency chain of section 3's class
 * steps).  Synchronizes `stream`.  out[0] = 0 (walk start), out[1] = walk
 * end, out[2 + 2s] = when the last vertex of rank s published its color,
 * out[3 + 2s] = the same for the split rows of rank s (-1 if none), all in
 * nanoseconds since the first workgroup started.  Fills min(cap, 2 + 2k)
 * entries (k = the pass's classes) and sets *count to 2 + 2k.  GC_ERR_ARG if
 * no walk was traced on ctx.
 */
gc_status gc_ctx_get_trace(gc_ctx *ctx, int64_t *out, int64_t cap, int64_t *count, void *stream);
gc_status gc_ctx_get_timing(gc_ctx *ctx, int64_t *launches, double *ms, int cap);

/*
 * Check the CSR preconditions on the device: row_ptr[0] = 0, non-decreasing,
 * row_ptr[n] = nnz, ids in [0, n), no self-loops, symmetric with multiplicity
 * (checked by per-entry reverse search, so rows must be sorted for it to be
 * fast; unsorted rows are still checked correctly).  Returns GC_OK or
 * GC_ERR_GRAPH.  Synchronizes the stream.
 */
gc_status gc_check_csr(gc_ctx *ctx, const gc_csr *g, void *stream);

/*
 * Speculative initial coloring (section 2.2 framework, run as one superstep
 * per round over every uncolored vertex).  Round r: every vertex v of the
 * uncolored set W_r takes a tentative color from the colors its neighbors
 * held at the start of the round: the (j+1)-th smallest positive color not
 * among them, j = 0 for First Fit and j = hash(seed, v, r) mapped to [0, X)
 * for Random-X Fit (section 3.2).  Then v loses if a neighbor in W_r has the
 * same tentative color and a larger priority key (a hash of seed, vertex and
 * round; the random total order of section 2.2), losers form W_{r+1}, winners
 * keep their colors.  Repeats until no vertex loses.
 *
 * colors (device, n, output) receives the coloring.  max_rounds = 0 means no
 * limit (the process always ends within n rounds); with a limit, the call
 * returns GC_ERR_NOT_CONVERGED after that many rounds, with the vertices
 * still uncolored at <= 0.  X must be in [1, GC_MAX_X] for GC_RANDOM_X and is
 * ignored for GC_FIRST_FIT.
 *
 * flags: GC_FLAG_FIXED_PRIORITY keeps round 0's keys in every round (the
 * paper's fixed random order); GC_FLAG_PRIO_LF (Largest First: the larger
 * degree wins, ties by round 0's keys) and GC_FLAG_PRIO_NATURAL (the smaller
 * id wins) use those vertex-visit orders of section 2.1 as the conflict
 * priority and exclude each other.  GC_FLAG_DISTANCE2 computes a distance-2
 * coloring (section 1's distance-k problem with k = 2: vertices joined by a
 * path of one or two edges differ), the same rounds with N(v) read as
 * N(v) u N(N(v)) minus v; it takes rows shorter than 2^25 entries, and not
 * GC_FLAG_PRIO_LF; st->round_degsum is left at 0 for it.  Unknown flags give
 * GC_ERR_ARG.
 */
gc_status gc_init_color(gc_ctx *ctx, const gc_csr *g, int32_t select, int32_t X, uint64_t seed,
                        int32_t max_rounds, uint32_t flags, int32_t *colors, gc_stats *st, void *stream);

/*
 * gc_init_color that also records, for every vertex, the round in which its
 * color became final (section 2.2's rounds, 0-based: round 0 is the first
 * speculative round; a vertex commits in the round in which it wins its
 * conflicts).  vertex_round (device, n, output): the commit round, or -1 for
 * a vertex still uncolored when max_rounds stopped the coloring.  The
 * vertices with a commit round >= r are those of W_r, so st->round_sizes[r]
 * counts them.  A debugging aid, to find where two colorings part: the
 * colors and statistics are gc_init_color's.  Not available with
 * GC_FLAG_DISTANCE2 (GC_ERR_ARG); vertex_round NULL with n > 0: GC_ERR_ARG.
 */
gc_status gc_init_color_rounds(gc_ctx *ctx, const gc_csr *g, int32_t select, int32_t X, uint64_t seed,
                               int32_t max_rounds, uint32_t flags, int32_t *colors, int32_t *vertex_round,
                               gc_stats *st, void *stream);

/*
 * One iterated-greedy recoloring pass (section 2.1, Culberson's Iterated
 * Greedy; section 3, synchronous recoloring RC).  The classes of colors_in
 * are visited in the order `perm` picks; every vertex of the current class
 * takes the smallest positive color not held by a neighbor recolored earlier
 * in this pass.  The result never has more colors than the input.
 *
 * colors_in (device, n): a proper coloring with colors in [1, n + GC_MAX_X];
 * colors_out (device, n) may equal colors_in (in place).  `pass` is the pass
 * index that seeds GC_PERM_RANDOM (with `seed`).  An input color outside the
 * range gives GC_ERR_COLORING when st != NULL (checked at the synchronization
 * the stats need); without stats such input leaves colors_out unspecified.
 */
gc_status gc_recolor(gc_ctx *ctx, const gc_csr *g, int32_t perm, uint64_t seed, int32_t pass,
                     const int32_t *colors_in, int32_t *colors_out, gc_stats *st, void *stream);

/*
 * `passes` recoloring passes in a row (section 3: recoloring iterated, each
 * pass on the previous one's result): pass p (0-based) is exactly
 * gc_recolor(ctx, g, perms[p], seed, pass0 + p, ...) with colors_in the
 * previous pass's colors_out (colors_in itself for p = 0); colors_out ends
 * with the last pass's colors.  perms (host, passes entries) each in [0, 3];
 * st (host, NULL or `passes` records) gets each pass's statistics, as
 * gc_recolor's.  passes = 0 copies colors_in to colors_out.
 *
 * The passes are queued on `stream` back to back (one call for a whole
 * schedule, as the hybrid schedules of gc_schedule_perm give it); with st
 * NULL nothing synchronizes.  Error behavior as gc_recolor, for the first
 * pass that fails (later passes are then not queued).
 */
gc_status gc_recolor_passes(gc_ctx *ctx, const gc_csr *g, const int32_t *perms, int32_t passes, uint64_t seed,
                            int32_t pass0, const int32_t *colors_in, int32_t *colors_out, gc_stats *st,
                            void *stream);

/*
 * gc_recolor for a distance-2 coloring: the same class order, and every
 * vertex of the current class takes the smallest positive color not held by
 * a vertex within two edges recolored earlier in this pass.  colors_in must
 * be a distance-2 coloring (vertices of one class are then never within two
 * edges, so a class is recolored at once); any other input leaves
 * colors_out unspecified (color range errors as gc_recolor).  Rows shorter
 * than 2^25 entries (GC_ERR_ARG otherwise).  Synchronizes the stream once
 * per pass to size the per-class launches.
 */
gc_status gc_recolor_d2(gc_ctx *ctx, const gc_csr *g, int32_t perm, uint64_t seed, int32_t pass,
                        const int32_t *colors_in, int32_t *colors_out, gc_stats *st, void *stream);

/*
 * Asynchronous recoloring aRC (section 3): the classes of colors_in, in the
 * order `perm` picks (as gc_recolor), give each vertex a rank, and a second
 * speculative coloring runs in rounds with First Fit where, of two neighbors
 * with the same tentative color, the one of the earlier class keeps it
 * (the vertex-visit order taken from the previous coloring, read as the
 * conflict priority of the Jacobi rounds).  Trades color count against the
 * class-by-class dependency chain of gc_recolor.  colors_in must be a proper
 * coloring with colors in [1, n + GC_MAX_X] (GC_ERR_COLORING otherwise);
 * colors_out may equal colors_in.  Synchronizes like gc_init_color;
 * st->rounds counts its rounds, st->k_classes the input classes.
 */
gc_status gc_arc_recolor(gc_ctx *ctx, const gc_csr *g, int32_t perm, uint64_t seed, int32_t pass,
                         const int32_t *colors_in, int32_t *colors_out, gc_stats *st, void *stream);

/*
 * Check of the problem statement's condition (section 1: a distance-1
 * coloring gives the two ends of every edge different colors).
 * conflict_edges: adjacency entries (u, w) with u < w and colors[u] ==
 * colors[w] > 0 (each undirected edge once; a duplicated entry counts once
 * per copy); uncolored: vertices with colors[v] <= 0.  colors is a proper
 * coloring iff both are 0.  colors: device, n entries.  Host outputs;
 * synchronizes.  Either pointer may be NULL.  Errors: GC_ERR_ARG for a NULL
 * context, graph or (n > 0) colors, or a graph above the context's capacity;
 * GC_ERR_DEVICE if a HIP call fails.
 */
gc_status gc_validate(gc_ctx *ctx, const gc_csr *g, const int32_t *colors, int64_t *conflict_edges,
                      int64_t *uncolored, void *stream);

/*
 * Distance-2 check (section 1's distance-k condition with k = 2: two
 * vertices joined by a path of at most two edges differ).
 * conflict_pairs: unordered pairs {u, w}, u != w, within two edges of each
 * other with colors[u] == colors[w] > 0, each pair once however many paths
 * join it; uncolored: vertices with colors[v] <= 0.  colors is a distance-2
 * coloring iff both are 0.  Rows shorter than 2^25 entries.  Host outputs;
 * synchronizes.  Either pointer may be NULL.
 */
gc_status gc_validate_d2(gc_ctx *ctx, const gc_csr *g, const int32_t *colors, int64_t *conflict_pairs,
                         int64_t *uncolored, void *stream);

/*
 * Autotuning.  The knobs of gc_tuning change how the work is scheduled,
 * never a color.  gc_autotune runs the initial coloring and `passes`
 * recoloring passes on g (arguments as gc_init_color / gc_recolor) under
 * candidate settings of deg_wave, group, walk_group, deg_split and
 * grid_per_cu, one knob at a time with the others held at the best so far,
 * timing each with HIP events (best of two runs).  It checks that every
 * candidate gives the same colors (a 64-bit checksum of the (vertex, color)
 * pairs; GC_ERR_DEVICE if one differs) and leaves the fastest setting in ctx.
 * colors (device, n) receives the coloring; *best (may be NULL) the setting
 * and *best_ms (may be NULL) its time.  Synchronizes the stream often; runs
 * the method roughly 40 times.
 */
gc_status gc_autotune(gc_ctx *ctx, const gc_csr *g, int32_t select, int32_t X, int32_t perm, int32_t passes,
                      uint64_t seed, int32_t *colors, gc_tuning *best, double *best_ms, void *stream);

/*
 * Color counts of section 1: the number of colors of a coloring is its
 * largest color, and a coloring partitions the vertices into independent
 * sets, one per color in use.  num_colors: distinct positive values in
 * colors[0..n) (the number of non-empty classes); max_color: the largest
 * (0 if none).  The two agree for First Fit and recolored outputs; Random-X
 * can leave unused colors below the largest.  colors: device, n entries.
 * Host outputs; synchronizes; either output pointer may be NULL.  Errors:
 * GC_ERR_ARG for a NULL context, n < 0, n above the context's capacity, or
 * colors NULL with n > 0; GC_ERR_OOM if the color bitmap cannot grow to the
 * largest color; GC_ERR_DEVICE if a HIP call fails.
 */
gc_status gc_count_colors(gc_ctx *ctx, int32_t n, const int32_t *colors, int32_t *num_colors, int32_t *max_color,
                          void *stream);

/*
 * gc_count_colors for callers that cannot allocate device memory (harnesses
 * that forbid hipMalloc, tight serving loops): same results, no context, and
 * no allocation of any kind.  The kernels work in one static device array of
 * the library (about 128 KiB per GPU, held until the process ends) that
 * every call on that GPU shares: calls that overlap on one GPU (from several
 * host threads or streams at once) race and give wrong counts.  Runs on the
 * calling thread's current HIP device; `stream` must belong to it.  Colors
 * are counted up to GC_STATIC_MAX_COLOR: a larger color gives GC_ERR_ARG.
 * Host outputs (either may be NULL); synchronizes the stream, so it cannot
 * be captured into a HIP graph.  Errors: GC_ERR_ARG for n < 0, colors NULL
 * with n > 0, or a color above GC_STATIC_MAX_COLOR; GC_ERR_DEVICE if a HIP
 * call fails.
 */
#define GC_STATIC_MAX_COLOR (1 << 20)
gc_status gc_count_colors_static(int32_t n, const int32_t *colors, int32_t *num_colors, int32_t *max_color,
                                 void *stream);

/* ---------------------------------------------------------------------------
 * Batched coloring: many independent graphs in one persistent launch.
 *
 * Packed CSR: graph g has n_g = vtx_off[g+1] - vtx_off[g] vertices and
 * nnz_g = edge_off[g+1] - edge_off[g] entries; its local row_ptr (n_g + 1
 * entries, values in [0, nnz_g]) is at row_ptr + vtx_off[g] + g, its local
 * col_idx (ids in [0, n_g)) at col_idx + edge_off[g], and its colors at
 * colors + vtx_off[g].  Offsets are int64 (the packed arrays may exceed 2^31
 * entries); each graph must have n_g <= 2^31 - 1 and nnz_g < 2^31.
 */
typedef struct gc_batch_csr {
    int32_t num_graphs;
    int32_t reserved;
    const int64_t *vtx_off;   /* device, G + 1 */
    const int64_t *edge_off;  /* device, G + 1 */
    const int32_t *row_ptr;   /* device, vtx_off[G] + G */
    const int32_t *col_idx;   /* device, edge_off[G] */
} gc_batch_csr;

/* Per-graph result of gc_batch_color (device array of G entries). */
typedef struct gc_graph_stats {
    int32_t rounds;          /* initial-coloring rounds */
    int32_t colors_init;     /* distinct colors after the initial coloring */
    int32_t colors_final;    /* colors after the last pass */
    int32_t status;          /* gc_status of this graph (GC_ERR_NOT_CONVERGED if max_rounds hit) */
} gc_graph_stats;

/*
 * Color every graph of the batch: initial coloring with seed_g, then `passes`
 * recoloring passes with class order `perm` (pass index p = 0..passes-1).
 * seed_g = mix64(base_seed + 0x9E3779B97F4A7C15 * (4 << 32 | g)) (SplitMix64
 * output function), so that gc_init_color / gc_recolor called on graph g
 * alone with seed_g give the same colors bit for bit.  max_vertices_per_graph
 * bounds n_g (the caller knows it; it sizes the workspace).  per_graph may be
 * NULL.  Asynchronous on `stream`.
 */
gc_status gc_batch_color(gc_ctx *ctx, const gc_batch_csr *b, int32_t select, int32_t X, int32_t perm,
                         int32_t passes, uint64_t base_seed, int32_t max_rounds, int32_t max_vertices_per_graph,
                         int32_t *colors, gc_graph_stats *per_graph, void *stream);

/* seed_g of graph g in a batch (host helper, same formula as above). */
uint64_t gc_batch_graph_seed(uint64_t base_seed, int32_t g);

/*
 * gc_autotune for gc_batch_color (arguments as there): tries every
 * combination of batch_order (0, 1) and batch_wg_per_cu (1..5) on the batch,
 * once each after a warm-up run with the current setting, checks that every
 * one gives the same colors and per-graph statistics, and leaves the fastest
 * in ctx.  Batches of at least one graph.
 */
gc_status gc_autotune_batch(gc_ctx *ctx, const gc_batch_csr *b, int32_t select, int32_t X, int32_t perm,
                            int32_t passes, uint64_t base_seed, int32_t max_rounds, int32_t max_vertices_per_graph,
                            int32_t *colors, gc_graph_stats *per_graph, gc_tuning *best, double *best_ms,
                            void *stream);


/*
 * Class-order schedules over recoloring iterations (section 4.2.1, the
 * sequential study of random permutations).  Iteration t counts from 1.
 *   GC_SCHED_FIXED:       `base` at every iteration;
 *   GC_SCHED_ND_RAND_X:   RAND when t is a multiple of x (x >= 1), ND otherwise;
 *   GC_SCHED_ND_RAND_POW2: RAND when t is a power of two >= 2, ND otherwise.
 * gc_schedule_perm returns the gc_perm of iteration t, or -1 for a bad
 * argument (unknown schedule, t < 1, base outside gc_perm, x < 1 for
 * GC_SCHED_ND_RAND_X).  Host only; pass t - 1 as gc_recolor's `pass`.
 */
typedef enum gc_schedule { GC_SCHED_FIXED = 0, GC_SCHED_ND_RAND_X = 1, GC_SCHED_ND_RAND_POW2 = 2 } gc_schedule;
int32_t gc_schedule_perm(int32_t schedule, int32_t base, int32_t x, int32_t t);

/*
 * Parameter presets (section 4.3): GC_PRESET_SPEED = First Fit initial
 * coloring, no recoloring; GC_PRESET_QUALITY = Random-X Fit with X = 5 and
 * one recoloring pass in ND order (pass index 0).  The paper's presets also
 * fix a processor-local vertex order ("internal first"), a distributed-memory
 * notion with no counterpart in the single-GPU rounds.  Same arguments,
 * synchronization and errors as gc_init_color; st (optional) receives the
 * initial coloring's rounds and the final color counts.
 */
typedef enum gc_preset { GC_PRESET_SPEED = 0, GC_PRESET_QUALITY = 1 } gc_preset;
gc_status gc_color_preset(gc_ctx *ctx, const gc_csr *g, int32_t preset, uint64_t seed, int32_t *colors, gc_stats *st,
                          void *stream);

#ifdef __cplusplus
}
#endif

#endif /* GC_H */
