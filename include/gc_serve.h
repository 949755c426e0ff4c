/*
 * gc_serve.h - request server of libgc.so: colors a stream of independent
 * graphs on one GPU with continuous batching.
 *
 * Each request is one graph in HOST memory plus the method's parameters
 * (initial coloring, then recoloring passes; gc.h).  The server owns
 * `slots` worker threads, each with its own HIP stream and gc_ctx, and one
 * device arena of `hbm_budget` bytes from which every admitted request takes
 * its footprint (row_ptr, col_idx and colors, each rounded up to 256 bytes;
 * the per-slot workspace is allocated once at creation and not counted).
 *
 * Admission is first come, first served: the oldest waiting request starts
 * as soon as a slot is idle and its footprint fits in the arena's free
 * space; requests that arrive while others run join as slots and memory free
 * up, and the admitted requests run concurrently on their own streams.  The
 * graph and its colors stay resident in the arena from the first kernel of
 * the initial coloring to the last recoloring pass; the colors are copied to
 * the caller's host buffer at the end.
 *
 * A request's result does not depend on what else runs: every slot runs the
 * same kernels as the single-graph calls of gc.h with the request's seed.
 *
 * Device sharing (cu_partition):
 *   1: every slot's stream is confined to its own disjoint set of compute
 *      units (a compute-unit mask taking an equal share of every XCD), so the
 *      initial colorings and the recoloring passes of different requests run
 *      on the device at the same time without interfering: each slot's
 *      persistent class walk is sized, at creation, to what its own compute
 *      units hold, and no other kernel can take them.  Needs at least 8
 *      compute units per slot; otherwise, or if the runtime refuses the mask,
 *      the server falls back to 0.
 *   0: the slots share all compute units.  Initial colorings of different
 *      slots overlap; a recoloring pass (the persistent walk needs all of its
 *      workgroups resident at once) has the device to itself: it waits until
 *      the initial colorings in flight have finished, and new ones wait for
 *      it.
 *
 * Threads: gc_server_submit, gc_server_poll and gc_server_stats may be
 * called from any host thread.  gc_server_destroy waits for every submitted
 * request to finish.
 */
#ifndef GC_SERVE_H
#define GC_SERVE_H

#include <stdint.h>

#include "gc.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct gc_server gc_server;

typedef struct gc_server_config {
    int32_t device;
    int32_t slots;        /* requests in flight at once (1..64) */
    int64_t hbm_budget;   /* bytes of the device arena for request graphs and colors */
    int64_t max_n;        /* largest request accepted (vertices, CSR entries); sizes each slot's workspace */
    int64_t max_nnz;
    int32_t cu_partition; /* 1 = each slot on its own compute units (passes overlap), 0 = shared device */
    int32_t reserved;
} gc_server_config;

/* One coloring request.  row_ptr, col_idx (host, the CSR of gc.h) and
 * colors (host, n entries, written at completion) are the caller's and must
 * stay valid until the request is reported done by gc_server_poll. */
typedef struct gc_request {
    int32_t n;
    int32_t reserved;
    int64_t nnz;
    const int32_t *row_ptr;
    const int32_t *col_idx;
    int32_t *colors;
    int32_t select;       /* gc_select */
    int32_t X;            /* Random-X width (1 for First Fit) */
    int32_t perm;         /* gc_perm of every recoloring pass */
    int32_t passes;       /* recoloring passes after the initial coloring (>= 0) */
    uint64_t seed;
    uint64_t tag;         /* caller's identifier, returned with the result */
} gc_request;

/* Completion record.  Times are seconds on the server's steady clock
 * (gc_server_now); device_ms is the request's stream time from the first
 * copy to the colors on the host; pass_start_ms / pass_end_ms bound its
 * recoloring passes on the device, in ms since a reference event the server
 * records at creation (comparable across slots: they show which requests'
 * passes overlapped on the device). */
typedef struct gc_request_done {
    uint64_t tag;
    int32_t status;       /* gc_status of the request */
    int32_t slot;
    int32_t rounds;       /* rounds of the initial coloring */
    int32_t colors_init;  /* distinct colors after the initial coloring */
    int32_t colors_final; /* distinct colors after the last pass */
    int32_t running_at_admit;  /* requests in flight when this one was admitted, itself included */
    int64_t footprint;    /* arena bytes it held */
    double t_submit, t_admit, t_done;
    double device_ms;
    double pass_start_ms, pass_end_ms;
} gc_request_done;

typedef struct gc_server_stats {
    int64_t submitted, completed, waiting, running;
    int64_t peak_running;
    int64_t arena_size, arena_used, arena_peak;
    int64_t cu_partition;  /* the sharing mode in effect (cu_partition of the config, or 0 after a fallback) */
    int64_t slot_cus;      /* compute units per slot */
} gc_server_stats;

/* Creates the server: the arena, and per slot a stream, a gc_ctx sized for
 * (max_n, max_nnz) and a worker thread.  GC_ERR_ARG for sizes out of range,
 * GC_ERR_OOM when the arena or a workspace cannot be allocated. */
gc_status gc_server_create(const gc_server_config *cfg, gc_server **out);

/* Queues a request (never waits for the GPU).  GC_ERR_ARG when the graph is
 * above max_n / max_nnz, its footprint is above the whole arena, or a
 * parameter is out of range (the gc_init_color / gc_recolor rules). */
gc_status gc_server_submit(gc_server *s, const gc_request *r);

/* Moves up to `cap` completion records into `out` (oldest first), waiting up
 * to timeout_ms (0 = do not wait, < 0 = wait without limit) for the first
 * one; *count receives how many were written. */
gc_status gc_server_poll(gc_server *s, gc_request_done *out, int32_t cap, int32_t *count, int32_t timeout_ms);

gc_status gc_server_get_stats(gc_server *s, gc_server_stats *out);

/* Seconds since the server was created (the clock of the completion records). */
double gc_server_now(gc_server *s);

/* Waits for every submitted request, then frees the server. */
void gc_server_destroy(gc_server *s);

#ifdef __cplusplus
}
#endif

#endif /* GC_SERVE_H */
