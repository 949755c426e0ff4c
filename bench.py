#!/usr/bin/env python3
"""Benchmark: speculative coloring + iterated recoloring on one MI355X.

A step is one pass of the whole method over one synthetic graph resident in
HBM: the speculative initial coloring followed by P recoloring passes.
Default workload: 3D 27-point mesh 128^3 (n = 2,097,152; nnz = 53,645,816),
Random-X initial coloring with X = 4, then 10 recoloring passes in
non-increasing class-size order (NI), seed 1.

Metric (GTEPS/pass): undirected edges m = nnz / 2 times the passes of a step
(the initial coloring counts as one pass) per second of the whole step.
Printed as ONE JSON line on stdout; progress goes to stderr.

    python bench.py [--steps K] [--warmup W] [--workload mesh128|er10k|rmat22|batch4096]

The batch4096 workload colors 4,096 random geometric graphs (n uniform in
[500, 50000], target degree uniform in [8, 40]) packed into one CSR, each with
Random-X (X=4) + 5 reverse-order recoloring passes, in one persistent launch,
and compares graphs/s with plain per-graph calls of the same library on the
same GPU (same seeds, colorings checked identical).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, 8 TB/s


def log(*a):
    print(*a, file=sys.stderr, flush=True)


WORKLOADS = {
    # name: (description, graph builder, select, X, perm name, passes)
    "mesh128": ("3D 27-point mesh 128^3, Random-X (X=4) initial coloring + 10 NI recoloring passes",
                lambda gen: gen.mesh27(128), "RANDOM_X", 4, "NI", 10),
    "er10k": ("Erdos-Renyi G(n=10000, m=50000), First Fit initial coloring + 3 RV recoloring passes",
              lambda gen: gen.er(10000, 50000, 1), "FIRST_FIT", 1, "RV", 3),
    "rmat22": ("RMAT scale 22, edge factor 16, (0.57,0.19,0.19,0.05), First Fit initial coloring + 10 RAND passes",
               lambda gen: gen.rmat(22, 16, 0.57, 0.19, 0.19, 1), "FIRST_FIT", 1, "RAND", 10),
}


# committed rocprofv3 counter summaries of the walk, per workload
TRAFFIC_RECORDS = {"mesh128": os.path.join(ROOT, "profiles", "pmc_traffic_k_walk_flow_mesh27_128.txt"),
                   "rmat22": os.path.join(ROOT, "profiles", "pmc_traffic_k_walk_flow_rmat22.txt")}


def recorded_traffic(workload, tuning):
    """HBM-side bytes per walk launch from the committed rocprofv3 counter
    summary, or None when that record does not describe the kernel that runs
    now (different workload, tuning or kernel source)."""
    import hashlib

    if workload not in TRAFFIC_RECORDS:
        return None
    try:
        rec = dict(line.split(": ", 1) for line in open(TRAFFIC_RECORDS[workload]).read().splitlines()
                   if ": " in line and not line.startswith("#"))
    except OSError:
        return None
    src = b"".join(open(os.path.join(ROOT, "paper_1407_6745_amd", "csrc", f), "rb").read()
                   for f in ("gc_recolor.hip", "gc_internal.h"))
    want = {k: int(v) for k, v in (kv.split("=") for kv in rec.get("tuning", "").split())}
    if (rec.get("workload") != workload or hashlib.sha256(src).hexdigest() != rec.get("kernel_source_sha256")
            or any(tuning.get(k) != v for k, v in want.items())):
        return None
    return int(rec["traffic_bytes_per_launch"])


def cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    import platform

    return platform.processor() or "unknown"


class OneCore:
    """Pins the calling thread to one host core (the lowest this process may
    use) while the block runs, in-process (no re-exec); restores the mask."""

    def __enter__(self):
        self.saved = os.sched_getaffinity(0)
        self.core = min(self.saved)
        os.sched_setaffinity(0, {self.core})
        return self

    def __exit__(self, *exc):
        os.sched_setaffinity(0, self.saved)
        return False


ORACLE_BUILD = "gcc -O3 -march=x86-64-v3, single thread"


def _oracle_fast():
    import oracle

    oracle.use_variant("fast")
    return oracle


def cpu_baseline(g, select, X, perms, passes, seed, method="rc", budget_s=20.0, repeats=3):
    """The oracle as it stands (plain single-threaded C, -O3 build) on the same
    workload, pinned to one host core: the initial coloring and each pass timed
    separately, median over `repeats` repetitions.  A workload whose first
    repetition exceeds budget_s / repeats is timed once, on the initial
    coloring and as many passes as fit (at least one).  Returns (record, colors
    after the timed passes, number of timed passes)."""
    oracle = _oracle_fast()
    sel = oracle.FIRST_FIT if select == "FIRST_FIT" else oracle.RANDOM_X
    recolor = oracle.recolor if method == "rc" else oracle.arc_recolor
    runs, k = [], passes
    with OneCore() as pin:
        t_start = time.perf_counter()
        for r in range(repeats):
            t0 = time.perf_counter()
            c = oracle.init_color(g, sel, X, seed).colors
            t_init = time.perf_counter() - t0
            t_pass = []
            for p in range(k):
                t0 = time.perf_counter()
                c = recolor(g, c, perms[p], seed, p).colors
                t_pass.append(time.perf_counter() - t0)
                if r == 0 and p + 1 < k and time.perf_counter() - t_start > budget_s / repeats:
                    k = p + 1  # the budget is spent: later repetitions time these k passes
                    break
            runs.append((t_init, t_pass))
            if r == 0 and time.perf_counter() - t_start > budget_s / repeats:
                break
    med_init = float(np.median([x[0] for x in runs]))
    med_pass = [float(np.median([x[1][p] for x in runs])) for p in range(k)]
    total = med_init + sum(med_pass)
    rec = {"value": round(g.m * (1 + k) / total / 1e9, 5), "unit": "GTEPS", "cores": 1, "kind": "oracle",
           "sample": f"initial coloring + the first {k} of {passes} passes of the same graph, "
                     f"{len(runs)} repetition(s), median per phase, one thread pinned to one core",
           "build": ORACLE_BUILD, "cpu_model": cpu_model(), "host_cpus": os.cpu_count(), "pinned_core": pin.core,
           "init_s": round(med_init, 4), "pass_s": [round(t, 4) for t in med_pass],
           "seconds": round(sum(sum(x[1]) + x[0] for x in runs), 3)}
    return rec, c, k


def batch_cpu_baseline(b, X, passes, seed, budget_s=12.0):
    """The oracle (single thread, as it stands, -O3 build) on the first graphs
    of the batch, whole method per graph, pinned to one core."""
    import paper_1407_6745_amd as gc

    oracle = _oracle_fast()
    with OneCore() as pin:
        t0 = time.perf_counter()
        done = 0
        edges = 0
        while done < b.num_graphs and time.perf_counter() - t0 < budget_s:
            g = b.graph(done)
            sg = gc.batch_graph_seed(seed, done)
            c = oracle.init_color(g, oracle.RANDOM_X, X, sg).colors
            for p in range(passes):
                c = oracle.recolor(g, c, oracle.PERM_REVERSE, sg, p).colors
            edges += g.m
            done += 1
        el = time.perf_counter() - t0
    return {"value": round(done / el, 3), "unit": "graphs/s", "cores": 1, "kind": "oracle",
            "sample": f"graphs 0..{done - 1} of the batch ({edges} undirected edges), whole method each, "
                      f"one thread pinned to one core",
            "build": ORACLE_BUILD, "cpu_model": cpu_model(), "pinned_core": pin.core,
            "gteps": round(edges * (passes + 1) / el / 1e9, 4), "seconds": round(el, 3)}


def batch_cpu_baseline_all_cores(b, X, passes, seed, budget_s=10.0):
    """The same oracle on every host core this process may use: one graph per
    task, threads taking graph ids in order (the oracle is plain C behind
    ctypes, which releases the GIL during each call)."""
    import itertools
    import threading
    from concurrent.futures import ThreadPoolExecutor

    import paper_1407_6745_amd as gc

    oracle = _oracle_fast()
    oracle._load()
    workers = len(os.sched_getaffinity(0))
    ids = itertools.count()
    lock = threading.Lock()
    t0 = time.perf_counter()
    deadline = t0 + budget_s

    def work():
        done, edges = 0, 0
        while time.perf_counter() < deadline:
            with lock:
                i = next(ids)
            if i >= b.num_graphs:
                break
            g = b.graph(i)
            sg = gc.batch_graph_seed(seed, i)
            c = oracle.init_color(g, oracle.RANDOM_X, X, sg).colors
            for p in range(passes):
                c = oracle.recolor(g, c, oracle.PERM_REVERSE, sg, p).colors
            done += 1
            edges += g.m
        return done, edges

    with ThreadPoolExecutor(workers) as ex:
        res = [f.result() for f in [ex.submit(work) for _ in range(workers)]]
    el = time.perf_counter() - t0
    done, edges = sum(r[0] for r in res), sum(r[1] for r in res)
    return {"value": round(done / el, 3), "unit": "graphs/s", "cores": workers, "kind": "oracle",
            "sample": f"the first {done} graphs of the batch ({edges} undirected edges), whole method each, "
                      f"one graph per task on {workers} threads",
            "build": ORACLE_BUILD.replace("single thread", "one thread per task"), "cpu_model": cpu_model(),
            "gteps": round(edges * (passes + 1) / el / 1e9, 4), "seconds": round(el, 3)}


def run_batch(args):
    import torch

    import gen
    import paper_1407_6745_amd as gc

    X, passes, G = 4, 5, args.graphs
    t0 = time.perf_counter()
    b = gen.rgg_batch(G, args.seed)
    n_tot, nnz_tot = int(b.vtx_off[-1]), int(b.edge_off[-1])
    log(f"[bench] batch of {G} RGGs: n={n_tot} nnz={nnz_tot} ({time.perf_counter() - t0:.1f}s)")
    dev = torch.device("cuda:0")
    vo = torch.from_numpy(b.vtx_off).to(dev)
    eo = torch.from_numpy(b.edge_off).to(dev)
    rp = torch.from_numpy(b.row_ptr).to(dev)
    col = torch.from_numpy(b.col).to(dev)
    ns = np.diff(b.vtx_off)
    max_n = int(ns.max())
    max_nnz = int(np.diff(b.edge_off).max())
    ctx = gc.Context(max_n, max_nnz)
    if args.tune:
        ctx.set_tuning(**{k: int(v) for k, v in (kv.split("=") for kv in args.tune.split(","))})
    colors = torch.empty(n_tot, dtype=torch.int32, device=dev)
    per = torch.empty((G, 4), dtype=torch.int32, device=dev)

    def batched():
        gc.batch_color(vo, eo, rp, col, gc.RANDOM_X, X, gc.PERM_REVERSE, passes, args.seed,
                       max_vertices_per_graph=max_n, out=colors, per_graph=per, ctx=ctx)

    # the autotuner picks the graph order and workgroups per CU on this batch
    # (every candidate checked to give the same colors), unless --tune fixes them
    tuned = None
    if not args.tune and not args.no_autotune:
        t0 = time.perf_counter()
        best, best_ms, _, _ = gc.autotune_batch(vo, eo, rp, col, gc.RANDOM_X, X, gc.PERM_REVERSE, passes, args.seed,
                                                max_vertices_per_graph=max_n, out=colors, per_graph=per, ctx=ctx)
        tuned = {"batch_order": best["batch_order"], "batch_wg_per_cu": best["batch_wg_per_cu"],
                 "launch_ms": round(best_ms, 3), "seconds": round(time.perf_counter() - t0, 2)}
        log(f"[bench] autotuned: {tuned}")

    for _ in range(args.warmup):
        batched()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        batched()
    torch.cuda.synchronize()
    t_b = (time.perf_counter() - t0) / args.steps
    pg = per.cpu().numpy()
    log(f"[bench] batched: {t_b * 1e3:.1f} ms per launch, {G / t_b:.0f} graphs/s")

    # plain: the single-graph library calls, graph after graph on the same stream
    plain = torch.zeros(n_tot, dtype=torch.int32, device=dev)
    seeds = [gc.batch_graph_seed(args.seed, g) for g in range(G)]
    views = []
    for g in range(G):
        a, z = int(b.vtx_off[g]), int(b.vtx_off[g + 1])
        e0, e1 = int(b.edge_off[g]), int(b.edge_off[g + 1])
        views.append((rp[a + g:z + g + 1], col[e0:e1], plain[a:z]))

    def plain_all():
        for g in range(G):
            grp, gcol, out = views[g]
            gc.init_color(grp, gcol, gc.RANDOM_X, X, seeds[g], out=out, stats=False, ctx=ctx)
            for p in range(passes):
                gc.recolor(grp, gcol, out, gc.PERM_REVERSE, seeds[g], p, out=out, stats=False, ctx=ctx)

    torch.cuda.synchronize()
    t0 = time.perf_counter()
    plain_all()
    torch.cuda.synchronize()
    t_p = time.perf_counter() - t0
    identical = bool(torch.equal(plain, colors))
    log(f"[bench] plain: {t_p:.2f} s, {G / t_p:.0f} graphs/s; identical={identical}")
    m_tot = nnz_tot // 2
    # algorithmic bytes of one launch, a lower bound: round 0 of every graph
    # (16 per entry + 28 per vertex) and its passes (8 per entry + 12 per
    # vertex each); later rounds of the initial colorings are not counted
    batch_bytes = 16 * nnz_tot + 28 * n_tot + passes * (8 * nnz_tot + 12 * n_tot)
    out = {
        "metric": "graphs/s (batched)", "value": round(G / t_b, 2), "unit": "graphs/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(t_b * 1e3, 3), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "int32", "data": "synthetic",
        "config": {"workload": f"{G} random geometric graphs, n uniform in [500, 50000], target degree uniform in "
                               f"[8, 40], Random-X (X=4) + {passes} reverse-order recoloring passes each",
                   "graphs": G, "n": n_tot, "nnz": nnz_tot, "m": m_tot, "seed": args.seed, "tuning": ctx.tuning,
                   "autotuned": tuned},
        "gteps_batched": round(m_tot * (passes + 1) / t_b / 1e9, 3),
        "plain": {"graphs_per_s": round(G / t_p, 2), "seconds": round(t_p, 3),
                  "gteps": round(m_tot * (passes + 1) / t_p / 1e9, 3)},
        "speedup_vs_plain": round(t_p / t_b, 2),
        "roofline": {"kernel": "k_batch (whole method per graph, one launch)", "bound": "hbm",
                     "achieved": round(batch_bytes / t_b / 1e9, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(batch_bytes / t_b / 1e9 / HBM_PEAK_GBS, 4), "traffic": None,
                     "bytes_per_launch": batch_bytes, "avg_launch_ms": round(t_b * 1e3, 3),
                     "bytes_note": "lower bound: initial-coloring rounds after the first not counted"},
        "identical_to_plain": identical,
        "all_converged": bool((pg[:, 3] == 0).all()),
        "colors_final": {"min": int(pg[:, 2].min()), "mean": round(float(pg[:, 2].mean()), 3),
                         "max": int(pg[:, 2].max())},
        "rounds": {"mean": round(float(pg[:, 0].mean()), 3), "max": int(pg[:, 0].max())},
    }
    if not args.no_cpu_baseline:
        log("[bench] cpu baseline (oracle) ...")
        out["cpu_baseline"] = batch_cpu_baseline(b, X, passes, args.seed)
        log("[bench] cpu baseline on all host cores (oracle) ...")
        out["cpu_baseline_all_cores"] = batch_cpu_baseline_all_cores(b, X, passes, args.seed)
    else:
        out["cpu_baseline"] = None
    return out


def run_d2(args):
    """Distance-2 coloring of the 27-point mesh 128^3 (the column coloring that
    compresses a sparse Jacobian or Hessian with that stencil pattern)."""
    import torch

    import gen
    import paper_1407_6745_amd as gc

    X, passes, perm = 4, 5, gc.PERM_NONINC
    t0 = time.perf_counter()
    g = gen.mesh27(128)
    deg = g.degrees
    two_hop = int(deg.sum() + (deg[g.col].astype(np.int64)).sum())  # entries one sweep over N2 visits
    log(f"[bench] mesh27_128 distance-2: n={g.n} nnz={g.nnz} two-hop entries per sweep={two_hop} "
        f"({time.perf_counter() - t0:.1f}s)")
    dev = torch.device("cuda:0")
    rp = torch.from_numpy(g.row_ptr).to(dev)
    col = torch.from_numpy(g.col).to(dev)
    colors = torch.empty(g.n, dtype=torch.int32, device=dev)
    ctx = gc.Context(g.n, g.nnz)
    if args.tune:
        ctx.set_tuning(**{k: int(v) for k, v in (kv.split("=") for kv in args.tune.split(","))})
    flags = gc.FLAG_DISTANCE2

    def step(stats=False):
        c, s0 = gc.init_color(rp, col, gc.RANDOM_X, X, args.seed, flags=flags, out=colors, stats=stats, ctx=ctx)
        hist = [s0]
        for p in range(passes):
            c, sp = gc.recolor_d2(rp, col, c, perm, args.seed, p, out=c, stats=stats, ctx=ctx)
            hist.append(sp)
        return c, hist

    c, hist = step(stats=True)
    conflicts, uncolored = gc.validate_d2(rp, col, c, ctx=ctx)
    colors_trace = [h["num_colors"] for h in hist]
    rounds, round_sizes = hist[0]["rounds"], hist[0]["round_sizes"]
    log(f"[bench] colors {colors_trace} rounds={rounds} valid={(conflicts, uncolored) == (0, 0)}")
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(passes + 2)]
    ev[0].record(stream)
    gc.init_color(rp, col, gc.RANDOM_X, X, args.seed, flags=flags, out=colors, stats=False, ctx=ctx)
    ev[1].record(stream)
    for p in range(passes):
        gc.recolor_d2(rp, col, colors, perm, args.seed, p, out=colors, stats=False, ctx=ctx)
        ev[p + 2].record(stream)
    torch.cuda.synchronize()
    t_init = ev[0].elapsed_time(ev[1])
    t_pass = [ev[p + 1].elapsed_time(ev[p + 2]) for p in range(passes)]

    ctx.set_timing(True, kinds=["walk"])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    kt_walk = ctx.timing()
    ctx.set_timing(True)
    step()
    kt = ctx.timing()
    ctx.set_timing(False)
    ms_step = el / args.steps * 1e3
    m = g.nnz // 2
    value = m * (passes + 1) / (ms_step / 1e3) / 1e9
    # the class kernels of one pass sweep N2 once: two_hop entries, each a
    # col_idx word and a color word, plus one row-pointer pair per neighbor slot
    launches, walk_ms = kt_walk["walk"]
    sweep_ms = walk_ms / (args.steps * passes)
    sweep_bytes = 8 * two_hop + 8 * g.nnz + 8 * g.n
    out = {
        "metric": "GTEPS/pass", "value": round(value, 3), "unit": "GTEPS", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms_step, 4), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "int32", "data": "synthetic",
        "config": {"workload": "3D 27-point mesh 128^3, distance-2 coloring: Random-X (X=4) initial coloring + "
                               "5 NI recoloring passes", "n": g.n, "nnz": g.nnz, "m": m, "passes": passes,
                   "two_hop_entries_per_sweep": two_hop, "seed": args.seed, "tuning": ctx.tuning},
        "colors": {"init": colors_trace[0], "after_pass": colors_trace[1:]},
        "valid_distance2": (conflicts, uncolored) == (0, 0),
        "init": {"rounds": rounds, "round_sizes": round_sizes, "ms": round(t_init, 4)},
        "recolor_pass": {"ms": [round(t, 4) for t in t_pass], "mean_ms": round(sum(t_pass) / passes, 4),
                         "class_kernels_ms": round(sweep_ms, 4),
                         "two_hop_entries_per_s": round(two_hop / (sweep_ms / 1e3), 1),
                         "gather_bytes": sweep_bytes,
                         "gather_gbs": round(sweep_bytes / (sweep_ms / 1e3) / 1e9, 1)},
        "kernel_ms_one_step": {k: {"launches": v[0], "total_ms": round(v[1], 4)} for k, v in kt.items() if v[0]},
        "cpu_baseline": None,
    }
    return out


def pct(xs, q):
    return float(np.percentile(np.asarray(xs, dtype=np.float64), q)) if len(xs) else None


def run_serve(args):
    """Open-loop serving run: Poisson arrivals at a fixed fraction of the
    saturated throughput, requests admitted by footprint into a device arena."""
    import threading

    import torch

    import gen
    import paper_1407_6745_amd as gc

    X, passes = 4, 3
    t0 = time.perf_counter()
    pool = gen.serve_pool(args.pool, args.seed)
    log(f"[bench] serve pool: {len(pool)} graphs, n {min(g.n for g in pool)}..{max(g.n for g in pool)}, "
        f"nnz {min(g.nnz for g in pool)}..{max(g.nnz for g in pool)} ({time.perf_counter() - t0:.1f}s)")
    max_n, max_nnz = max(g.n for g in pool), max(g.nnz for g in pool)
    budget = int(args.budget_gib * (1 << 30))
    budget = max(budget, max(gc.request_footprint(g.n, g.nnz) for g in pool))

    def closed_loop(slots, reqs):
        srv = gc.Server(slots=slots, hbm_budget=budget, max_n=max_n, max_nnz=max_nnz)
        for gi in range(len(pool)):  # warm-up: every graph once
            srv.submit(pool[gi].row_ptr, pool[gi].col, gc.RANDOM_X, X, gc.PERM_REVERSE, passes, 1, tag=10**9 + gi)
        got = 0
        while got < len(pool):
            got += len(srv.poll(timeout_ms=60000))
        ts = srv.now()
        for k, (gi, sd) in enumerate(reqs):
            srv.submit(pool[gi].row_ptr, pool[gi].col, gc.RANDOM_X, X, gc.PERM_REVERSE, passes, sd, tag=k)
        res = []
        while len(res) < len(reqs):
            res += srv.poll(timeout_ms=60000)
        te = max(d["t_done"] for d in res)
        srv.close()
        return len(reqs) / (te - ts), res

    # saturated throughput (queue never empty) with all slots, and one slot (requests one after another)
    rng = np.random.default_rng(args.seed)
    sat_reqs = [(int(rng.integers(0, len(pool))), int(rng.integers(1, 2**62))) for _ in range(min(4 * len(pool), 256))]
    sat, _ = closed_loop(args.slots, sat_reqs)
    sat1, _ = closed_loop(1, sat_reqs)
    log(f"[bench] saturated: {sat:.1f} req/s with {args.slots} slots, {sat1:.1f} req/s with one slot")

    lam = args.load * sat
    R = int(min(args.requests, max(50, 60.0 * lam)))
    arr, which, seeds = gen.serve_trace(R, len(pool), lam, args.seed)
    srv = gc.Server(slots=args.slots, hbm_budget=budget, max_n=max_n, max_nnz=max_nnz)
    for gi in range(len(pool)):
        srv.submit(pool[gi].row_ptr, pool[gi].col, gc.RANDOM_X, X, gc.PERM_REVERSE, passes, 1, tag=10**9 + gi)
    warm = 0
    while warm < len(pool):
        warm += len(srv.poll(timeout_ms=60000))
    results = []

    def collector():
        while len(results) < R:
            results.extend(srv.poll(timeout_ms=1000))

    th = threading.Thread(target=collector)
    th.start()
    base = srv.now()
    arrival = {}
    for k in range(R):
        due = base + float(arr[k])
        while True:
            dt = due - srv.now()
            if dt <= 0:
                break
            time.sleep(min(dt, 0.002))
        arrival[k] = due
        g = pool[int(which[k])]
        srv.submit(g.row_ptr, g.col, gc.RANDOM_X, X, gc.PERM_REVERSE, passes, int(seeds[k]), tag=k)
    th.join()
    st = srv.stats()
    srv.close()
    makespan = max(d["t_done"] for d in results) - base
    lat = [(d["t_done"] - arrival[d["tag"]]) * 1e3 for d in results]
    queue = [(d["t_admit"] - arrival[d["tag"]]) * 1e3 for d in results]
    dev = [d["device_ms"] for d in results]
    service = [(d["t_done"] - d["t_admit"]) * 1e3 for d in results]
    ok = all(d["status"] == 0 for d in results)
    if args.dump:
        with open(args.dump, "w") as f:
            for d in results:
                g = pool[int(which[d["tag"]])]
                rec = {k: v for k, v in d.items() if k != "colors"}
                rec.update(graph=g.name, n=g.n, nnz=g.nnz, arrival=arrival[d["tag"]])
                f.write(json.dumps(rec) + "\n")

    # alone == in the mix: plain single-graph calls on a sample of the requests
    by_tag = {d["tag"]: d for d in results}
    sample = list(range(0, R, max(1, R // 32)))
    same = True
    d0 = torch.device("cuda:0")
    for k in sample:
        g = pool[int(which[k])]
        rp = torch.from_numpy(g.row_ptr).to(d0)
        col = torch.from_numpy(g.col).to(d0)
        c, _ = gc.init_color(rp, col, gc.RANDOM_X, X, int(seeds[k]), stats=False)
        for p in range(passes):
            c, _ = gc.recolor(rp, col, c, gc.PERM_REVERSE, int(seeds[k]), p, out=c, stats=False)
        same &= bool(np.array_equal(c.cpu().numpy(), by_tag[k]["colors"]))
    edges = sum(pool[int(which[k])].m for k in range(R))
    log(f"[bench] open loop: {R} requests at {lam:.1f} req/s, p50 {pct(lat, 50):.2f} ms, p99 {pct(lat, 99):.2f} ms")
    out = {
        "metric": "served requests/s at a fixed offered load (p50/p99 latency)", "value": round(R / makespan, 3),
        "unit": "requests/s", "n_gpus": 1, "steps": R, "warmup": len(pool), "ms_per_step": round(makespan / R * 1e3, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "int32", "data": "synthetic",
        "config": {"workload": f"Poisson arrivals of coloring requests over {len(pool)} graphs (2D 5-point grids side "
                               f"32..2048, Erdos-Renyi n 1e3..1e6 avg degree 4..32, RMAT scale 10..20 ef 16), "
                               f"Random-X (X=4) + {passes} reverse-order recoloring passes each",
                   "requests": R, "pool": len(pool), "slots": args.slots, "hbm_budget": budget, "seed": args.seed,
                   "offered_load_req_s": round(lam, 3), "load_fraction_of_saturation": args.load},
        "latency_ms": {"p50": round(pct(lat, 50), 3), "p99": round(pct(lat, 99), 3), "mean": round(float(np.mean(lat)), 3)},
        "queueing_ms": {"p50": round(pct(queue, 50), 3), "p99": round(pct(queue, 99), 3)},
        "device_ms": {"p50": round(pct(dev, 50), 3), "p99": round(pct(dev, 99), 3)},
        "service_ms": {"p50": round(pct(service, 50), 3), "p99": round(pct(service, 99), 3)},
        "saturated_req_s": {"slots": round(sat, 3), "one_slot": round(sat1, 3), "speedup": round(sat / sat1, 3)},
        "served_gteps": round(edges * (passes + 1) / makespan / 1e9, 4),
        "peak_running": st["peak_running"], "arena_peak": st["arena_peak"],
        "mean_running_at_admit": round(float(np.mean([d["running_at_admit"] for d in results])), 3),
        "all_ok": ok, "identical_to_plain": same, "checked": len(sample),
        "cpu_baseline": None,
    }
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="mesh128", choices=sorted(WORKLOADS) + ["batch4096", "serve", "mesh128d2"])
    ap.add_argument("--graphs", type=int, default=4096, help="batch4096: number of graphs")
    ap.add_argument("--requests", type=int, default=2000, help="serve: requests in the arrival trace")
    ap.add_argument("--pool", type=int, default=48, help="serve: distinct request graphs")
    ap.add_argument("--slots", type=int, default=8, help="serve: requests in flight at once")
    ap.add_argument("--budget-gib", type=float, default=2.0, help="serve: device arena for request graphs (GiB)")
    ap.add_argument("--load", type=float, default=0.7, help="serve: offered load as a fraction of saturation")
    ap.add_argument("--dump", default="", help="serve: write one JSON record per request to this file")
    ap.add_argument("--seed", type=int, default=1)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--tune", default="", help="comma list key=value of library tuning knobs")
    ap.add_argument("--no-autotune", action="store_true", help="batch4096: keep the default batch tuning")
    ap.add_argument("--method", default="rc", choices=("rc", "arc"),
                    help="recoloring: synchronous class walk (rc) or asynchronous speculative rounds (arc)")
    ap.add_argument("--schedule", default="fixed", choices=("fixed", "ndrand5", "ndrand10", "ndrand2i"),
                    help="class order per pass: the workload's fixed order, or a hybrid ND/RAND schedule")
    ap.add_argument("--no-sub", action="store_true",
                    help="mesh128: skip the RMAT-22, batch and serving sub-records of the default line")
    ap.add_argument("--sub-steps", type=int, default=5, help="timed steps of the RMAT-22 and batch sub-records")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="only run a plain device-to-device copy of MIB MiB three times (counter calibration)")
    args = ap.parse_args()
    if args.calibrate_copy:
        import torch

        a = torch.ones(args.calibrate_copy * 2**18, dtype=torch.int32, device="cuda")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        log(f"[bench] copied {args.calibrate_copy} MiB three times")
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}): the coloring of one graph here is a "
              "single-GPU kernel pipeline; sharding across GPUs is not built.", file=sys.stderr)
        sys.exit(2)

    if args.workload == "batch4096":
        out = run_batch(args)
    elif args.workload == "serve":
        out = run_serve(args)
    elif args.workload == "mesh128d2":
        out = run_d2(args)
    else:
        out = run_graph(args, args.workload)
        if args.workload == "mesh128" and not args.no_sub:
            # the other targets of the benchmark, one record each beside the headline
            out["sub_workloads"] = run_sub_workloads(args)
    print(json.dumps(out), flush=True)


def run_sub_workloads(args):
    import copy

    import torch

    subs = {}
    for name, fn in (("rmat22", lambda a: run_graph(a, "rmat22")), ("batch4096", run_batch), ("serve", run_serve)):
        a = copy.copy(args)
        a.workload, a.tune = name, ""
        a.steps, a.warmup = (args.sub_steps, 1) if name != "serve" else (args.steps, args.warmup)
        t0 = time.perf_counter()
        log(f"[bench] sub-workload {name} ...")
        try:
            rec = fn(a)
        except Exception as e:  # a failing sub-record must not hide the headline
            rec = {"error": f"{type(e).__name__}: {e}"}
        rec["wall_s"] = round(time.perf_counter() - t0, 1)
        subs[name] = rec
        torch.cuda.synchronize()
        torch.cuda.empty_cache()
    return subs


def run_graph(args, workload):
    import torch

    import gen
    import paper_1407_6745_amd as gc

    desc, build, select, X, perm, passes = WORKLOADS[workload]
    sel = getattr(gc, select)
    pm = gc.PERM_NAMES[perm]
    t0 = time.perf_counter()
    g = build(gen)
    log(f"[bench] graph {workload}: n={g.n} nnz={g.nnz} max_deg={g.max_deg} ({time.perf_counter() - t0:.1f}s)")
    dev = torch.device("cuda:0")
    rp = torch.from_numpy(g.row_ptr).to(dev)
    col = torch.from_numpy(g.col).to(dev)
    colors = torch.empty(g.n, dtype=torch.int32, device=dev)
    ctx = gc.Context(g.n, g.nnz)
    if args.tune:
        ctx.set_tuning(**{k: int(v) for k, v in (kv.split("=") for kv in args.tune.split(","))})
    stream = torch.cuda.current_stream()

    sched = {"fixed": (gc.SCHED_FIXED, 0), "ndrand5": (gc.SCHED_ND_RAND_X, 5), "ndrand10": (gc.SCHED_ND_RAND_X, 10),
             "ndrand2i": (gc.SCHED_ND_RAND_POW2, 0)}[args.schedule]
    perms = [gc.schedule_perm(sched[0], pm, sched[1], p + 1) for p in range(passes)]
    recolor_fn = gc.recolor if args.method == "rc" else gc.arc_recolor

    def recolor_all(c, stats=False):
        """The step's passes: one gc_recolor_passes call (synchronous
        recoloring), or one call per pass (asynchronous recoloring)."""
        if args.method == "rc":
            c, sts = gc.recolor_passes(rp, col, c, perms, args.seed, 0, out=c, stats=stats, ctx=ctx)
            return c, sts if sts is not None else [None] * passes
        sts = []
        for p in range(passes):
            c, sp = recolor_fn(rp, col, c, perms[p], args.seed, p, out=c, stats=stats, ctx=ctx)
            sts.append(sp)
        return c, sts

    def step(stats=False):
        c, s0 = gc.init_color(rp, col, sel, X, args.seed, out=colors, stats=stats, ctx=ctx)
        c, sts = recolor_all(c, stats)
        return c, [s0] + sts

    # untimed: statistics run (color counts after the initial coloring and after each pass, rounds)
    c, hist = step(stats=True)
    conflicts, uncolored = gc.validate(rp, col, c, ctx=ctx)
    colors_trace = [h["num_colors"] for h in hist]
    rounds = hist[0]["rounds"]
    round_sizes = hist[0]["round_sizes"]
    round_degsum = hist[0]["round_degsum"]
    log(f"[bench] colors {colors_trace} rounds={rounds} valid={(conflicts, uncolored) == (0, 0)}")

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()

    # per-phase split (one instrumented step, events on the launch stream):
    # the initial coloring, then the step's passes as the step runs them
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
    ev[0].record(stream)
    gc.init_color(rp, col, sel, X, args.seed, out=colors, stats=False, ctx=ctx)
    ev[1].record(stream)
    recolor_all(colors)
    ev[2].record(stream)
    torch.cuda.synchronize()
    t_init = ev[0].elapsed_time(ev[1])
    t_all_passes = ev[1].elapsed_time(ev[2])
    # the same passes one call each (every pass lays its classes out anew)
    gc.init_color(rp, col, sel, X, args.seed, out=colors, stats=False, ctx=ctx)
    evs = [torch.cuda.Event(enable_timing=True) for _ in range(passes + 1)]
    evs[0].record(stream)
    for p in range(passes):
        recolor_fn(rp, col, colors, perms[p], args.seed, p, out=colors, stats=False, ctx=ctx)
        evs[p + 1].record(stream)
    torch.cuda.synchronize()
    t_pass = [evs[p].elapsed_time(evs[p + 1]) for p in range(passes)]

    # timed region: K whole steps; HIP events around the walk launches only
    # (the roofline kernel), so that timing adds no host work elsewhere
    ctx.set_timing(True, kinds=["walk"])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    kt_walk = ctx.timing()
    # per-kernel breakdown: one more step with every kind timed (outside the timed region)
    ctx.set_timing(True)
    step()
    kt = ctx.timing()
    c_step = colors.clone()  # one whole step's colors (the CPU baseline compares against them)
    # passes after a 1 GiB scrub write (L2 and Infinity Cache hold other data
    # when each pass starts): pass time and walk time, outside the timed region;
    # they recolor the step's result further, so they work on a copy
    colors = c_step.clone()
    scrub = torch.empty(1 << 28, dtype=torch.int32, device=dev)
    ctx.set_timing(True, kinds=["walk"])
    cold = []
    for p in range(min(passes, 5)):
        scrub.fill_(p + 1)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        recolor_fn(rp, col, colors, perms[p], args.seed, p, out=colors, stats=False, ctx=ctx)
        e1.record(stream)
        torch.cuda.synchronize()
        cold.append(e0.elapsed_time(e1))
    kt_cold = ctx.timing()
    ctx.set_timing(False)
    del scrub
    # the validation kernel (section 1's condition) on the step's colors, timed alone
    ev_v = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    vt = []
    for _ in range(3):
        ev_v[0].record(stream)
        gc.validate(rp, col, c_step, ctx=ctx)
        ev_v[1].record(stream)
        torch.cuda.synchronize()
        vt.append(ev_v[0].elapsed_time(ev_v[1]))
    validate_ms = min(vt)
    validate_bytes = 8 * g.nnz + 8 * g.n + 4  # col_idx + neighbor colors + row_ptr + own color
    # one traced pass (outside the timed region): when each class finished
    ctx.set_tuning(trace=1)
    colors = c_step.clone()
    recolor_fn(rp, col, colors, perms[0], args.seed, 0, out=colors, stats=False, ctx=ctx)
    walk_trace = None
    if args.method == "rc":
        tr = ctx.walk_trace()
        done = np.asarray(tr["class_done"], np.float64) / 1e3
        split = np.asarray(tr["split_done"], np.float64) / 1e3
        gaps = np.diff(np.concatenate([[0.0], np.maximum.accumulate(done)]))
        walk_trace = {"classes": int(done.size), "walk_us": round(tr["end"] / 1e3, 2),
                      "last_class_done_us": round(float(done.max()), 2) if done.size else 0.0,
                      "class_gap_us": {"median": round(float(np.median(gaps)), 3) if done.size else 0.0,
                                       "p90": round(float(np.percentile(gaps, 90)), 3) if done.size else 0.0,
                                       "max": round(float(gaps.max()), 3) if done.size else 0.0},
                      "classes_with_split_rows": int((split > 0).sum()),
                      "split_row_finishes_class": int(((split > 0) & (split >= done)).sum()),
                      "class_done_us": [round(float(x), 2) for x in done[:512]]}
    ctx.set_tuning(trace=0)
    ms_step = el / args.steps * 1e3
    m = g.nnz // 2
    value = m * (passes + 1) / (ms_step / 1e3) / 1e9

    dom = max(kt, key=lambda k: kt[k][1])
    walk_launches, walk_ms = kt_walk["walk"]
    walk_avg_ms = walk_ms / max(walk_launches, 1)
    walk_bytes = 8 * g.nnz + 8 * g.n + 4  # col_idx + neighbor-color gather + row_ptr + color write
    pass_bytes = 8 * g.nnz + 12 * g.n + 4
    achieved = walk_bytes / (walk_avg_ms / 1e3) / 1e9 if walk_launches else 0.0
    roofline = {"kernel": "k_walk_flow (recoloring class walk)", "bound": "hbm", "achieved": round(achieved, 1),
                "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                "traffic": recorded_traffic(workload, ctx.tuning),
                "bytes_per_launch": walk_bytes, "avg_launch_ms": round(walk_avg_ms, 5), "launches": walk_launches,
                "dominant_kind": dom}
    out = {
        "metric": "GTEPS/pass", "value": round(value, 3), "unit": "GTEPS", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms_step, 4), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "int32", "data": "synthetic",
        "config": {"workload": desc, "n": g.n, "nnz": g.nnz, "m": m, "passes": passes, "X": X, "select": select,
                   "perm": perm, "method": args.method, "schedule": args.schedule, "seed": args.seed,
                   "tuning": ctx.tuning, "launch": ctx.info()},
        "colors": {"init": colors_trace[0], "after_pass": colors_trace[1:]},
        "valid": (conflicts, uncolored) == (0, 0),
        "init": {"rounds": rounds, "round_sizes": round_sizes, "round_degsum": round_degsum, "ms": round(t_init, 4),
                 "gteps": round(m / (t_init / 1e3) / 1e9, 3)},
        "recolor_pass": {"mean_ms": round(t_all_passes / passes, 4),
                         "gteps": round(m / (t_all_passes / passes / 1e3) / 1e9, 3),
                         "entries_per_s": round(g.nnz / (t_all_passes / passes / 1e3), 1),
                         "algorithmic_bytes": pass_bytes,
                         "gbs": round(pass_bytes / (t_all_passes / passes / 1e3) / 1e9, 1),
                         "one_call_per_pass_ms": [round(t, 4) for t in t_pass],
                         "one_call_per_pass_mean_ms": round(sum(t_pass) / passes, 4)},
        "recolor_pass_after_scrub": {
            "scrub_bytes": 1 << 30, "passes": len(cold), "mean_ms": round(sum(cold) / len(cold), 4),
            "walk_avg_ms": round(kt_cold["walk"][1] / max(kt_cold["walk"][0], 1), 5),
            "walk_gbs": round(walk_bytes / (kt_cold["walk"][1] / max(kt_cold["walk"][0], 1) / 1e3) / 1e9, 1)
            if kt_cold["walk"][0] else None},
        "kernel_ms_one_step": {k: {"launches": v[0], "total_ms": round(v[1], 4)} for k, v in kt.items() if v[0]},
        "walk_trace_one_pass": walk_trace,
        "validate": {"ms": round(validate_ms, 4), "algorithmic_bytes": validate_bytes,
                     "frac_of_peak": round(validate_bytes / (validate_ms / 1e3) / 1e9 / HBM_PEAK_GBS, 4),
                     "note": "gc_validate call incl. its scalar resets and read-back, events on the stream"},
        "roofline": roofline,
    }
    # the initial coloring against its algorithmic bytes (16 per scanned entry
    # + 28 per vertex of each round, from the round statistics)
    init_bytes = sum(16 * d + 28 * w for w, d in zip(round_sizes, round_degsum))
    out["init"]["algorithmic_bytes"] = init_bytes
    out["init"]["frac_of_peak"] = round(init_bytes / (t_init / 1e3) / 1e9 / HBM_PEAK_GBS, 4)
    out["recolor_pass"]["frac_of_peak"] = round(out["recolor_pass"]["gbs"] / HBM_PEAK_GBS, 4)
    if not args.no_cpu_baseline:
        log("[bench] cpu baseline (oracle) ...")
        cb, cref, k = cpu_baseline(g, select, X, perms, passes, args.seed, args.method)
        if k < passes:  # the GPU's colors after the same passes
            gc.init_color(rp, col, sel, X, args.seed, out=colors, stats=False, ctx=ctx)
            for p in range(k):
                recolor_fn(rp, col, colors, perms[p], args.seed, p, out=colors, stats=False, ctx=ctx)
            c_step = colors.clone()
        cb["matches_gpu"] = bool(np.array_equal(cref, c_step.cpu().numpy()))
        out["cpu_baseline"] = cb
    else:
        out["cpu_baseline"] = None
    ctx.raise_status()
    ctx.close()
    return out


if __name__ == "__main__":
    main()
