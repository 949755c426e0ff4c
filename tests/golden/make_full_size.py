"""Writes tests/golden/full_size.json: the oracle's results on the full-size
workloads, as SHA-256 digests of the color arrays plus the round and color
statistics, so that GPU tests can compare whole colorings at full size
without running the oracle where the GPU tests run.

Calls only gen/ (inputs) and oracle/ (expected values).  Run from the
repository root:  python tests/golden/make_full_size.py [--only NAME ...]
(--only recomputes the named entries: workload names, "batch", and keeps
the others from the existing file).
"""
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import gen  # noqa: E402
import oracle  # noqa: E402

PERMS = {"RV": oracle.PERM_REVERSE, "NI": oracle.PERM_NONINC, "ND": oracle.PERM_NONDEC, "RAND": oracle.PERM_RANDOM}

# name: (graph builder expression, select, X, seed, class order, passes)
WORKLOADS = {
    "er10k": ("gen.er(10000, 50000, 1)", "FIRST_FIT", 1, 1, "RV", 3),
    "mesh128": ("gen.mesh27(128)", "RANDOM_X", 4, 1, "NI", 10),
    "rmat22": ("gen.rmat(22, 16, 0.57, 0.19, 0.19, 1)", "FIRST_FIT", 1, 1, "RAND", 10),
}
# distance-2 workloads (section 1's distance-k problem, k = 2): the oracle's
# distance-1 routines on the square graph
WORKLOADS_D2 = {
    "mesh128d2": ("gen.mesh27(128)", "RANDOM_X", 4, 1, "NI", 5),
}
# sampled graphs of the 4096-graph batch of random geometric graphs (seed 1):
# Random-X X=4 + 5 RV passes with the graph's own seed
BATCH_SAMPLE = [0, 1, 2, 511, 1024, 2047, 3071, 4095]


def digest(a):
    return hashlib.sha256(np.ascontiguousarray(a, dtype="<i4").tobytes()).hexdigest()


def run(g, select, X, seed, perm, passes, dist=1):
    sel = oracle.FIRST_FIT if select == "FIRST_FIT" else oracle.RANDOM_X
    sq = oracle.square(g) if dist == 2 else None
    ini = oracle.init_color_d2(g, sel, X, seed, sq=sq) if dist == 2 else oracle.init_color(g, sel, X, seed)
    out = {"n": g.n, "nnz": g.nnz, "graph_sha256": gen.checksum(g), "select": select, "X": X, "seed": seed,
           "perm": perm, "passes": passes,
           "init": {"rounds": ini.rounds, "round_sizes": ini.w_sizes.tolist(), "round_degsum": ini.w_degsum.tolist(),
                    "num_colors": ini.stats["num_colors"], "max_color": ini.stats["max_color"],
                    "sha256": digest(ini.colors)},
           "passes_out": []}
    c = ini.colors
    for p in range(passes):
        r = oracle.recolor_d2(g, c, PERMS[perm], seed, p, sq=sq) if dist == 2 else oracle.recolor(g, c, PERMS[perm], seed, p)
        assert r.status == 0
        out["passes_out"].append({"k": len(r.pi), "num_colors": r.stats["num_colors"], "sha256": digest(r.colors)})
        c = r.colors
    return out


def main():
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "full_size.json")
    only = set(sys.argv[sys.argv.index("--only") + 1:]) if "--only" in sys.argv else None
    res = {"note": "oracle results; regenerate with python tests/golden/make_full_size.py", "workloads": {},
           "workloads_d2": {},
           "batch": {"G": 4096, "seed": 1, "select": "RANDOM_X", "X": 4, "perm": "RV", "passes": 5, "graphs": {}}}
    if only is not None:
        old = json.load(open(path))
        for key in ("workloads", "workloads_d2"):
            res[key].update({k: v for k, v in old.get(key, {}).items() if k not in only})
        if "batch" not in only:
            res["batch"] = old["batch"]
    for key, table, dist in (("workloads", WORKLOADS, 1), ("workloads_d2", WORKLOADS_D2, 2)):
        for name, (expr, select, X, seed, perm, passes) in table.items():
            if only is not None and name not in only:
                continue
            t = time.time()
            g = eval(expr)
            res[key][name] = dict(run(g, select, X, seed, perm, passes, dist), graph=expr)
            print(name, g.n, g.nnz, f"{time.time() - t:.1f}s", flush=True)
    if only is None or "batch" in only:
        b = res["batch"]
        for gi in BATCH_SAMPLE:
            g = gen.rgg_batch_graph(gi, 1)
            sg = oracle.graph_seed(1, gi)
            b["graphs"][str(gi)] = run(g, "RANDOM_X", 4, sg, "RV", 5)
            print("batch graph", gi, g.n, g.nnz, flush=True)
    with open(path, "w") as f:
        json.dump(res, f, indent=1)


if __name__ == "__main__":
    main()
