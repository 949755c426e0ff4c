"""GPU parity at full size: the whole coloring after the initial coloring and
after every recoloring pass, compared with the oracle's results (SHA-256 of
the color array, written by tests/golden/make_full_size.py from oracle/
only), plus rounds, per-round set sizes and color counts.  Also the batched
kernel against plain per-graph calls and against the oracle on sampled graphs
of the random-geometric-graph batch."""
import hashlib
import json
import os
import time

import numpy as np
import pytest

import gen

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "full_size.json")))
PERM = {"RV": 0, "NI": 1, "ND": 2, "RAND": 3}


@pytest.fixture(scope="module")
def gc():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1407_6745_amd as m

    m.lib()
    return m


def digest(t):
    return hashlib.sha256(t.cpu().numpy().astype("<i4").tobytes()).hexdigest()


def check_workload(gc, g, ref, ctx=None):
    assert gen.checksum(g) == ref["graph_sha256"], "generator output differs from the one the oracle saw"
    d = torch.device("cuda:0")
    rp = torch.from_numpy(g.row_ptr).to(d)
    col = torch.from_numpy(g.col).to(d)
    sel = gc.FIRST_FIT if ref["select"] == "FIRST_FIT" else gc.RANDOM_X
    c, st = gc.init_color(rp, col, sel, ref["X"], ref["seed"], round_cap=8192, ctx=ctx)
    ri = ref["init"]
    assert st["rounds"] == ri["rounds"]
    assert st["round_sizes"] == ri["round_sizes"]
    assert st["round_degsum"] == ri["round_degsum"]
    assert (st["num_colors"], st["max_color"]) == (ri["num_colors"], ri["max_color"])
    assert digest(c) == ri["sha256"], "initial coloring differs from the oracle"
    for p, rp_ in enumerate(ref["passes_out"]):
        c, sp = gc.recolor(rp, col, c, PERM[ref["perm"]], ref["seed"], p, out=c, ctx=ctx)
        assert sp["k_classes"] == rp_["k"] and sp["num_colors"] == rp_["num_colors"], p
        assert digest(c) == rp_["sha256"], f"pass {p} differs from the oracle"
    assert gc.validate(rp, col, c, ctx=ctx) == (0, 0)


@pytest.mark.parametrize("name", sorted(GOLD["workloads"]))
def test_full_size_workload(gc, name):
    ref = GOLD["workloads"][name]
    print(f"[full-size] {name}: {ref['graph']}", flush=True)
    g = eval(ref["graph"])
    check_workload(gc, g, ref)


def test_full_size_workload_other_tunings(gc):
    """The mesh at full size under non-default launch shapes (same colors)."""
    ref = GOLD["workloads"]["mesh128"]
    g = eval(ref["graph"])
    for t in (dict(group=8, xcd_chunks=1), dict(group=16, walk_group=16, deg_wave=8), dict(walk_group=4),
              dict(walk_mode=1)):
        print(f"[full-size] mesh128 tuning {t}", flush=True)
        ctx = gc.Context(g.n, g.nnz)
        ctx.set_tuning(**t)
        check_workload(gc, g, ref, ctx)
        ctx.close()


def test_batch_prefix_vs_plain_and_oracle(gc):
    """First 48 graphs of the RGG batch: one batched launch == plain per-graph
    calls with the graph's seed == the oracle on the sampled graph ids."""
    B = GOLD["batch"]
    G = 48
    b = gen.rgg_batch(G, B["seed"])
    d = torch.device("cuda:0")
    vo = torch.from_numpy(b.vtx_off).to(d)
    eo = torch.from_numpy(b.edge_off).to(d)
    rp = torch.from_numpy(b.row_ptr).to(d)
    col = torch.from_numpy(b.col).to(d)
    colors, per = gc.batch_color(vo, eo, rp, col, gc.RANDOM_X, B["X"], PERM[B["perm"]], B["passes"], B["seed"])
    torch.cuda.synchronize()
    per = per.cpu().numpy()
    assert (per[:, 3] == 0).all()
    for gi in range(G):
        a, z = int(b.vtx_off[gi]), int(b.vtx_off[gi + 1])
        cg = colors[a:z]
        sub = b.graph(gi)
        srp = torch.from_numpy(sub.row_ptr).to(d)
        scol = torch.from_numpy(sub.col).to(d)
        seed = gc.batch_graph_seed(B["seed"], gi)
        c, s0 = gc.init_color(srp, scol, gc.RANDOM_X, B["X"], seed)
        assert per[gi, 0] == s0["rounds"] and per[gi, 1] == s0["num_colors"], gi
        for p in range(B["passes"]):
            c, sp = gc.recolor(srp, scol, c, PERM[B["perm"]], seed, p, out=c)
        assert per[gi, 2] == sp["num_colors"], gi
        assert torch.equal(cg, c), f"graph {gi}: batched != plain"
        ref = B["graphs"].get(str(gi))
        if ref is not None:
            assert gen.checksum(sub) == ref["graph_sha256"]
            assert digest(c) == ref["passes_out"][-1]["sha256"], f"graph {gi}: differs from the oracle"
            assert per[gi, 0] == ref["init"]["rounds"]


@pytest.mark.parametrize("name", sorted(GOLD.get("workloads_d2", {})))
def test_full_size_workload_d2(gc, name):
    """The distance-2 benchmark configuration at full size against the
    oracle's distance-1 routines on the square graph: the coloring after the
    initial coloring and after every pass, rounds, per-round set sizes and
    color counts."""
    ref = GOLD["workloads_d2"][name]
    print(f"[full-size] {name}: {ref['graph']} distance 2", flush=True)
    g = eval(ref["graph"])
    assert gen.checksum(g) == ref["graph_sha256"]
    d = torch.device("cuda:0")
    rp = torch.from_numpy(g.row_ptr).to(d)
    col = torch.from_numpy(g.col).to(d)
    sel = gc.FIRST_FIT if ref["select"] == "FIRST_FIT" else gc.RANDOM_X
    c, st = gc.init_color(rp, col, sel, ref["X"], ref["seed"], flags=gc.FLAG_DISTANCE2, round_cap=8192)
    ri = ref["init"]
    assert st["rounds"] == ri["rounds"]
    assert st["round_sizes"] == ri["round_sizes"]
    assert (st["num_colors"], st["max_color"]) == (ri["num_colors"], ri["max_color"])
    assert digest(c) == ri["sha256"], "distance-2 initial coloring differs from the oracle"
    for p, rp_ in enumerate(ref["passes_out"]):
        c, sp = gc.recolor_d2(rp, col, c, PERM[ref["perm"]], ref["seed"], p, out=c)
        assert sp["k_classes"] == rp_["k"] and sp["num_colors"] == rp_["num_colors"], p
        assert digest(c) == rp_["sha256"], f"distance-2 pass {p} differs from the oracle"
    assert gc.validate_d2(rp, col, c) == (0, 0)


def _plain_batch(gc, b, rp, col, X, perm, passes, seed, ctx):
    """Every graph of the batch through the single-graph calls (no stats: one
    launch sequence per graph on the same stream), into one packed array."""
    d = torch.device("cuda:0")
    out = torch.zeros(int(b.vtx_off[-1]), dtype=torch.int32, device=d)
    for gi in range(b.num_graphs):
        a, z = int(b.vtx_off[gi]), int(b.vtx_off[gi + 1])
        e0, e1 = int(b.edge_off[gi]), int(b.edge_off[gi + 1])
        grp, gcol, o = rp[a + gi:z + gi + 1], col[e0:e1], out[a:z]
        sg = gc.batch_graph_seed(seed, gi)
        gc.init_color(grp, gcol, gc.RANDOM_X, X, sg, out=o, stats=False, ctx=ctx)
        for p in range(passes):
            gc.recolor(grp, gcol, o, perm, sg, p, out=o, stats=False, ctx=ctx)
    ctx.raise_status()
    return out


@pytest.mark.timeout(900)
def test_full_batch_4096(gc):
    """The whole 4,096-graph batch (packed col_idx of 2.46e9 entries, past
    2^31) in one launch, under the default and the tuned launch settings
    (largest-first order, 2 workgroups per CU): batched == plain per-graph
    calls for every graph, == the oracle's digests and statistics on the
    sampled graphs, every graph converged."""
    B = GOLD["batch"]
    t0 = time.time()
    b = gen.rgg_batch(B["G"], B["seed"])
    assert int(b.edge_off[-1]) > 2**31, "the batch must cross 2^31 packed entries"
    print(f"[full-batch] generated n={int(b.vtx_off[-1])} nnz={int(b.edge_off[-1])} ({time.time() - t0:.1f}s)",
          flush=True)
    d = torch.device("cuda:0")
    vo = torch.from_numpy(b.vtx_off).to(d)
    eo = torch.from_numpy(b.edge_off).to(d)
    rp = torch.from_numpy(b.row_ptr).to(d)
    col = torch.from_numpy(b.col).to(d)
    ns = np.diff(b.vtx_off)
    max_n, max_nnz = int(ns.max()), int(np.diff(b.edge_off).max())
    ctx = gc.Context(max_n, max_nnz)
    perm = PERM[B["perm"]]
    plain = _plain_batch(gc, b, rp, col, B["X"], perm, B["passes"], B["seed"], ctx)
    print(f"[full-batch] plain calls done ({time.time() - t0:.1f}s)", flush=True)
    for tune in ({}, {"batch_order": 1, "batch_wg_per_cu": 2}):
        if tune:
            ctx.set_tuning(**tune)
        colors, per = gc.batch_color(vo, eo, rp, col, gc.RANDOM_X, B["X"], perm, B["passes"], B["seed"],
                                     max_vertices_per_graph=max_n, ctx=ctx)
        ctx.raise_status()
        per = per.cpu().numpy()
        print(f"[full-batch] batched {tune or 'default'} ({time.time() - t0:.1f}s)", flush=True)
        assert (per[:, 3] == 0).all(), "every graph converges"
        assert torch.equal(colors, plain), f"{tune}: batched != plain"
        for gi, ref in B["graphs"].items():
            gi = int(gi)
            a, z = int(b.vtx_off[gi]), int(b.vtx_off[gi + 1])
            assert gen.checksum(b.graph(gi)) == ref["graph_sha256"]
            assert digest(colors[a:z]) == ref["passes_out"][-1]["sha256"], f"graph {gi}: differs from the oracle"
            assert per[gi, 0] == ref["init"]["rounds"] and per[gi, 1] == ref["init"]["num_colors"], gi
            assert per[gi, 2] == ref["passes_out"][-1]["num_colors"], gi
        del colors
    ctx.close()


@pytest.mark.parametrize("name", ["rmat22", "mesh128"])
def test_full_size_no_stats_path(gc, name):
    """The benchmark's call sequence: whole steps without statistics (the
    timed path: no synchronization inside a pass), a traced pass, then the
    initial coloring and every pass again without statistics, each compared
    with the oracle's digest."""
    ref = GOLD["workloads"][name]
    g = eval(ref["graph"])
    d = torch.device("cuda:0")
    rp = torch.from_numpy(g.row_ptr).to(d)
    col = torch.from_numpy(g.col).to(d)
    sel = gc.FIRST_FIT if ref["select"] == "FIRST_FIT" else gc.RANDOM_X
    perm = PERM[ref["perm"]]
    ctx = gc.Context(g.n, g.nnz)
    c = torch.empty(g.n, dtype=torch.int32, device=d)
    for step in range(2):
        gc.init_color(rp, col, sel, ref["X"], ref["seed"], out=c, stats=False, ctx=ctx)
        for p in range(len(ref["passes_out"])):
            gc.recolor(rp, col, c, perm, ref["seed"], p, out=c, stats=False, ctx=ctx)
        ctx.raise_status()
        assert digest(c) == ref["passes_out"][-1]["sha256"], f"step {step}: differs from the oracle"
    ctx.set_tuning(trace=1)
    t = c.clone()
    gc.recolor(rp, col, t, perm, ref["seed"], 0, out=t, stats=False, ctx=ctx)
    tr = ctx.walk_trace()
    assert len(tr["class_done"]) == ref["passes_out"][-1]["num_colors"] and tr["end"] > 0
    assert all(0 < x <= tr["end"] for x in tr["class_done"])
    ctx.set_tuning(trace=0)
    gc.init_color(rp, col, sel, ref["X"], ref["seed"], out=c, stats=False, ctx=ctx)
    assert digest(c) == ref["init"]["sha256"], "initial coloring without statistics"
    for p, rp_ in enumerate(ref["passes_out"]):
        gc.recolor(rp, col, c, perm, ref["seed"], p, out=c, stats=False, ctx=ctx)
        assert digest(c) == rp_["sha256"], f"pass {p} without statistics"
    ctx.raise_status()
    ctx.close()


@pytest.mark.parametrize("name", sorted(GOLD["workloads"]))
def test_full_size_recolor_passes(gc, name):
    """All of a workload's passes in one gc_recolor_passes call (the
    benchmark's step), with and without statistics: the oracle's final colors
    and per-pass color counts."""
    ref = GOLD["workloads"][name]
    print(f"[full-size passes] {name}", flush=True)
    g = eval(ref["graph"])
    d = torch.device("cuda:0")
    rp = torch.from_numpy(g.row_ptr).to(d)
    col = torch.from_numpy(g.col).to(d)
    sel = gc.FIRST_FIT if ref["select"] == "FIRST_FIT" else gc.RANDOM_X
    perms = [PERM[ref["perm"]]] * len(ref["passes_out"])
    ctx = gc.Context(g.n, g.nnz)
    c = torch.empty(g.n, dtype=torch.int32, device=d)
    for stats in (True, False, True):
        gc.init_color(rp, col, sel, ref["X"], ref["seed"], out=c, stats=False, ctx=ctx)
        c, st = gc.recolor_passes(rp, col, c, perms, ref["seed"], 0, out=c, stats=stats, ctx=ctx)
        ctx.raise_status()
        assert digest(c) == ref["passes_out"][-1]["sha256"], f"stats={stats}: differs from the oracle"
        if stats:
            assert [s["num_colors"] for s in st] == [p["num_colors"] for p in ref["passes_out"]]
            assert [s["k_classes"] for s in st] == [p["k"] for p in ref["passes_out"]]
    assert gc.validate(rp, col, c, ctx=ctx) == (0, 0)
    ctx.close()
