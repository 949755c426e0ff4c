"""GPU parity at full size: the whole coloring after the initial coloring and
after every recoloring pass, compared with the oracle's results (SHA-256 of
the color array, written by tests/golden/make_full_size.py from oracle/
only), plus rounds, per-round set sizes and color counts.  Also the batched
kernel against plain per-graph calls and against the oracle on sampled graphs
of the random-geometric-graph batch."""
import hashlib
import json
import os

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
