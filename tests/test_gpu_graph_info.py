"""The per-graph analysis a context runs before coloring a new graph: longest
row and number of far adjacency entries (|u - w| >= 32768, which pick the
default color copy of the initial coloring), against their plain definitions
on the host.  Shapes cover entry chunks of 4096 that start inside a row, hub
rows spread over many chunks, long runs of empty rows, and empty graphs."""
import numpy as np
import pytest

import gen

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

NEAR = 32768


@pytest.fixture(scope="module")
def gc():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1407_6745_amd as m

    m.lib()
    return m


def _sparse_rows(n, k, seed):
    """k random edges among vertices spread over [0, n): most rows empty."""
    rng = np.random.default_rng(seed)
    a = rng.integers(0, n, k)
    b = rng.integers(0, n, k)
    keep = a != b
    return gen.from_pairs(n, np.stack([a[keep], b[keep]], 1))


GRAPHS = {
    "rmat16": lambda: gen.rmat(16, 16, seed=3),
    "mesh40_relabel": lambda: gen.relabel(gen.mesh27(40), np.random.default_rng(2).permutation(64000)),
    "mesh40": lambda: gen.mesh27(40),
    "star": lambda: gen.star(150000),
    "sparse_rows": lambda: _sparse_rows(400000, 3000, 5),
    "er": lambda: gen.er(90001, 400003, 7),
    "path": lambda: gen.path(5),
}


def _expected(g):
    rp = np.asarray(g.row_ptr, np.int64)
    deg = np.diff(rp)
    u = np.repeat(np.arange(g.n, dtype=np.int64), deg)
    far = int((np.abs(np.asarray(g.col, np.int64) - u) >= NEAR).sum())
    return (int(deg.max()) if g.n else 0), far


@pytest.mark.parametrize("name", sorted(GRAPHS))
def test_graph_analysis(gc, name):
    g = GRAPHS[name]()
    d = torch.device("cuda:0")
    rp = torch.from_numpy(np.ascontiguousarray(g.row_ptr)).to(d)
    col = torch.from_numpy(np.ascontiguousarray(g.col)).to(d)
    ctx = gc.Context(g.n, g.nnz)
    assert ctx.info()["max_degree"] == -1 and ctx.info()["far_entries"] == -1
    gc.init_color(rp, col, gc.RANDOM_X, 4, 1, ctx=ctx)
    info = ctx.info()
    assert (info["max_degree"], info["far_entries"]) == _expected(g)
    ctx.close()


def test_graph_analysis_follows_graph(gc):
    """A second graph on the same context is analysed afresh."""
    ctx = gc.Context(400000, 4000000)
    d = torch.device("cuda:0")
    for name in ("rmat16", "mesh40", "rmat16"):
        g = GRAPHS[name]()
        rp = torch.from_numpy(np.ascontiguousarray(g.row_ptr)).to(d)
        col = torch.from_numpy(np.ascontiguousarray(g.col)).to(d)
        gc.init_color(rp, col, gc.FIRST_FIT, 1, 1, ctx=ctx)
        info = ctx.info()
        assert (info["max_degree"], info["far_entries"]) == _expected(g), name
    ctx.close()
