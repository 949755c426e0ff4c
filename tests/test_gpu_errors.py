"""Error paths and state across calls, on the GPU through the C ABI: the
sticky device error of the class walk (a bounded wait made to give up from
the host), the input properness check, the batch workspace across slice
layouts with many colors, and a checkpoint/resume of the recoloring passes.
Every kernel here exits normally; failures are forced only through the
walk's own wait limit."""
import numpy as np
import pytest

import gen
import oracle

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def gc():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1407_6745_amd as m

    m.lib()
    return m


def dev(g):
    d = torch.device("cuda:0")
    return torch.from_numpy(np.ascontiguousarray(g.row_ptr)).to(d), torch.from_numpy(np.ascontiguousarray(g.col)).to(d)


def test_sticky_wait_error(gc):
    """K_1500 colored 1..1500: every recoloring rank waits for all lower
    ranks.  With a wait limit of one poll, waits give up (the kernel still
    ends); passes queued without stats return OK, and the next synchronizing
    call reports the failure once.  A pass with stats reports it itself."""
    g = gen.complete(1500)
    rp, col = dev(g)
    ctx = gc.Context(g.n, g.nnz)
    c, st = gc.init_color(rp, col, gc.FIRST_FIT, 1, 1, ctx=ctx)
    assert st["num_colors"] == 1500
    ref = oracle.recolor(g, c.cpu().numpy(), oracle.PERM_REVERSE, 1, 0).colors
    assert ctx.status() == gc.OK
    ctx.set_tuning(spin_limit=1)
    out = torch.empty_like(c)
    print("[errors] three passes without stats, wait limit 1", flush=True)
    for _ in range(3):
        gc.recolor(rp, col, c, gc.PERM_REVERSE, 1, 0, out=out, stats=False, ctx=ctx)
    assert ctx.status() == gc.ERR_DEVICE
    assert "gave up" in ctx.last_error()
    assert ctx.status() == gc.OK, "reported once"
    print("[errors] one pass with stats, wait limit 1", flush=True)
    with pytest.raises(gc.GCError) as e:
        gc.recolor(rp, col, c, gc.PERM_REVERSE, 1, 0, out=out, ctx=ctx)
    assert e.value.status == gc.ERR_DEVICE
    assert ctx.status() == gc.OK
    # a synchronizing call of another kind reports a failure of earlier work too
    gc.recolor(rp, col, c, gc.PERM_REVERSE, 1, 0, out=out, stats=False, ctx=ctx)
    with pytest.raises(gc.GCError) as e:
        gc.count_colors(c, ctx=ctx)
    assert e.value.status == gc.ERR_DEVICE
    ctx.set_tuning(spin_limit=0)
    out, st = gc.recolor(rp, col, c, gc.PERM_REVERSE, 1, 0, ctx=ctx)
    assert np.array_equal(out.cpu().numpy(), ref)
    assert ctx.status() == gc.OK
    ctx.close()


def test_check_input(gc):
    """With check_input, recoloring rejects an improper input (a conflicting
    edge, an uncolored vertex, a distance-2 conflict for the distance-2 pass)
    with GC_ERR_COLORING; proper inputs pass and give the oracle's colors."""
    g = gen.grid5(41, 29)
    rp, col = dev(g)
    ctx = gc.Context(g.n, g.nnz)
    ctx.set_tuning(check_input=1)
    c, _ = gc.init_color(rp, col, gc.RANDOM_X, 3, 5, ctx=ctx)
    out, _ = gc.recolor(rp, col, c, gc.PERM_NONINC, 5, 0, ctx=ctx)
    ref = oracle.recolor(g, c.cpu().numpy(), oracle.PERM_NONINC, 5, 0).colors
    assert np.array_equal(out.cpu().numpy(), ref)
    bad = c.clone()
    bad[1] = bad[0]  # vertices 0 and 1 are adjacent in the grid
    zero = c.clone()
    zero[77] = 0
    for x in (bad, zero):
        for fn in (gc.recolor, gc.arc_recolor):
            with pytest.raises(gc.GCError) as e:
                fn(rp, col, x, gc.PERM_REVERSE, 1, 0, ctx=ctx, stats=False)
            assert e.value.status == gc.ERR_COLORING, fn.__name__
    # distance 2: vertices 0 and 2 of a grid row are two edges apart
    d2, _ = gc.init_color(rp, col, gc.FIRST_FIT, 1, 2, flags=gc.FLAG_DISTANCE2, ctx=ctx)
    out2, _ = gc.recolor_d2(rp, col, d2, gc.PERM_REVERSE, 2, 0, ctx=ctx)
    assert gc.validate_d2(rp, col, out2, ctx=ctx) == (0, 0)
    d2b = d2.clone()
    d2b[2] = d2b[0]
    assert gc.validate(rp, col, d2b, ctx=ctx) == (0, 0)
    with pytest.raises(gc.GCError) as e:
        gc.recolor_d2(rp, col, d2b, gc.PERM_REVERSE, 2, 0, ctx=ctx)
    assert e.value.status == gc.ERR_COLORING
    gc.recolor(rp, col, d2b, gc.PERM_REVERSE, 2, 0, ctx=ctx)  # distance-1 proper: accepted
    ctx.close()


def _pack(graphs):
    G = len(graphs)
    vo = np.zeros(G + 1, np.int64)
    eo = np.zeros(G + 1, np.int64)
    vo[1:] = np.cumsum([g.n for g in graphs])
    eo[1:] = np.cumsum([g.nnz for g in graphs])
    rp = np.concatenate([np.asarray(g.row_ptr, np.int32) for g in graphs])
    col = np.concatenate([np.asarray(g.col, np.int32) for g in graphs])
    d = torch.device("cuda:0")
    return [torch.from_numpy(a).to(d) for a in (vo, eo, rp, col)], vo


def test_batch_many_colors_after_layout_change(gc):
    """Graphs with 1,024 colors or more keep their class tables in the batch
    workspace.  A first batch with another per-graph vertex bound (another
    slice layout) fills the workspace with worklists and class lists; the
    second batch must still match plain calls and the oracle graph by graph."""
    ctx = gc.Context(6000, 2_000_000)
    first = [gen.rgg(5000, 0.03, 1), gen.er(4000, 20000, 2), gen.rgg(4500, 0.04, 3)]
    (vo, eo, rp, col), _ = _pack(first)
    gc.batch_color(vo, eo, rp, col, gc.RANDOM_X, 4, gc.PERM_REVERSE, 5, 9, max_vertices_per_graph=5000, ctx=ctx)
    ctx.raise_status()
    graphs = [gen.complete(1100), gen.rgg(3000, 0.05, 3), gen.complete(1030), gen.star(900)]
    (vo, eo, rp, col), voh = _pack(graphs)
    colors, per = gc.batch_color(vo, eo, rp, col, gc.RANDOM_X, 4, gc.PERM_NONINC, 3, 7,
                                 max_vertices_per_graph=3000, ctx=ctx)
    per = per.cpu().numpy()
    got = colors.cpu().numpy()
    for gi, g in enumerate(graphs):
        sg = gc.batch_graph_seed(7, gi)
        ref = oracle.init_color(g, oracle.RANDOM_X, 4, sg)
        assert per[gi, 0] == ref.rounds and per[gi, 1] == ref.stats["num_colors"], gi
        rc = ref.colors
        for p in range(3):
            rc = oracle.recolor(g, rc, oracle.PERM_NONINC, sg, p).colors
        assert np.array_equal(got[voh[gi]:voh[gi + 1]], rc), f"graph {gi} differs from the oracle"
        assert per[gi, 2] == len(np.unique(rc)) and per[gi, 3] == 0
    assert per[0, 2] == 1100 and per[2, 2] == 1030
    ctx.close()


@pytest.mark.parametrize("name", ["rmat", "mesh"])
def test_checkpoint_resume_identity(gc, name):
    """Ten recoloring passes in one run equal five passes, a checkpoint of the
    colors to the host, a fresh context and device buffer restored from it, and
    five more passes (pass indices 5..9): the pass is a function of the input
    coloring, the seed and the pass index only.  Both equal the oracle."""
    g = gen.rmat(12, 16, seed=5) if name == "rmat" else gen.mesh27(14)
    rp, col = dev(g)
    perm = gc.PERM_RANDOM
    ctx = gc.Context(g.n, g.nnz)
    c, _ = gc.init_color(rp, col, gc.RANDOM_X, 4, 3, ctx=ctx)
    c0 = c.cpu().numpy()
    for p in range(10):
        c, _ = gc.recolor(rp, col, c, perm, 3, p, out=c, stats=False, ctx=ctx)
    whole = c.cpu().numpy()
    c = torch.from_numpy(c0).cuda()
    for p in range(5):
        c, _ = gc.recolor(rp, col, c, perm, 3, p, out=c, stats=False, ctx=ctx)
    ctx.raise_status()
    ckpt = c.cpu().numpy().copy()
    ctx.close()
    del c
    ctx2 = gc.Context(g.n, g.nnz)
    c = torch.from_numpy(ckpt).cuda()
    for p in range(5, 10):
        c, _ = gc.recolor(rp, col, c, perm, 3, p, out=c, stats=False, ctx=ctx2)
    ctx2.raise_status()
    assert np.array_equal(c.cpu().numpy(), whole)
    rc = c0
    for p in range(10):
        rc = oracle.recolor(g, rc, oracle.PERM_RANDOM, 3, p).colors
    assert np.array_equal(whole, rc)
    ctx2.close()


def test_validate_d2_counts_pairs(gc):
    """Distance-2 conflicts are counted as distinct pairs however many paths
    join them, also past the deduplication set's size: a star whose 3,000
    leaves share one color with the center (every pair of the 3,001 vertices
    is within two edges), the all-ones mesh, and random colorings against the
    oracle."""
    g = gen.star(3000)
    rp, col = dev(g)
    ones = torch.ones(g.n, dtype=torch.int32, device="cuda")
    assert gc.validate_d2(rp, col, ones) == (3001 * 3000 // 2, 0)
    assert gc.validate(rp, col, ones) == (3000, 0)
    m = gen.mesh27(9)
    mrp, mcol = dev(m)
    ones = torch.ones(m.n, dtype=torch.int32, device="cuda")
    sq = oracle.square(m)
    assert gc.validate_d2(mrp, mcol, ones) == oracle.validate_d2(m, ones.cpu().numpy(), sq=sq)
    assert oracle.validate_d2(m, ones.cpu().numpy(), sq=sq)[0] == sq.nnz // 2
    rng = np.random.default_rng(4)
    for k in (2, 9, 40):
        c = rng.integers(1, k + 1, size=m.n).astype(np.int32)
        c[rng.random(m.n) < 0.03] = 0
        assert gc.validate_d2(mrp, mcol, torch.from_numpy(c).cuda()) == oracle.validate_d2(m, c, sq=sq), k
