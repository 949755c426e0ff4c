"""Autotuner on the GPU: every candidate setting gives the same colors (the
knobs only schedule work), the chosen setting is left in the context, and the
colors it returns equal the oracle's (single graphs) or the plain per-graph
calls (batches).  Also the batch's largest-first graph order, including a batch
above the 8192 graphs the ordering kernel sorts."""
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


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(torch.device("cuda:0"))


@pytest.mark.parametrize("graph", ["mesh", "rmat"])
def test_autotune_single_graph(gc, graph):
    g = gen.mesh27(18) if graph == "mesh" else gen.rmat(12, 16, seed=4)
    rp, col = dev(g.row_ptr), dev(g.col)
    ctx = gc.Context(g.n, g.nnz)
    best, ms, c = gc.autotune(rp, col, gc.RANDOM_X, 4, gc.PERM_NONINC, 3, 7, ctx=ctx)
    assert ms > 0 and ctx.tuning == best
    ref = oracle.init_color(g, oracle.RANDOM_X, 4, 7).colors
    for p in range(3):
        ref = oracle.recolor(g, ref, oracle.PERM_NONINC, 7, p).colors
    assert np.array_equal(c.cpu().numpy(), ref)
    # the chosen setting, used by the plain calls afterwards
    c2, _ = gc.init_color(rp, col, gc.RANDOM_X, 4, 7, ctx=ctx)
    for p in range(3):
        c2, _ = gc.recolor(rp, col, c2, gc.PERM_NONINC, 7, p, out=c2, ctx=ctx)
    assert np.array_equal(c2.cpu().numpy(), ref)
    ctx.close()


def _batch(G, seed, n_lo, n_hi):
    b = gen.rgg_batch(G, seed, n_lo, n_hi)
    return b, dev(b.vtx_off), dev(b.edge_off), dev(b.row_ptr), dev(b.col)


def test_autotune_batch_and_every_candidate(gc):
    b, vo, eo, rp, col = _batch(96, 5, 300, 6000)
    V = int(np.diff(b.vtx_off).max())
    ctx = gc.Context(V, 1)
    ref_c, ref_p = gc.batch_color(vo, eo, rp, col, gc.RANDOM_X, 4, gc.PERM_REVERSE, 3, 11, ctx=ctx)
    ref_c, ref_p = ref_c.cpu().numpy(), ref_p.cpu().numpy()
    best, ms, c, per = gc.autotune_batch(vo, eo, rp, col, gc.RANDOM_X, 4, gc.PERM_REVERSE, 3, 11, ctx=ctx)
    assert ms > 0 and ctx.tuning == best
    assert best["batch_order"] in (0, 1) and 1 <= best["batch_wg_per_cu"] <= 5
    assert np.array_equal(c.cpu().numpy(), ref_c) and np.array_equal(per.cpu().numpy(), ref_p)
    for order in (0, 1):
        for wg in (1, 2, 3, 4, 5):
            ctx.set_tuning(batch_order=order, batch_wg_per_cu=wg)
            c, per = gc.batch_color(vo, eo, rp, col, gc.RANDOM_X, 4, gc.PERM_REVERSE, 3, 11, ctx=ctx)
            assert np.array_equal(c.cpu().numpy(), ref_c), (order, wg)
            assert np.array_equal(per.cpu().numpy(), ref_p), (order, wg)
    # graph 0 against the plain calls with its seed
    sub = b.graph(0)
    seed = gc.batch_graph_seed(11, 0)
    c0, _ = gc.init_color(dev(sub.row_ptr), dev(sub.col), gc.RANDOM_X, 4, seed)
    for p in range(3):
        c0, _ = gc.recolor(dev(sub.row_ptr), dev(sub.col), c0, gc.PERM_REVERSE, seed, p, out=c0)
    assert np.array_equal(c0.cpu().numpy(), ref_c[:sub.n])
    ctx.close()


def test_batch_order_beyond_sort_size(gc):
    """9000 tiny graphs: above the largest-first sort's 8192, id order is kept."""
    b, vo, eo, rp, col = _batch(9000, 6, 8, 40)
    V = int(np.diff(b.vtx_off).max())
    ctx = gc.Context(V, 1)
    a, pa = gc.batch_color(vo, eo, rp, col, gc.FIRST_FIT, 1, gc.PERM_NONINC, 2, 3, ctx=ctx)
    ctx.set_tuning(batch_order=1, batch_wg_per_cu=2)
    c, pc = gc.batch_color(vo, eo, rp, col, gc.FIRST_FIT, 1, gc.PERM_NONINC, 2, 3, ctx=ctx)
    assert torch.equal(a, c) and torch.equal(pa, pc)
    ctx.close()


def test_tuning_fields_validated(gc):
    ctx = gc.Context(10, 10)
    with pytest.raises(gc.GCError):
        ctx.set_tuning(batch_wg_per_cu=6)
    with pytest.raises(gc.GCError):
        ctx.set_tuning(batch_order=2)
    ctx.close()
