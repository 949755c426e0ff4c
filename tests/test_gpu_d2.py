"""Distance-2 coloring on the GPU against the CPU oracle (which colors the
square graph with the distance-1 routines), element by element: initial
coloring under every priority order and selection, recoloring passes under
every class order, validation, and the edge cases (empty, isolated, one
vertex, cliques of the square, more colors than one selection window)."""
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


GRAPHS = {
    "er": lambda: gen.er(2001, 8003, 3),
    "mesh": lambda: gen.mesh27(11),
    "grid": lambda: gen.grid5(47, 33),
    "rmat": lambda: gen.rmat(11, 8, seed=3),
    "rgg": lambda: gen.rgg(1500, 0.05, 7),
    "complete": lambda: gen.complete(40),
    "star": lambda: gen.star(300),
    "crown": lambda: gen.crown(20),
    "path": lambda: gen.path(700),
    "empty": lambda: gen.empty(300),
    "single": lambda: gen.empty(1),
}
_SQ = {}


def square(name, g):
    if name not in _SQ:
        _SQ[name] = oracle.square(g)
    return _SQ[name]


def _init_equal(gc, name, g, sel, X, seed, flags=0, ctx=None):
    rp, col = dev(g)
    c, st = gc.init_color(rp, col, sel, X, seed, flags=flags | gc.FLAG_DISTANCE2, ctx=ctx)
    ref = oracle.init_color_d2(g, sel, X, seed, flags=flags, sq=square(name, g))
    got = c.cpu().numpy()
    assert np.array_equal(got, ref.colors), f"{name}: {int((got != ref.colors).sum())} vertex colors differ"
    assert st["rounds"] == ref.stats["rounds"]
    assert st["round_sizes"] == ref.w_sizes.tolist()
    assert st["losers_total"] == ref.stats["losers_total"]
    assert (st["num_colors"], st["max_color"]) == (ref.stats["num_colors"], ref.stats["max_color"])
    return c, ref


@pytest.mark.parametrize("name", sorted(GRAPHS))
def test_d2_init_parity(gc, name):
    g = GRAPHS[name]()
    for sel, X in ((gc.FIRST_FIT, 1), (gc.RANDOM_X, 4)):
        for seed in (1, 77):
            _init_equal(gc, name, g, sel, X, seed)


@pytest.mark.parametrize("name", ["er", "mesh", "rmat", "path", "star"])
def test_d2_init_priority_orders(gc, name):
    g = GRAPHS[name]()
    for flags in (gc.FLAG_FIXED_PRIORITY, gc.FLAG_PRIO_NATURAL):
        for sel, X in ((gc.FIRST_FIT, 1), (gc.RANDOM_X, 3)):
            _init_equal(gc, name, g, sel, X, 21, flags=flags)


def test_d2_mesh_natural_closed_form(gc):
    """Natural order on the 27-point mesh: the period-3 pattern on each axis."""
    N = 9
    rp, col = dev(gen.mesh27(N))
    c, st = gc.init_color(rp, col, gc.FIRST_FIT, 1, 5, flags=gc.FLAG_DISTANCE2 | gc.FLAG_PRIO_NATURAL)
    want = [1 + x % 3 + 3 * (y % 3) + 9 * (z % 3) for z in range(N) for y in range(N) for x in range(N)]
    assert c.cpu().numpy().tolist() == want and st["num_colors"] == 27


def _recolor_equal(gc, name, g, c, rc, passes, seed=3):
    rp, col = dev(g)
    for p, perm in enumerate([gc.PERM_REVERSE, gc.PERM_RANDOM, gc.PERM_NONINC][:passes]):
        c, st = gc.recolor_d2(rp, col, c, perm, seed, p, out=c)
        r = oracle.recolor_d2(g, rc, perm, seed, p, sq=square(name, g))
        got = c.cpu().numpy()
        assert np.array_equal(got, r.colors), f"{name} pass {p}: {int((got != r.colors).sum())} differ"
        rc = r.colors
    return rc


def test_d2_beyond_one_window(gc):
    """Random-X with X = 1024 on RMAT (rows past 64 entries: a wavefront per
    vertex): colors far past the masks' range, in the rounds and the passes."""
    g = gen.rmat(11, 16, seed=5)
    c, ref = _init_equal(gc, "rmat16", g, gc.RANDOM_X, 1024, 3)
    assert ref.stats["max_color"] > 2048 and g.max_deg > 64
    rc = _recolor_equal(gc, "rmat16", g, c, ref.colors, 3)
    assert rc.max() > 128


def test_d2_beyond_masks_short_rows(gc):
    """Rows of at most 64 entries (8 lanes per vertex) with colors above the
    masks' 128: the in-group scan of the distance-2 neighborhood."""
    g = gen.rgg(3000, 0.06, 2)
    assert g.max_deg <= 64
    c, ref = _init_equal(gc, "rgg64", g, gc.RANDOM_X, 64, 3)
    assert ref.stats["max_color"] > 128
    _recolor_equal(gc, "rgg64", g, c, ref.colors, 3)


@pytest.mark.parametrize("star", [1, -1])
@pytest.mark.parametrize("name", ["er", "mesh", "rmat", "star", "grid", "path"])
def test_d2_detect_modes(gc, name, star):
    """Per-neighborhood marking in every round (rows past 64 entries take the
    marked-for-recheck path) and the distance-2 scan in every round."""
    g = GRAPHS[name]()
    ctx = gc.Context(g.n, g.nnz)
    ctx.set_tuning(d2_star=star)
    for sel, X in ((gc.FIRST_FIT, 1), (gc.RANDOM_X, 4)):
        _init_equal(gc, name, g, sel, X, 13, ctx=ctx)
    _init_equal(gc, name, g, gc.FIRST_FIT, 1, 13, flags=gc.FLAG_PRIO_NATURAL, ctx=ctx)
    ctx.close()


def test_d2_small_grid(gc):
    """One workgroup per CU: every kernel walks its worklist in grid strides."""
    g = GRAPHS["mesh"]()
    ctx = gc.Context(g.n, g.nnz)
    ctx.set_tuning(grid_per_cu=1)
    _init_equal(gc, "mesh", g, gc.RANDOM_X, 4, 9, ctx=ctx)
    ctx.close()


@pytest.mark.parametrize("name", ["er", "mesh", "grid", "rmat", "rgg", "complete", "crown", "path", "single"])
def test_d2_recolor_parity(gc, name):
    g = GRAPHS[name]()
    sq = square(name, g)
    rp, col = dev(g)
    c, ref = _init_equal(gc, name, g, gc.RANDOM_X, 5, 11)
    rc = ref.colors
    perms = [gc.PERM_REVERSE, gc.PERM_RANDOM, gc.PERM_NONINC, gc.PERM_NONDEC, gc.PERM_RANDOM]
    for p, perm in enumerate(perms):
        c, st = gc.recolor_d2(rp, col, c, perm, 11, p, out=c)
        r = oracle.recolor_d2(g, rc, perm, 11, p, sq=sq)
        assert r.status == oracle.OK
        got = c.cpu().numpy()
        assert np.array_equal(got, r.colors), f"{name} pass {p}: {int((got != r.colors).sum())} differ"
        assert (st["num_colors"], st["max_color"], st["k_classes"]) == \
            (r.stats["num_colors"], r.stats["max_color"], len(r.pi))
        rc = r.colors
    assert gc.validate_d2(rp, col, c) == (0, 0)


def test_d2_recolor_mesh_closed_form(gc):
    N = 8
    g = gen.mesh27(N)
    rp, col = dev(g)
    c0 = np.array([1 + x % 3 + 3 * (y % 3) + 9 * (z % 3) for z in range(N) for y in range(N) for x in range(N)],
                  np.int32)
    for perm, seed in ((gc.PERM_REVERSE, 1), (gc.PERM_NONINC, 1), (gc.PERM_RANDOM, 6)):
        c, _ = gc.recolor_d2(rp, col, torch.from_numpy(c0).cuda(), perm, seed, 0)
        pi = oracle.class_order(np.bincount(c0, minlength=28), perm, seed, 0)
        rank = {int(k): i for i, k in enumerate(pi)}
        assert c.cpu().numpy().tolist() == [rank[int(k)] + 1 for k in c0]


def test_d2_validate_parity(gc):
    rng = np.random.default_rng(4)
    for name in ("er", "mesh", "rmat", "grid", "path", "star", "empty", "single"):
        g = GRAPHS[name]()
        rp, col = dev(g)
        sq = square(name, g)
        for k in (3, 40, 10**6):
            c = rng.integers(1, k + 1, size=g.n).astype(np.int32)
            c[rng.random(g.n) < 0.05] = 0
            got = gc.validate_d2(rp, col, torch.from_numpy(c).cuda())
            assert got == oracle.validate_d2(g, c, sq=sq), (name, k)
        # a distance-1 coloring is usually not a distance-2 coloring; the oracle decides
        c1 = oracle.init_color(g, oracle.FIRST_FIT, 1, 2).colors
        assert gc.validate_d2(rp, col, torch.from_numpy(c1).cuda()) == oracle.validate_d2(g, c1, sq=sq)


def test_d2_arguments(gc):
    g = gen.path(10)
    rp, col = dev(g)
    with pytest.raises(gc.GCError):
        gc.init_color(rp, col, gc.FIRST_FIT, 1, 1, flags=gc.FLAG_DISTANCE2 | gc.FLAG_PRIO_LF)
    with pytest.raises(gc.GCError):
        gc.init_color(rp, col, gc.FIRST_FIT, 1, 1, flags=16)
    # no vertices
    e = torch.zeros(1, dtype=torch.int32, device="cuda:0")
    c, st = gc.init_color(e, e[:0], gc.FIRST_FIT, 1, 1, flags=gc.FLAG_DISTANCE2)
    assert c.numel() == 0 and st["rounds"] == 0
    assert gc.validate_d2(e, e[:0], c) == (0, 0)


def test_d2_full_size_mesh(gc):
    """The 128^3 mesh of the distance-2 benchmark, at full size.  Natural order:
    the closed form 1 + x%3 + 3(y%3) + 9(z%3) for every one of the 2,097,152
    vertices, and recoloring it gives rank + 1.  The benchmark's own
    configuration (Random-X X=4 + 5 NI passes): valid at distance 2, colors
    within |N2(v)| + X, passes never above rank + 1 nor above the input's
    class count."""
    N = 128
    g = gen.mesh27(N)
    rp, col = dev(g)
    z, y, x = np.meshgrid(np.arange(N), np.arange(N), np.arange(N), indexing="ij")
    want = (1 + x % 3 + 3 * (y % 3) + 9 * (z % 3)).astype(np.int32).ravel()
    c, st = gc.init_color(rp, col, gc.FIRST_FIT, 1, 7, flags=gc.FLAG_DISTANCE2 | gc.FLAG_PRIO_NATURAL)
    assert np.array_equal(c.cpu().numpy(), want) and st["num_colors"] == 27
    for perm, seed in ((gc.PERM_NONINC, 1), (gc.PERM_RANDOM, 9)):
        out, _ = gc.recolor_d2(rp, col, c, perm, seed, 0)
        pi = oracle.class_order(np.bincount(want, minlength=28), perm, seed, 0)
        rank = np.zeros(28, np.int32)
        rank[pi] = np.arange(len(pi), dtype=np.int32)
        assert np.array_equal(out.cpu().numpy(), rank[want] + 1)
    # the benchmark configuration
    c, st = gc.init_color(rp, col, gc.RANDOM_X, 4, 1, flags=gc.FLAG_DISTANCE2)
    assert gc.validate_d2(rp, col, c) == (0, 0)
    h = c.cpu().numpy()
    nx = np.minimum(x + 2, N - 1) - np.maximum(x - 2, 0) + 1
    ny = np.minimum(y + 2, N - 1) - np.maximum(y - 2, 0) + 1
    nz = np.minimum(z + 2, N - 1) - np.maximum(z - 2, 0) + 1
    n2 = (nx * ny * nz - 1).ravel()  # |N2(v)|: the Chebyshev ball of radius 2 minus v
    assert (h <= n2 + 4).all()
    k = st["num_colors"]
    for p in range(5):
        sizes = np.bincount(h, minlength=h.max() + 1)
        pi = oracle.class_order(sizes, gc.PERM_NONINC, 1, p)
        rank = np.zeros(h.max() + 1, np.int64)
        rank[pi] = np.arange(len(pi))
        c, sp = gc.recolor_d2(rp, col, c, gc.PERM_NONINC, 1, p, out=c)
        new = c.cpu().numpy()
        assert (new <= rank[h] + 1).all() and sp["num_colors"] <= k
        assert gc.validate_d2(rp, col, c) == (0, 0)
        h, k = new, sp["num_colors"]
