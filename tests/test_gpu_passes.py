"""GPU parity of gc_recolor_passes: several recoloring passes in one call
(section 3, recoloring iterated) equal the oracle's passes one by one, final
colors bit-exact and every pass's statistics, for class-order sequences that
settle (every vertex keeps its rank from pass to pass) and ones that do not."""
import numpy as np
import pytest

import gen
import oracle

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

RV, NI, ND, RAND = oracle.PERM_REVERSE, oracle.PERM_NONINC, oracle.PERM_NONDEC, oracle.PERM_RANDOM


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
    "er": lambda: gen.er(3001, 15007, 3),
    "mesh": lambda: gen.mesh27(13),
    "mesh40": lambda: gen.mesh27(40),
    "grid": lambda: gen.grid5(61, 37),
    "rmat": lambda: gen.rmat(12, 16, seed=5),
    "rgg": lambda: gen.rgg(2500, 0.05, 7),
    "complete100": lambda: gen.complete(100),
    # rows of exactly 64 entries (group rows at the default deg_wave) in 65
    # classes: the last rank's First Fit color is 65, past the register word
    "complete65": lambda: gen.complete(65),
    "star": lambda: gen.star(5000),
    "path": lambda: gen.path(1000),
    "single": lambda: gen.empty(1),
}

SEQS = {
    "ni": [NI] * 8,
    "mixed": [RV, NI, NI, NI, ND, ND, RAND, NI, NI],
    "rand": [RAND] * 4,
}


def _ranks(colors, pi):
    """Rank of every vertex's color in the class order pi (0-based)."""
    r = np.full(int(colors.max()) + 1 if colors.size else 1, -1, np.int64)
    r[np.asarray(pi)] = np.arange(len(pi))
    return r[colors]


def _oracle_passes(g, c0, perms, seed, pass0):
    """The oracle's passes; also how many passes kept every vertex at the rank
    it had in the pass before."""
    c, prev, kept, res = c0, None, 0, []
    for p, perm in enumerate(perms):
        r = oracle.recolor(g, c, perm, seed, pass0 + p)
        assert r.status == 0
        rk = _ranks(c, r.pi)
        if prev is not None and np.array_equal(rk, prev):
            kept += 1
        prev = rk
        res.append(r)
        c = r.colors
    return res, kept


def _check(gc, g, perms, seed=7, pass0=0, ctx=None, inplace=False, X=4, min_kept=0):
    rp, col = dev(g)
    c, _ = gc.init_color(rp, col, gc.RANDOM_X, X, seed, ctx=ctx)
    c0 = c.cpu().numpy()
    res, kept = _oracle_passes(g, c0, perms, seed, pass0)
    assert kept >= min_kept, f"{g.name}: the case keeps the layout in only {kept} passes"
    out, st = gc.recolor_passes(rp, col, c, perms, seed, pass0, out=c if inplace else None, ctx=ctx)
    got = out.cpu().numpy()
    exp = res[-1].colors if res else c0
    assert np.array_equal(got, exp), f"{g.name}: {int((got != exp).sum())} vertex colors differ"
    assert len(st) == len(perms)
    for p, (s, r) in enumerate(zip(st, res)):
        assert s["k_classes"] == len(r.pi), p
        assert (s["num_colors"], s["max_color"]) == (r.stats["num_colors"], r.stats["max_color"]), p
    return kept


@pytest.mark.parametrize("seq", sorted(SEQS))
@pytest.mark.parametrize("name", sorted(GRAPHS))
def test_passes_parity(gc, name, seq):
    g = GRAPHS[name]()
    _check(gc, g, SEQS[seq], inplace=seq == "mixed")


@pytest.mark.parametrize("inplace", [False, True])
@pytest.mark.parametrize("name", ["mesh", "mesh40", "grid", "path", "er", "rmat"])
def test_passes_keep_layout(gc, name, inplace):
    """Passes in one class order, in place and not: on these graphs the later
    passes keep every vertex's rank (a fixed point of the passes)."""
    kept = _check(gc, GRAPHS[name](), [NI] * 10, inplace=inplace)
    if name in ("mesh", "mesh40", "grid", "path"):
        assert kept >= 3, "nonincreasing-size passes settle on these graphs"


PASS_TUNINGS = [
    dict(deg_wave=8, deg_split=64, split_len=64),                 # split rows
    dict(deg_wave=8, deg_split=64, split_len=64, hub_words=1),
    dict(deg_wave=0, deg_split=1, split_len=64, group=1),          # every row of 2+ entries split
    dict(deg_wave=8, deg_split=64, split_len=64, walk_flags=3),
    dict(group=4, deg_wave=16), dict(xcd_chunks=0), dict(walk_mode=1),
]


@pytest.mark.parametrize("t", PASS_TUNINGS, ids=str)
@pytest.mark.parametrize("name", ["rmat", "star", "complete100", "complete65", "mesh"])
def test_passes_tunings(gc, name, t):
    g = GRAPHS[name]()
    ctx = gc.Context(g.n, g.nnz)
    ctx.set_tuning(**t)
    for seq in ("ni", "mixed"):
        _check(gc, g, SEQS[seq], ctx=ctx, inplace=seq == "ni")
    ctx.close()


def test_passes_many_classes(gc):
    """K_300 from a random proper coloring: 300 classes (two-byte color copy,
    ranks beyond one mask word); the classes stay singletons, so every pass
    after the first keeps every rank."""
    g = gen.complete(300)
    rp, col = dev(g)
    rng = np.random.default_rng(11)
    c0 = (rng.permutation(300) + 1).astype(np.int32)
    perms = [NI, NI, NI, RAND, NI, NI]
    res, kept = _oracle_passes(g, c0, perms, 5, 0)
    assert kept >= 3
    out, st = gc.recolor_passes(rp, col, torch.from_numpy(c0.copy()).cuda(), perms, 5, 0)
    assert np.array_equal(out.cpu().numpy(), res[-1].colors)
    assert [s["num_colors"] for s in st] == [300] * len(perms)


def test_passes_equal_single_calls(gc):
    """The same passes through gc_recolor one at a time (pass index pass0 + p
    seeds the random class order)."""
    g = GRAPHS["rgg"]()
    rp, col = dev(g)
    c, _ = gc.init_color(rp, col, gc.RANDOM_X, 3, 9)
    perms = [RAND, NI, RAND, ND, NI, NI]
    one = c.clone()
    for p, perm in enumerate(perms):
        one, _ = gc.recolor(rp, col, one, perm, 9, 5 + p, out=one)
    many, _ = gc.recolor_passes(rp, col, c, perms, 9, 5)
    assert torch.equal(one, many)


def test_passes_back_to_back_calls(gc):
    """Consecutive calls on one context, the second on a smaller graph and the
    third on a larger one (layout state never leaks between calls)."""
    ctx = gc.Context(70000, 2000000)
    for name, seq in (("mesh40", "ni"), ("grid", "ni"), ("rmat", "mixed"), ("mesh40", "mixed")):
        _check(gc, GRAPHS[name](), SEQS[seq], ctx=ctx)
    ctx.close()


def test_passes_edge_cases(gc):
    g = GRAPHS["er"]()
    rp, col = dev(g)
    c, _ = gc.init_color(rp, col, gc.FIRST_FIT, 1, 1)
    out, st = gc.recolor_passes(rp, col, c, [], 1, 0)  # no passes: a copy
    assert torch.equal(out, c) and st == []
    with pytest.raises(gc.GCError):
        gc.recolor_passes(rp, col, c, [NI, 4], 1, 0)
    with pytest.raises(gc.GCError):
        gc.recolor_passes(rp, col, c, [NI], 1, -1)
    e = gen.empty(0)
    rp0, col0 = dev(e)
    out0, st0 = gc.recolor_passes(rp0, col0, torch.zeros(0, dtype=torch.int32, device="cuda"), [NI, RV], 1, 0)
    assert out0.numel() == 0 and [s["num_colors"] for s in st0] == [0, 0]
