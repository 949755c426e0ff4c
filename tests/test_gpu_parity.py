"""GPU parity: the HIP path through the C ABI against the CPU oracle, element
by element (integer work: bit-exact), on seeded inputs of every family at
sizes that span several workgroups and a ragged tail, plus edge cases."""
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
    "er": lambda: gen.er(3001, 15007, 3),
    "mesh": lambda: gen.mesh27(13),
    "grid": lambda: gen.grid5(61, 37),
    "rmat": lambda: gen.rmat(12, 16, seed=5),
    "rgg": lambda: gen.rgg(2500, 0.05, 7),
    "complete": lambda: gen.complete(40),
    "complete100": lambda: gen.complete(100),
    "star": lambda: gen.star(700),
    "crown": lambda: gen.crown(30),
    "path": lambda: gen.path(1000),
    "empty": lambda: gen.empty(777),
    "single": lambda: gen.empty(1),
}


def _init_equal(gc, g, sel, X, seed, flags=0, ctx=None):
    rp, col = dev(g)
    c, st = gc.init_color(rp, col, sel, X, seed, flags=flags, ctx=ctx)
    ref = oracle.init_color(g, sel, X, seed, flags=flags)
    got = c.cpu().numpy()
    assert np.array_equal(got, ref.colors), f"{g.name}: {int((got != ref.colors).sum())} vertex colors differ"
    assert st["rounds"] == ref.stats["rounds"]
    assert st["round_sizes"] == ref.w_sizes.tolist()
    assert st["round_degsum"] == ref.w_degsum.tolist()
    assert st["losers_total"] == ref.stats["losers_total"]
    assert (st["num_colors"], st["max_color"]) == (ref.stats["num_colors"], ref.stats["max_color"])
    return c, ref


@pytest.mark.parametrize("t", [dict(compact_init=1), dict(compact_init=1, compact_sat=3), dict(compact_init=0)],
                         ids=str)
@pytest.mark.parametrize("name", sorted(GRAPHS))
def test_init_compact_copies(gc, name, t):
    """The initial coloring through each compact copy of the colors (one
    byte when the colors fit, else two bytes; a tiny saturation value sends
    most reads to the int32 colors) and without one: the oracle's colors and
    round statistics for both selections and the three priority orders."""
    g = GRAPHS[name]()
    ctx = gc.Context(max(g.n, 1), max(g.nnz, 1))
    ctx.set_tuning(**t)
    for sel, X, flags in ((gc.FIRST_FIT, 1, 0), (gc.RANDOM_X, 5, 0), (gc.RANDOM_X, 2, gc.FLAG_FIXED_PRIORITY),
                          (gc.FIRST_FIT, 1, gc.FLAG_PRIO_LF), (gc.RANDOM_X, 3, gc.FLAG_PRIO_NATURAL)):
        _init_equal(gc, g, sel, X, 13, flags=flags, ctx=ctx)
    ctx.close()


@pytest.mark.parametrize("name", sorted(GRAPHS))
def test_init_parity(gc, name):
    g = GRAPHS[name]()
    for sel, X in ((gc.FIRST_FIT, 1), (gc.RANDOM_X, 1), (gc.RANDOM_X, 4), (gc.RANDOM_X, 10)):
        for seed in (1, 77):
            _init_equal(gc, g, sel, X, seed)


def test_init_fixed_priority(gc):
    g = GRAPHS["rmat"]()
    _init_equal(gc, g, gc.FIRST_FIT, 1, 3, flags=gc.FLAG_FIXED_PRIORITY)
    _init_equal(gc, g, gc.RANDOM_X, 5, 3, flags=gc.FLAG_FIXED_PRIORITY)


@pytest.mark.parametrize("name", ["er", "mesh", "grid", "rmat", "rgg", "complete", "crown", "path", "single"])
def test_recolor_parity(gc, name):
    g = GRAPHS[name]()
    rp, col = dev(g)
    c, ref = _init_equal(gc, g, gc.RANDOM_X, 5, 11)
    rc = ref.colors
    for p in range(8):
        perm = (gc.PERM_REVERSE, gc.PERM_NONINC, gc.PERM_NONDEC, gc.PERM_RANDOM)[p % 4]
        inplace = p % 2 == 1
        out = c if inplace else None
        c2, st = gc.recolor(rp, col, c, perm, 11, p, out=out)
        r = oracle.recolor(g, rc, perm, 11, p)
        got = c2.cpu().numpy()
        assert np.array_equal(got, r.colors), f"{name} pass {p} perm {perm}: {int((got != r.colors).sum())} differ"
        assert st["k_classes"] == len(r.pi)
        assert (st["num_colors"], st["max_color"]) == (r.stats["num_colors"], r.stats["max_color"])
        c, rc = c2, r.colors


def test_validate_count_parity(gc):
    rng = np.random.default_rng(1)
    for name in ("er", "rmat", "mesh"):
        g = GRAPHS[name]()
        rp, col = dev(g)
        base = oracle.greedy_seq(g)
        for trial in range(4):
            c = base.copy()
            idx = rng.integers(0, g.n, 20)
            c[idx] = rng.integers(-2, 6, 20)  # plant conflicts and uncolored vertices
            ct = torch.from_numpy(c).cuda()
            assert gc.validate(rp, col, ct) == oracle.validate(g, c)
            assert gc.count_colors(ct) == oracle.count(c)


def _validate_expected(rp, col, c):
    """Entries (u, w), u < w, with equal positive colors; vertices with a color <= 0."""
    n = len(rp) - 1
    u = np.repeat(np.arange(n), np.diff(rp))
    w = np.asarray(col, np.int64)
    ok = (w >= 0) & (w < n) & (u < w)
    cu, cw = c[u[ok]], c[w[ok]]
    return int(((cu == cw) & (cu > 0)).sum()), int((c <= 0).sum())


def test_validate_graph_changed_in_place(gc):
    """A graph rewritten in place (same arrays, same sizes) after a validation:
    the longest row cached for the old contents is stale, and windows heavier
    than it promised are still checked where they are."""
    d = torch.device("cuda:0")
    rng = np.random.default_rng(8)
    n, deg = 1000, 40
    rp = (np.arange(n + 1) * deg).astype(np.int32)
    col = ((np.arange(n)[:, None] + np.arange(1, deg + 1)[None, :]) % n).astype(np.int32).ravel()
    rp_t, col_t = torch.from_numpy(rp).to(d), torch.from_numpy(col).to(d)
    ctx = gc.Context(n, n * deg)
    c = rng.integers(1, 6, n).astype(np.int32)
    c[rng.integers(0, n, 9)] = 0
    ct = torch.from_numpy(c).to(d)
    assert gc.validate(rp_t, col_t, ct, ctx=ctx) == _validate_expected(rp, col, c)
    # rows 0..63 now hold 600 entries each (one window of 38,400), the others 1 or 2
    lens = np.concatenate([np.full(64, 600), np.full(272, 1), np.full(664, 2)])
    assert lens.sum() == n * deg
    rp2 = np.concatenate([[0], np.cumsum(lens)]).astype(np.int32)
    col2 = rng.integers(0, n, n * deg).astype(np.int32)
    rp_t.copy_(torch.from_numpy(rp2))
    col_t.copy_(torch.from_numpy(col2))
    assert gc.validate(rp_t, col_t, ct, ctx=ctx) == _validate_expected(rp2, col2, c)
    ctx.close()


def test_validate_long_rows(gc):
    """Windows of 64 rows holding more than 4,096 entries are checked as
    (window, chunk) pairs, one wavefront per chunk; a full chunk list falls
    back to scanning the window in place.  Counts equal the oracle's
    (duplicate entries count once per copy)."""
    rng = np.random.default_rng(3)
    for g in (gen.star(10000), gen.rmat(14, 16, seed=2), gen.rmat(17, 16, seed=4), gen.complete(5000)):
        rp, col = dev(g)
        base = oracle.greedy_seq(g)
        for trial in range(3):
            c = base.copy()
            idx = rng.integers(0, g.n, 50)
            c[idx] = rng.integers(-1, 4, 50)
            if trial == 2:
                c[:] = 1
                c[rng.integers(0, g.n, 5)] = 0
            assert gc.validate(rp, col, torch.from_numpy(c).cuda()) == oracle.validate(g, c), (g.name, trial)
    # K_5000 on a context of 5,000 vertices: its 79 windows need about 6,170 chunks, so
    # the list fills part way and the later windows are scanned in place
    g = gen.complete(5000)
    rp, col = dev(g)
    ctx = gc.Context(g.n, g.nnz)
    c = rng.integers(1, 4000, g.n).astype(np.int32)
    c[rng.integers(0, g.n, 7)] = 0
    assert gc.validate(rp, col, torch.from_numpy(c).cuda(), ctx=ctx) == oracle.validate(g, c)
    ctx.close()
    # two vertices joined by 20,000 duplicate entries each way, on a context of two vertices:
    # 10 chunks do not fit the 2-entry chunk list
    d = torch.device("cuda:0")
    rp = torch.tensor([0, 20000, 40000], dtype=torch.int32, device=d)
    col = torch.cat([torch.ones(20000, dtype=torch.int32), torch.zeros(20000, dtype=torch.int32)]).to(d)
    ctx = gc.Context(2, 40000)
    assert gc.validate(rp, col, torch.tensor([3, 3], dtype=torch.int32, device=d), ctx=ctx) == (20000, 0)
    assert gc.validate(rp, col, torch.tensor([3, 4], dtype=torch.int32, device=d), ctx=ctx) == (0, 0)
    assert gc.validate(rp, col, torch.tensor([0, 4], dtype=torch.int32, device=d), ctx=ctx) == (0, 1)
    ctx.close()


def test_count_large_colors(gc):
    c = np.array([5, 2_000_000_000, 5, 7, -3, 0, 2_000_000_000, 123456789], np.int32)
    assert gc.count_colors(torch.from_numpy(c).cuda()) == oracle.count(c)


def test_check_csr(gc):
    g = GRAPHS["rmat"]()
    rp, col = dev(g)
    assert gc.check_csr(rp, col) == gc.OK
    g2 = gen.shuffle_rows(g, 3)  # unsorted rows are still valid
    assert gc.check_csr(*dev(g2)) == gc.OK
    bad = g.col.copy()
    e = int(g.row_ptr[5])
    bad[e] = 5 if g.row_ptr[6] > e else bad[e]  # self-loop
    assert gc.check_csr(rp, torch.from_numpy(bad).cuda()) == gc.ERR_GRAPH
    asym = gen.CSR(3, np.array([0, 1, 1, 1], np.int32), np.array([1], np.int32))
    assert gc.check_csr(*dev(asym)) == gc.ERR_GRAPH
    oob = g.col.copy()
    oob[0] = g.n + 3
    assert gc.check_csr(rp, torch.from_numpy(oob).cuda()) == gc.ERR_GRAPH


def test_not_converged(gc):
    g = gen.complete(30)
    rp, col = dev(g)
    c, st = gc.init_color(rp, col, gc.FIRST_FIT, 1, 4, max_rounds=7, allow_not_converged=True)
    ref = oracle.init_color(g, oracle.FIRST_FIT, 1, 4, max_rounds=7)
    assert st["status"] == gc.ERR_NOT_CONVERGED and ref.status == oracle.ERR_NOT_CONVERGED
    assert st["rounds"] == 7
    got = c.cpu().numpy()
    assert np.array_equal(got > 0, ref.colors > 0)
    assert np.array_equal(np.where(got > 0, got, 0), ref.colors)
    with pytest.raises(gc.GCError):
        gc.init_color(rp, col, gc.FIRST_FIT, 1, 4, max_rounds=7)


@pytest.mark.parametrize("max_rounds", list(range(1, 12)))
def test_round_cap_at_every_queue_position(gc, max_rounds):
    """Where no launch needs a host read, the initial coloring queues several
    rounds per read-back of the worklist counts; a round cap at any position
    of such a queue stops after exactly that round, with the oracle's colors
    and per-round statistics (K_30 with First Fit takes 30 rounds)."""
    g = gen.complete(30)
    rp, col = dev(g)
    c, st = gc.init_color(rp, col, gc.FIRST_FIT, 1, 4, max_rounds=max_rounds, allow_not_converged=True)
    ref = oracle.init_color(g, oracle.FIRST_FIT, 1, 4, max_rounds=max_rounds)
    assert st["status"] == gc.ERR_NOT_CONVERGED and ref.status == oracle.ERR_NOT_CONVERGED
    assert st["rounds"] == max_rounds == ref.stats["rounds"]
    assert st["round_sizes"] == ref.w_sizes.tolist()
    assert st["round_degsum"] == ref.w_degsum.tolist()
    got = c.cpu().numpy()
    assert np.array_equal(np.where(got > 0, got, 0), ref.colors)


def _cap_equal(gc, g, max_rounds, ctx=None):
    rp, col = dev(g)
    c, st = gc.init_color(rp, col, gc.FIRST_FIT, 1, 4, max_rounds=max_rounds, allow_not_converged=True, ctx=ctx)
    ref = oracle.init_color(g, oracle.FIRST_FIT, 1, 4, max_rounds=max_rounds)
    assert st["status"] == ref.status
    assert st["rounds"] == ref.stats["rounds"]
    assert st["round_sizes"] == ref.w_sizes.tolist()
    assert st["round_degsum"] == ref.w_degsum.tolist()
    got = c.cpu().numpy()
    assert np.array_equal(np.where(got > 0, got, 0), ref.colors)


@pytest.mark.parametrize("max_rounds", list(range(1, 20)) + [150, 151, 152, 153, 154, 155, 156, 157, 298, 299, 300, 301])
def test_round_cap_queued_with_lists(gc, max_rounds):
    """K_300: every row is long (masks and active lists, no split rows), and
    rounds are queued per read-back; a cap anywhere in a queue, and the
    natural end (300 rounds), match the oracle."""
    _cap_equal(gc, gen.complete(300), max_rounds)


@pytest.mark.parametrize("max_rounds", list(range(228, 252)) + [1, 2, 3])
def test_round_cap_split_then_queued(gc, max_rounds):
    """K_300 with rows split at 64 entries: the split path runs round by round
    until the rows' active lists fall under the threshold, then rounds are
    queued; caps around that switch match the oracle."""
    g = gen.complete(300)
    ctx = gc.Context(g.n, g.nnz)
    ctx.set_tuning(deg_wave=32, deg_split=64, split_len=64)
    _cap_equal(gc, g, max_rounds, ctx)
    ctx.close()


@pytest.mark.parametrize("extra", [0, 1, 2, 3, 4, 5, 6, 7, 8, 9])
def test_queued_rounds_end_anywhere_lists(gc, extra):
    """An RMAT graph with long rows (masks and lists): caps from the round
    count R to R + 9 all converge with the oracle's colors and statistics."""
    g = gen.rmat(12, 16, seed=5)
    ref = oracle.init_color(g, oracle.RANDOM_X, 4, 9)
    R = ref.stats["rounds"]
    rp, col = dev(g)
    c, st = gc.init_color(rp, col, gc.RANDOM_X, 4, 9, max_rounds=R + extra)
    assert st["rounds"] == R
    assert st["round_sizes"] == ref.w_sizes.tolist()
    assert st["round_degsum"] == ref.w_degsum.tolist()
    assert np.array_equal(c.cpu().numpy(), ref.colors)


@pytest.mark.parametrize("extra", [0, 1, 2, 3, 4, 5])
def test_queued_rounds_end_anywhere(gc, extra):
    """The coloring ends at every offset inside a queue of rounds: caps from
    the round count R to R + 5 all converge with the same colors and the
    same per-round statistics as the oracle (empty queued rounds leave no
    trace)."""
    g = gen.er(3001, 15007, 3)
    ref = oracle.init_color(g, oracle.RANDOM_X, 4, 9)
    R = ref.stats["rounds"]
    rp, col = dev(g)
    c, st = gc.init_color(rp, col, gc.RANDOM_X, 4, 9, max_rounds=R + extra)
    assert st["rounds"] == R
    assert st["round_sizes"] == ref.w_sizes.tolist()
    assert st["round_degsum"] == ref.w_degsum.tolist()
    assert np.array_equal(c.cpu().numpy(), ref.colors)


def test_empty_graph_and_bad_args(gc):
    rp = torch.zeros(1, dtype=torch.int32, device="cuda")
    col = torch.zeros(0, dtype=torch.int32, device="cuda")
    c, st = gc.init_color(rp, col)
    assert c.numel() == 0 and st["rounds"] == 0 and st["num_colors"] == 0
    c2, st2 = gc.recolor(rp, col, c)
    assert st2["num_colors"] == 0
    g = GRAPHS["er"]()
    rpg, colg = dev(g)
    with pytest.raises(gc.GCError) as e:
        gc.init_color(rpg, colg, gc.RANDOM_X, 0)
    assert e.value.status == gc.ERR_ARG
    with pytest.raises(gc.GCError) as e:
        gc.recolor(rpg, colg, torch.zeros(g.n, dtype=torch.int32, device="cuda"))
    assert e.value.status == gc.ERR_COLORING
    with pytest.raises(TypeError):
        gc.init_color(rpg.long(), colg)


def test_many_small_random_graphs(gc):
    rng = np.random.default_rng(123)
    for t in range(60):
        n = int(rng.integers(1, 200))
        m = int(rng.integers(0, min(n * (n - 1) // 2, 6 * n) + 1))
        g = gen.er(n, m, int(rng.integers(1, 10**9))) if n >= 2 else gen.empty(n)
        sel = int(rng.integers(0, 2))
        X = int(rng.integers(1, 12))
        seed = int(rng.integers(1, 2**63))
        c, ref = _init_equal(gc, g, sel, X, seed)
        if g.n:
            rp, col = dev(g)
            perm = int(rng.integers(0, 4))
            c2, _ = gc.recolor(rp, col, c, perm, seed, t)
            assert np.array_equal(c2.cpu().numpy(), oracle.recolor(g, ref.colors, perm, seed, t).colors)


TUNINGS = [
    dict(group=1, walk_group=1), dict(group=2, walk_group=2), dict(group=4, walk_group=4), dict(group=16, walk_group=16),
    dict(group=32, walk_group=32), dict(group=64, walk_group=64), dict(group=8, walk_group=0), dict(group=2, walk_group=16),
    dict(deg_wave=0), dict(deg_wave=4), dict(deg_wave=1 << 30),
    dict(walk_mode=1), dict(walk_mode=1, deg_wave=3),
    dict(xcd_chunks=1), dict(xcd_chunks=1, group=4, deg_wave=16),
    dict(block=64, grid_per_cu=1), dict(block=1024, grid_per_cu=2),
    dict(deg_split=0), dict(deg_wave=4, deg_split=16, split_len=64),
    dict(deg_wave=8, deg_split=64, split_len=64, group=8, xcd_chunks=1),
    dict(deg_wave=4, deg_split=16, split_len=64, hub_words=1),
    dict(tail_max=-1), dict(tail_max=1 << 30), dict(tail_max=1 << 30, deg_wave=4),
    dict(walk_flags=1), dict(walk_flags=2), dict(walk_flags=3, deg_wave=4, deg_split=16, split_len=64),
    dict(walk_flags=4), dict(walk_flags=4, deg_wave=4, deg_split=16, split_len=64),
    dict(deg_wave=1024, walk_group=2, deg_split=0),  # 512 entries per lane: late batches wait in place
    dict(compact_init=1), dict(compact_init=1, tail_max=1 << 30), dict(compact_init=0),
    dict(compact_init=1, compact_sat=5), dict(compact_init=1, compact_sat=1, deg_wave=4),
]


@pytest.mark.parametrize("name", ["rmat", "mesh", "star", "complete", "complete100"])
def test_tuning_invariance(gc, name):
    """No tuning knob changes any color (integer work: bit-exact)."""
    g = GRAPHS[name]()
    rp, col = dev(g)
    ref = oracle.init_color(g, oracle.RANDOM_X, 4, 9)
    passes = [(p, (gc.PERM_NONINC, gc.PERM_RANDOM, gc.PERM_REVERSE)[p % 3]) for p in range(3)]
    refs = []
    c = ref.colors
    for p, perm in passes:
        c = oracle.recolor(g, c, perm, 9, p).colors
        refs.append(c)
    for t in TUNINGS:
        ctx = gc.Context(g.n, g.nnz)
        ctx.set_tuning(**t)
        cur, st = gc.init_color(rp, col, gc.RANDOM_X, 4, 9, ctx=ctx)
        assert np.array_equal(cur.cpu().numpy(), ref.colors), t
        for (p, perm), r in zip(passes, refs):
            cur, _ = gc.recolor(rp, col, cur, perm, 9, p, out=cur, ctx=ctx)
            assert np.array_equal(cur.cpu().numpy(), r), (t, p)
        ctx.close()


def test_recolor_without_stats_matches(gc):
    """The asynchronous path (no stats, no host synchronisation) gives the same colors."""
    g = GRAPHS["rmat"]()
    rp, col = dev(g)
    c0 = oracle.init_color(g, oracle.FIRST_FIT, 1, 2).colors
    c = torch.from_numpy(c0.copy()).cuda()
    exp = c0
    for p in range(6):
        c, st = gc.recolor(rp, col, c, gc.PERM_RANDOM, 2, p, out=c, stats=False)
        assert st is None
        exp = oracle.recolor(g, exp, oracle.PERM_RANDOM, 2, p).colors
    torch.cuda.synchronize()
    assert np.array_equal(c.cpu().numpy(), exp)


MANY_CLASS_TUNINGS = [
    dict(),                                         # rows in the wavefront bin, LDS mask words
    dict(group=1, deg_wave=512),                    # one lane per row: 64-color windows beyond the LDS word
    dict(group=4, deg_wave=512),
    dict(deg_wave=16, deg_split=128, split_len=64),  # split rows, multi-word hub bitmaps
    dict(deg_wave=16, deg_split=128, split_len=64, hub_words=1),  # ranks >= 64: long rows on one wavefront
    dict(deg_wave=16, deg_split=128, split_len=64, walk_flags=3),  # split rows first, early merge of sub-chunks
    dict(deg_wave=16, deg_split=64, split_len=64, walk_flags=2),
    dict(walk_flags=1),
    dict(walk_flags=4),
    dict(deg_wave=16, deg_split=128, split_len=64, walk_flags=4),
    dict(walk_mode=1),
]


@pytest.mark.parametrize("t", MANY_CLASS_TUNINGS, ids=str)
def test_recolor_many_classes(gc, t):
    """K_300 from a random proper coloring (300 classes, every rank >= 64 needs
    colors above the first 64): all walk paths against the oracle."""
    g = gen.complete(300)
    rp, col = dev(g)
    rng = np.random.default_rng(11)
    c0 = (rng.permutation(300) + 1).astype(np.int32)
    ctx = gc.Context(g.n, g.nnz)
    ctx.set_tuning(**t)
    exp = c0
    cur = torch.from_numpy(c0.copy()).cuda()
    for p, perm in enumerate((gc.PERM_REVERSE, gc.PERM_RANDOM, gc.PERM_NONINC, gc.PERM_RANDOM)):
        cur, st = gc.recolor(rp, col, cur, perm, 5, p, out=cur, ctx=ctx)
        exp = oracle.recolor(g, exp, perm, 5, p).colors
        assert np.array_equal(cur.cpu().numpy(), exp), (t, p)
        assert st["num_colors"] == 300
    ctx.close()


def test_recolor_beyond_hub_ranks(gc):
    """K_4200 colored 1..4200: rows longer than the split threshold at ranks
    below 4096 take the split path, those above the wavefront bin."""
    g = gen.complete(4200)
    rp, col = dev(g)
    c0 = np.arange(1, 4201, dtype=np.int32)
    cur = torch.from_numpy(c0.copy()).cuda()
    exp = c0
    for p, perm in enumerate((gc.PERM_RANDOM, gc.PERM_NONINC)):
        print(f"[K_4200] pass {p}", flush=True)
        cur, st = gc.recolor(rp, col, cur, perm, 3, p, out=cur)
        exp = oracle.recolor(g, exp, perm, 3, p).colors
        assert np.array_equal(cur.cpu().numpy(), exp), p


SPLIT_TUNINGS = [
    dict(deg_wave=8, deg_split=64, split_len=64),
    dict(deg_wave=8, deg_split=64, split_len=64, hub_words=1),  # colors above 64: the row is rescanned
    dict(deg_wave=0, deg_split=1, split_len=64, group=1),        # every row of 2+ entries split
    dict(deg_wave=8, deg_split=64, split_len=64, walk_flags=3),  # split rows first, early merge
    dict(deg_wave=0, deg_split=1, split_len=64, group=1, walk_flags=2),
    dict(deg_wave=8, deg_split=64, split_len=64, walk_flags=4),
    dict(deg_wave=8, deg_split=64, split_len=64, compact_init=1),  # split rows write the compact copy too
    dict(deg_wave=8, deg_split=64, split_len=64, compact_init=1, compact_sat=3),
    dict(deg_wave=0, deg_split=1, split_len=64, group=1, compact_init=1, compact_sat=2),
]


@pytest.mark.parametrize("t", SPLIT_TUNINGS, ids=str)
@pytest.mark.parametrize("name", ["rmat", "star", "complete100", "er"])
def test_init_split_rows(gc, name, t):
    """Initial coloring with long rows split across wavefronts (round 0 and
    later rounds, First Fit and Random-X) against the oracle."""
    g = GRAPHS[name]()
    ctx = gc.Context(g.n, g.nnz)
    ctx.set_tuning(**t)
    for sel, X, seed in ((gc.FIRST_FIT, 1, 4), (gc.RANDOM_X, 7, 5)):
        _init_equal(gc, g, sel, X, seed, ctx=ctx)
    ctx.close()


def test_init_split_many_colors(gc):
    """K_300 with First Fit (one vertex per round, colors up to 300) under
    split rows with one hub word: every round past color 64 rescans."""
    g = gen.complete(300)
    ctx = gc.Context(g.n, g.nnz)
    ctx.set_tuning(deg_wave=16, deg_split=128, split_len=64, hub_words=1)
    c, ref = _init_equal(gc, g, gc.FIRST_FIT, 1, 6, ctx=ctx)
    assert ref.stats["rounds"] == 300
    ctx.close()


@pytest.mark.parametrize("name", ["er", "rmat", "mesh"])
def test_presets(gc, name):
    """"speed" = First Fit alone; "quality" = Random-X (X = 5) + one ND pass (section 4.3)."""
    g = GRAPHS[name]()
    rp, col = dev(g)
    c, st = gc.color_preset(rp, col, gc.PRESET_SPEED, 13)
    ref = oracle.init_color(g, oracle.FIRST_FIT, 1, 13)
    assert np.array_equal(c.cpu().numpy(), ref.colors) and st["rounds"] == ref.stats["rounds"]
    c, st = gc.color_preset(rp, col, gc.PRESET_QUALITY, 13)
    ref = oracle.init_color(g, oracle.RANDOM_X, 5, 13)
    exp = oracle.recolor(g, ref.colors, oracle.PERM_NONDEC, 13, 0)
    assert np.array_equal(c.cpu().numpy(), exp.colors)
    assert st["rounds"] == ref.stats["rounds"] and st["num_colors"] == exp.stats["num_colors"]


@pytest.mark.parametrize("kind,x", [(1, 3), (2, 0)])
def test_hybrid_schedules(gc, kind, x):
    """ND-RAND%x and ND-RAND%2^i over 9 iterations against the oracle."""
    g = GRAPHS["rgg"]()
    rp, col = dev(g)
    c0 = oracle.init_color(g, oracle.FIRST_FIT, 1, 21).colors
    cur = torch.from_numpy(c0.copy()).cuda()
    exp = c0
    for t in range(1, 10):
        perm = gc.schedule_perm(kind, 0, x, t)
        assert perm == oracle.schedule_perm(kind, 0, x, t)
        cur, _ = gc.recolor(rp, col, cur, perm, 21, t - 1, out=cur)
        exp = oracle.recolor(g, exp, perm, 21, t - 1).colors
        assert np.array_equal(cur.cpu().numpy(), exp), t


@pytest.mark.parametrize("name", ["er", "mesh", "grid", "rmat", "rgg", "complete100", "star", "crown", "path", "single"])
def test_arc_parity(gc, name):
    """Asynchronous recoloring (aRC) against the oracle, every class order."""
    g = GRAPHS[name]()
    rp, col = dev(g)
    c0 = oracle.init_color(g, oracle.RANDOM_X, 3, 8).colors
    cin = torch.from_numpy(c0.copy()).cuda()
    for perm in range(4):
        c, st = gc.arc_recolor(rp, col, cin, perm, 8, 2)
        ref = oracle.arc_recolor(g, c0, perm, 8, 2)
        assert np.array_equal(c.cpu().numpy(), ref.colors), (name, perm)
        assert st["rounds"] == ref.stats["rounds"] and st["num_colors"] == ref.stats["num_colors"]


def test_arc_tunings_and_in_place(gc):
    g = GRAPHS["rmat"]()
    rp, col = dev(g)
    c0 = oracle.init_color(g, oracle.FIRST_FIT, 1, 4).colors
    ref = oracle.arc_recolor(g, c0, oracle.PERM_RANDOM, 4, 5).colors
    for t in (dict(), dict(group=1, deg_wave=8), dict(deg_wave=4, deg_split=16, split_len=64),
              dict(group=64, deg_wave=0)):
        ctx = gc.Context(g.n, g.nnz)
        ctx.set_tuning(**t)
        cur = torch.from_numpy(c0.copy()).cuda()
        cur, _ = gc.arc_recolor(rp, col, cur, gc.PERM_RANDOM, 4, 5, out=cur, ctx=ctx)
        assert np.array_equal(cur.cpu().numpy(), ref), t
        ctx.close()


@pytest.mark.parametrize("flags", [1, 2, 4], ids=["fixed", "lf", "natural"])
@pytest.mark.parametrize("name", ["er", "mesh", "grid", "rmat", "star", "complete100", "path"])
def test_init_priority_orders(gc, name, flags):
    """Initial coloring under the fixed random order, Largest First and the
    natural order (first fit and Random-X) against the oracle."""
    g = GRAPHS[name]()
    for sel, X in ((gc.FIRST_FIT, 1), (gc.RANDOM_X, 4)):
        _init_equal(gc, g, sel, X, 17, flags=flags)


def test_init_priority_orders_split_rows(gc):
    g = GRAPHS["rmat"]()
    ctx = gc.Context(g.n, g.nnz)
    ctx.set_tuning(deg_wave=8, deg_split=64, split_len=64)
    for flags in (2, 4):
        _init_equal(gc, g, gc.FIRST_FIT, 1, 19, flags=flags, ctx=ctx)
    ctx.close()


@pytest.mark.parametrize("name", ["mesh", "grid", "er", "path"])
def test_recolor_unaligned_col(gc, name):
    """col_idx that starts 4 bytes past a 16-byte boundary (a view into a
    larger buffer): same colors as the oracle."""
    g = GRAPHS[name]()
    d = torch.device("cuda:0")
    rp = torch.from_numpy(np.ascontiguousarray(g.row_ptr)).to(d)
    big = torch.zeros(g.nnz + 4, dtype=torch.int32, device=d)
    big[1:1 + g.nnz] = torch.from_numpy(np.ascontiguousarray(g.col)).to(d)
    col = big[1:1 + g.nnz]
    assert col.data_ptr() % 16 == 4
    ref = oracle.init_color(g, oracle.RANDOM_X, 3, 5).colors
    c = torch.from_numpy(ref.copy()).to(d)
    for p, perm in enumerate((gc.PERM_REVERSE, gc.PERM_NONINC, gc.PERM_RANDOM)):
        c, _ = gc.recolor(rp, col, c, perm, 5, p, out=c)
        ref = oracle.recolor(g, ref, perm, 5, p).colors
        assert np.array_equal(c.cpu().numpy(), ref), f"{name} pass {p}"


TAIL = [dict(tail_max=-1), dict(tail_max=0), dict(tail_max=1 << 30), dict(tail_max=1 << 30, deg_wave=8),
        dict(tail_max=1 << 30, deg_split=0), dict(tail_max=50), dict(tail_max=16384), dict(tail_max=-1, compact_init=1),
        dict(tail_max=1 << 30, compact_init=1), dict(tail_max=1 << 30, compact_init=1, compact_sat=4)]


@pytest.mark.parametrize("name", ["er", "rmat", "mesh", "star", "complete100", "path", "rgg", "crown"])
@pytest.mark.parametrize("t", TAIL, ids=str)
def test_init_tail_rounds(gc, name, t):
    """The persistent launch that runs the last rounds of the initial coloring
    (from round 1 with tail_max = 2^30) gives the oracle's colors, rounds,
    round sizes and degree sums, for every selection and conflict priority."""
    g = GRAPHS[name]()
    ctx = gc.Context(g.n, g.nnz)
    ctx.set_tuning(**t)
    for sel, X, flags in ((gc.FIRST_FIT, 1, 0), (gc.RANDOM_X, 4, 0), (gc.RANDOM_X, 3, gc.FLAG_FIXED_PRIORITY),
                          (gc.FIRST_FIT, 1, gc.FLAG_PRIO_LF), (gc.RANDOM_X, 2, gc.FLAG_PRIO_NATURAL)):
        _init_equal(gc, g, sel, X, 5, flags=flags, ctx=ctx)
    ctx.close()


@pytest.mark.parametrize("max_rounds", [1, 2, 3, 5, 8, 13])
def test_init_tail_round_cap(gc, max_rounds):
    """A round cap that falls inside the persistent tail launch stops it there
    (GC_ERR_NOT_CONVERGED, the same colors and statistics as the oracle)."""
    g = GRAPHS["complete"]()
    rp, col = dev(g)
    ctx = gc.Context(g.n, g.nnz)
    ctx.set_tuning(tail_max=1 << 30)
    c, st = gc.init_color(rp, col, gc.FIRST_FIT, 1, 3, max_rounds=max_rounds, ctx=ctx, allow_not_converged=True)
    ref = oracle.init_color(g, oracle.FIRST_FIT, 1, 3, max_rounds=max_rounds)
    assert st["status"] == gc.ERR_NOT_CONVERGED and ref.status == oracle.ERR_NOT_CONVERGED
    got = c.cpu().numpy()
    assert np.array_equal(np.where(got > 0, got, 0), ref.colors)
    assert st["rounds"] == ref.stats["rounds"] == max_rounds
    assert st["round_sizes"] == ref.w_sizes.tolist()
    assert st["round_degsum"] == ref.w_degsum.tolist()
    ctx.close()


def test_arc_tail_rounds(gc):
    """Asynchronous recoloring's rounds (class-rank priorities) through the tail launch."""
    g = GRAPHS["rmat"]()
    rp, col = dev(g)
    ctx = gc.Context(g.n, g.nnz)
    ctx.set_tuning(tail_max=1 << 30)
    c, _ = gc.init_color(rp, col, gc.RANDOM_X, 4, 2, ctx=ctx)
    for p, perm in enumerate((gc.PERM_NONINC, gc.PERM_RANDOM)):
        ref = oracle.arc_recolor(g, c.cpu().numpy(), perm, 2, p)
        c, st = gc.arc_recolor(rp, col, c, perm, 2, p, out=c, ctx=ctx)
        assert np.array_equal(c.cpu().numpy(), ref.colors)
        assert st["rounds"] == ref.stats["rounds"]
    ctx.close()


ROUND_TUNINGS = [dict(), dict(deg_wave=8, deg_split=64, split_len=64), dict(tail_max=1 << 30),
                 dict(compact_init=1, compact_sat=3), dict(group=1, deg_wave=4)]


@pytest.mark.parametrize("t", ROUND_TUNINGS, ids=str)
@pytest.mark.parametrize("name", ["er", "rmat", "mesh", "star", "complete100", "path", "rgg", "crown", "empty"])
def test_init_commit_rounds(gc, name, t):
    """Each vertex's commit round (gc_init_color_rounds) equals the oracle's,
    vertex by vertex, on every launch path: lane groups, wavefront rows,
    split rows, the persistent tail and the compact copies; a round cap leaves
    -1 for the vertices still uncolored."""
    g = GRAPHS[name]()
    rp, col = dev(g)
    ctx = gc.Context(max(g.n, 1), max(g.nnz, 1))
    ctx.set_tuning(**t)
    for sel, X, flags, cap in ((gc.FIRST_FIT, 1, 0, 0), (gc.RANDOM_X, 4, 0, 0), (gc.RANDOM_X, 2, gc.FLAG_PRIO_LF, 0),
                               (gc.FIRST_FIT, 1, gc.FLAG_PRIO_NATURAL, 0), (gc.FIRST_FIT, 1, 0, 2)):
        c, vr, st = gc.init_color_rounds(rp, col, sel, X, 5, max_rounds=cap, flags=flags, ctx=ctx,
                                         allow_not_converged=True)
        ref, cr = oracle.init_color_rounds(g, sel, X, 5, max_rounds=cap, flags=flags)
        got = c.cpu().numpy()
        assert np.array_equal(np.where(got > 0, got, 0), ref.colors)
        assert np.array_equal(vr.cpu().numpy(), cr), f"{name} {t} sel={sel} flags={flags} cap={cap}"
        assert st["rounds"] == ref.stats["rounds"]
    ctx.close()


def test_init_commit_rounds_args(gc):
    g = GRAPHS["er"]()
    rp, col = dev(g)
    with pytest.raises(gc.GCError):
        gc.init_color_rounds(rp, col, gc.FIRST_FIT, 1, 1, flags=gc.FLAG_DISTANCE2)
    c, vr, st = gc.init_color_rounds(rp, col, gc.FIRST_FIT, 1, 1)
    c2, _ = gc.init_color(rp, col, gc.FIRST_FIT, 1, 1)
    assert torch.equal(c, c2)
