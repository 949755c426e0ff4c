"""Pins for the CPU oracle: published values, closed forms, brute force and
invariants that a plausible mistake in the oracle (a dropped term, a wrong
sign or index, a swapped operand) would break.  CPU only."""
import itertools
import os

import numpy as np
import pytest

import gen
import oracle

GOLD = os.path.join(os.path.dirname(__file__), "golden")
M32 = 0xFFFFFFFF


# ---------------------------------------------------------------- hash

def _read_vectors():
    rows = []
    with open(os.path.join(GOLD, "hash_vectors.txt")) as f:
        for line in f:
            line = line.split("#")[0].strip()
            if line:
                kind, a, b = line.split()
                rows.append((kind, int(a, 16), int(b, 16)))
    return rows


def test_hash_published_vectors():
    rows = _read_vectors()
    assert len(rows) == 6
    for kind, a, b in rows:
        got = oracle.mix64(a) if kind == "mix64" else oracle.fmix32(a)
        assert got == b, (kind, hex(a), hex(got), hex(b))


def test_fmix32_is_bijection():
    # invert with multiplicative inverses mod 2^32 and xorshift inverses
    def unxorshift(h, s):
        x = h
        for _ in range(32 // s + 1):
            x = h ^ (x >> s)
        return x & M32

    inv1, inv2 = pow(0x85EBCA6B, -1, 2**32), pow(0xC2B2AE35, -1, 2**32)
    rng = np.random.default_rng(5)
    for x in rng.integers(0, 2**32, 2000, dtype=np.uint64).tolist():
        h = oracle.fmix32(x)
        h = unxorshift(h, 16)
        h = (h * inv2) & M32
        h = unxorshift(h, 13)
        h = (h * inv1) & M32
        h = unxorshift(h, 16)
        assert h == x


def test_priority_keys_unique_and_pick_in_range():
    seed = 12345
    for r in (0, 1, 7):
        prios = {oracle.prio(seed, r, v) for v in range(3000)}
        assert len(prios) == 3000  # bijection of v for a fixed round
        assert all(oracle.key(seed, r, v) == (oracle.prio(seed, r, v) << 32 | v) for v in range(0, 3000, 97))
    for X in (1, 2, 4, 5, 10, 50):
        picks = [oracle.pick(seed, 3, v, X) for v in range(2000)]
        assert min(picks) >= 0 and max(picks) < X
        if X == 1:
            assert set(picks) == {0}
    # rounds and tags give different streams
    assert oracle.stream(1, 1, 0) != oracle.stream(1, 1, 1)
    assert oracle.stream(1, 1, 0) != oracle.stream(1, 2, 0)


def test_pick_uniform_chi2():
    X, N = 5, 50000
    counts = np.bincount([oracle.pick(7, 0, v, X) for v in range(N)], minlength=X)
    chi2 = float(((counts - N / X) ** 2 / (N / X)).sum())
    assert chi2 < 20.5  # 4 dof, p ~ 0.0004


# ---------------------------------------------------------------- Algorithm 1 closed forms

def test_greedy_path_cycles_complete_star():
    for n in (1, 2, 5, 8):
        c = oracle.greedy_seq(gen.path(n))
        assert c.tolist() == [1 + (i & 1) for i in range(n)]
    for n in (4, 6, 10):
        c = oracle.greedy_seq(gen.cycle(n))
        assert c.tolist() == [1 + (i & 1) for i in range(n)]
    for n in (3, 5, 9):
        c = oracle.greedy_seq(gen.cycle(n))
        assert c.tolist() == [1 + (i & 1) for i in range(n - 1)] + [3]
    for n in (1, 4, 9):
        assert oracle.greedy_seq(gen.complete(n)).tolist() == list(range(1, n + 1))
    c = oracle.greedy_seq(gen.star(6))
    assert c.tolist() == [1] + [2] * 6


def test_greedy_crown_orders():
    for m in (3, 5, 8):
        inter = oracle.greedy_seq(gen.crown(m, interleaved=True))
        # u_i and v_i both get colour i+1: Delta + 1 = m colours, the bound is tight
        assert inter.tolist() == [i // 2 + 1 for i in range(2 * m)]
        bip = oracle.greedy_seq(gen.crown(m, interleaved=False))
        assert bip.tolist() == [1] * m + [2] * m


def test_greedy_grids_and_mesh():
    N = 7
    c = oracle.greedy_seq(gen.grid5(N))
    assert c.tolist() == [1 + ((x + y) & 1) for y in range(N) for x in range(N)]
    c = oracle.greedy_seq(gen.grid9(N))
    assert c.tolist() == [1 + (x & 1) + 2 * (y & 1) for y in range(N) for x in range(N)]
    N = 6
    c = oracle.greedy_seq(gen.mesh27(N))
    exp = [1 + (x & 1) + 2 * (y & 1) + 4 * (z & 1) for z in range(N) for y in range(N) for x in range(N)]
    assert c.tolist() == exp  # 8 colours = chromatic number (every 2x2x2 block is K_8)


def _random_graph(n, p, rng):
    pairs = [(i, j) for i in range(n) for j in range(i + 1, n) if rng.random() < p]
    return gen.from_pairs(n, pairs) if pairs else gen.empty(n)


def test_greedy_some_order_is_optimal_and_bound():
    rng = np.random.default_rng(11)
    for _ in range(6):
        n = int(rng.integers(4, 8))
        g = _random_graph(n, 0.5, rng)
        chi = oracle.chromatic(g)
        best = min(int(oracle.greedy_seq(g, np.array(o)).max()) for o in itertools.permutations(range(n)))
        assert best == chi
        for _ in range(20):
            c = oracle.greedy_seq(g, rng.permutation(n))
            assert c.max() <= g.max_deg + 1 and oracle.validate(g, c) == (0, 0)


def test_chromatic_known_graphs():
    pet = gen.from_pairs(10, [(i, (i + 1) % 5) for i in range(5)] + [(5 + i, 5 + (i + 2) % 5) for i in range(5)]
                         + [(i, i + 5) for i in range(5)])
    wheel5 = gen.from_pairs(6, [(i, (i + 1) % 5) for i in range(5)] + [(5, i) for i in range(5)])
    assert oracle.chromatic(pet) == 3
    assert oracle.chromatic(wheel5) == 4
    assert oracle.chromatic(gen.cycle(7)) == 3
    assert oracle.chromatic(gen.cycle(8)) == 2
    assert oracle.chromatic(gen.complete(6)) == 6
    assert oracle.chromatic(gen.crown(5)) == 2
    assert oracle.chromatic(gen.empty(4)) == 1
    assert oracle.chromatic(gen.mesh27(2)) == 8


def test_chromatic_vs_exhaustive_python():
    rng = np.random.default_rng(3)
    for _ in range(8):
        n = int(rng.integers(3, 7))
        g = _random_graph(n, 0.55, rng)
        edges = [(u, int(w)) for u in range(n) for w in g.neighbors(u) if u < w]
        chi = next(k for k in range(1, n + 1)
                   if any(all(c[a] != c[b] for a, b in edges) for c in itertools.product(range(k), repeat=n)))
        assert oracle.chromatic(g) == chi


# ---------------------------------------------------------------- count / validate

def test_count_validate_bruteforce_and_injected():
    rng = np.random.default_rng(2)
    for _ in range(10):
        n = int(rng.integers(2, 30))
        g = _random_graph(n, 0.3, rng)
        c = rng.integers(-1, 5, n).astype(np.int32)
        pos = [x for x in c.tolist() if x > 0]
        assert oracle.count(c) == (len(set(pos)), max(pos) if pos else 0)
        cf = sum(1 for u in range(n) for w in g.neighbors(u) if u < w and c[u] > 0 and c[u] == c[w])
        assert oracle.validate(g, c) == (cf, int((c <= 0).sum()))
    g = gen.mesh27(5)
    c = oracle.greedy_seq(g)
    assert oracle.validate(g, c) == (0, 0)
    # plant exactly one conflicting edge: copy a neighbour's colour onto an isolated-colour setting
    c2 = c.copy()
    c2[0] = 9  # vertex 0 alone in colour 9
    w = int(g.neighbors(0)[0])
    c2[w] = 9
    assert oracle.validate(g, c2) == (1, 0)
    c2[1] = 0
    assert oracle.validate(g, c2)[1] == 1


def test_check_csr():
    assert oracle.check_csr(gen.mesh27(3)) == 0
    g = gen.path(4)
    bad = gen.CSR(g.n, g.row_ptr.copy(), g.col.copy())
    bad.col[0] = 0  # self-loop on vertex 0
    assert oracle.check_csr(bad) == oracle.ERR_GRAPH
    asym = gen.CSR(3, np.array([0, 1, 1, 1], np.int32), np.array([1], np.int32))
    assert oracle.check_csr(asym) == oracle.ERR_GRAPH


# ---------------------------------------------------------------- speculative initial colouring

FAMILIES = [
    lambda: gen.er(300, 1500, 4),
    lambda: gen.mesh27(6),
    lambda: gen.grid5(17, 13),
    lambda: gen.rmat(9, 8, seed=2),
    lambda: gen.rgg(400, 0.09, 3),
    lambda: gen.complete(12),
    lambda: gen.star(40),
    lambda: gen.crown(7),
    lambda: gen.empty(10),
]


def _grundy_ok(g, c):
    for v in range(g.n):
        nb = {int(c[w]) for w in g.neighbors(v)}
        if any(k not in nb for k in range(1, int(c[v]))):
            return False
    return True


@pytest.mark.parametrize("fam", range(len(FAMILIES)))
def test_init_invariants(fam):
    g = FAMILIES[fam]()
    for seed in (1, 99):
        ff = oracle.init_color(g, oracle.FIRST_FIT, 1, seed)
        assert ff.status == 0
        assert oracle.validate(g, ff.colors) == (0, 0)
        assert _grundy_ok(g, ff.colors)
        deg = g.degrees
        assert np.all(ff.colors <= deg + 1)
        assert ff.stats["rounds"] == len(ff.w_sizes) and (g.n == 0 or ff.w_sizes[0] == g.n)
        assert np.all(np.diff(ff.w_sizes) < 0)  # the top key of each component always survives
        assert ff.stats["losers_total"] == int(ff.w_sizes.sum()) - g.n
        assert ff.w_degsum[0] == g.nnz
        for X in (4, 10):
            rx = oracle.init_color(g, oracle.RANDOM_X, X, seed)
            assert oracle.validate(g, rx.colors) == (0, 0)
            assert np.all(rx.colors <= deg + X)
        x1 = oracle.init_color(g, oracle.RANDOM_X, 1, seed)
        assert np.array_equal(x1.colors, ff.colors) and np.array_equal(x1.w_sizes, ff.w_sizes)


def test_init_vs_chromatic_exhaustive_small():
    # every labelled graph on 5 vertices (1024 graphs)
    n = 5
    pairs = [(i, j) for i in range(n) for j in range(i + 1, n)]
    for mask in range(1 << len(pairs)):
        g = gen.from_pairs(n, [p for b, p in enumerate(pairs) if mask >> b & 1]) if mask else gen.empty(n)
        chi = oracle.chromatic(g)
        r = oracle.init_color(g, oracle.FIRST_FIT, 1, mask)
        assert oracle.validate(g, r.colors) == (0, 0)
        k = oracle.count(r.colors)[0]
        assert chi <= k <= g.max_deg + 1
        rc = oracle.recolor(g, r.colors, oracle.PERM_REVERSE, 1, 0)
        assert chi <= rc.stats["num_colors"] <= k


def test_init_edgeless():
    g = gen.empty(50)
    r = oracle.init_color(g, oracle.FIRST_FIT, 1, 3)
    assert r.colors.tolist() == [1] * 50 and r.rounds == 1
    r = oracle.init_color(g, oracle.RANDOM_X, 6, 3)
    assert r.rounds == 1
    assert r.colors.tolist() == [oracle.pick(3, 0, v, 6) + 1 for v in range(50)]


def test_init_first_round_local_maxima():
    g = gen.er(400, 1200, 9)
    seed = 17
    r = oracle.init_color(g, oracle.FIRST_FIT, 1, seed, max_rounds=1)
    assert r.status == oracle.ERR_NOT_CONVERGED and r.rounds == 1
    for v in range(g.n):
        kv = oracle.key(seed, 0, v)
        is_max = all(oracle.key(seed, 0, int(w)) < kv for w in g.neighbors(v))
        assert r.colors[v] == (1 if is_max else 0)


def test_init_complete_graph_one_per_round():
    n, seed = 9, 5
    g = gen.complete(n)
    r = oracle.init_color(g, oracle.FIRST_FIT, 1, seed)
    assert r.rounds == n and r.w_sizes.tolist() == list(range(n, 0, -1))
    left = set(range(n))
    for rnd in range(n):
        top = max(left, key=lambda v: oracle.key(seed, rnd, v))
        assert r.colors[top] == rnd + 1
        left.remove(top)
    # fixed-priority reading: the order of the colours follows key_0 alone
    f = oracle.init_color(g, oracle.FIRST_FIT, 1, seed, flags=oracle.FIXED_PRIORITY)
    order = sorted(range(n), key=lambda v: -oracle.key(seed, 0, v))
    assert [int(f.colors[v]) for v in order] == list(range(1, n + 1))


def test_init_star():
    for seed in range(1, 30):
        g = gen.star(12)
        r = oracle.init_color(g, oracle.FIRST_FIT, 1, seed)
        assert r.rounds == 2 and oracle.count(r.colors) == (2, 2)
        center_wins = oracle.key(seed, 0, 0) > max(oracle.key(seed, 0, v) for v in range(1, 13))
        assert (r.colors[0] == 1) == center_wins


def test_init_schedule_independence():
    g = gen.rmat(10, 8, seed=4)
    g2 = gen.shuffle_rows(g, 8)
    for sel, X in ((oracle.FIRST_FIT, 1), (oracle.RANDOM_X, 5)):
        a = oracle.init_color(g, sel, X, 21)
        b = oracle.init_color(g2, sel, X, 21)
        assert np.array_equal(a.colors, b.colors) and np.array_equal(a.w_sizes, b.w_sizes)


def test_init_not_converged_cap():
    g = gen.complete(6)
    r = oracle.init_color(g, oracle.FIRST_FIT, 1, 1, max_rounds=3)
    assert r.status == oracle.ERR_NOT_CONVERGED and r.rounds == 3
    assert int((r.colors > 0).sum()) == 3


@pytest.mark.parametrize("fam", range(len(FAMILIES)))
def test_init_commit_rounds_consistent(fam):
    """The per-vertex commit rounds: the same colours as init_color, -1 exactly
    for uncoloured vertices, and the vertices still uncommitted at the start
    of round r are the |W_r| of the round statistics."""
    g = FAMILIES[fam]()
    for sel, X, flags, cap in ((oracle.FIRST_FIT, 1, 0, 0), (oracle.RANDOM_X, 4, 0, 0),
                               (oracle.FIRST_FIT, 1, oracle.PRIO_LF, 0), (oracle.RANDOM_X, 3, 0, 2)):
        ref = oracle.init_color(g, sel, X, 7, max_rounds=cap, flags=flags)
        r, cr = oracle.init_color_rounds(g, sel, X, 7, max_rounds=cap, flags=flags)
        assert np.array_equal(r.colors, ref.colors) and np.array_equal(r.w_sizes, ref.w_sizes)
        assert np.array_equal(cr < 0, ref.colors == 0)
        for rnd, size in enumerate(ref.w_sizes):
            assert int(((cr >= rnd) | (cr < 0)).sum()) == size


def test_init_commit_rounds_closed_forms():
    # K_n with First Fit: the vertex committing in round r takes colour r + 1
    g = gen.complete(11)
    r, cr = oracle.init_color_rounds(g, oracle.FIRST_FIT, 1, 3)
    assert np.array_equal(cr, r.colors - 1)
    # round 0 keeps exactly the local maxima of round 0's keys (First Fit)
    g = gen.er(400, 1200, 9)
    _, cr = oracle.init_color_rounds(g, oracle.FIRST_FIT, 1, 17)
    for v in range(g.n):
        kv = oracle.key(17, 0, v)
        assert (cr[v] == 0) == all(oracle.key(17, 0, int(w)) < kv for w in g.neighbors(v))
    # an edgeless graph commits everything in round 0
    _, cr = oracle.init_color_rounds(gen.empty(30), oracle.RANDOM_X, 5, 2)
    assert cr.tolist() == [0] * 30


# ---------------------------------------------------------------- recolouring

def test_recolor_golden_p4():
    rows = []
    with open(os.path.join(GOLD, "recolor_p4.txt")) as f:
        for line in f:
            line = line.split("#")[0].strip()
            if line:
                rows.append(line.split())
    g = gen.path(4)
    perms = {"RV": oracle.PERM_REVERSE, "NI": oracle.PERM_NONINC, "ND": oracle.PERM_NONDEC}
    for name, pi, res in rows:
        r = oracle.recolor(g, np.array([1, 2, 1, 3], np.int32), perms[name], 1, 0)
        assert r.pi.tolist() == [int(x) for x in pi.split(",")]
        assert r.colors.tolist() == [int(x) for x in res.split(",")]


def test_class_orders():
    sizes = np.array([0, 5, 0, 7, 7, 1, 3, 0, 5], np.int64)  # colours 1..8, 2 and 7 empty
    present = [c for c in range(1, 9) if sizes[c] > 0]
    assert oracle.class_order(sizes, oracle.PERM_REVERSE).tolist() == present[::-1]
    assert oracle.class_order(sizes, oracle.PERM_NONINC).tolist() == sorted(present, key=lambda c: (-sizes[c], c))
    assert oracle.class_order(sizes, oracle.PERM_NONDEC).tolist() == sorted(present, key=lambda c: (sizes[c], c))
    r = oracle.class_order(sizes, oracle.PERM_RANDOM, seed=3, pass_=2)
    assert sorted(r.tolist()) == present


def test_random_class_order_uniform():
    # Knuth shuffle: each class lands in each position with probability 1/k
    k, N = 5, 20000
    sizes = np.ones(k + 1, np.int64)
    pos = np.zeros((k, k), np.int64)
    for s in range(N):
        pi = oracle.class_order(sizes, oracle.PERM_RANDOM, seed=s + 1, pass_=s % 7)
        for p, c in enumerate(pi.tolist()):
            pos[c - 1, p] += 1
    exp = N / k
    chi2 = float(((pos - exp) ** 2 / exp).sum())
    assert chi2 < 50.0  # 16 dof, p ~ 3e-5
    # all 120 permutations appear
    seen = {tuple(oracle.class_order(sizes, oracle.PERM_RANDOM, seed=s, pass_=0).tolist()) for s in range(3000)}
    assert len(seen) == 120


def test_recolor_mesh_parity_closed_form():
    N = 6
    g = gen.mesh27(N)
    par = oracle.greedy_seq(g)  # 1 + (x&1) + 2(y&1) + 4(z&1)
    for perm, seed in ((oracle.PERM_REVERSE, 1), (oracle.PERM_NONINC, 1), (oracle.PERM_NONDEC, 1),
                       (oracle.PERM_RANDOM, 3), (oracle.PERM_RANDOM, 4)):
        r = oracle.recolor(g, par, perm, seed, 0)
        rank = {int(c): s for s, c in enumerate(r.pi)}
        # every vertex touches all 7 other parity classes, so rank s -> colour s + 1
        assert r.colors.tolist() == [rank[int(c)] + 1 for c in par]


def test_recolor_never_increases_and_rank_bound():
    for fam in range(len(FAMILIES)):
        g = FAMILIES[fam]()
        if g.n == 0:
            continue
        c = oracle.init_color(g, oracle.RANDOM_X, 5, 2).colors
        prev = oracle.count(c)[0]
        for p in range(10):
            perm = (oracle.PERM_REVERSE, oracle.PERM_NONINC, oracle.PERM_NONDEC, oracle.PERM_RANDOM)[p % 4]
            r = oracle.recolor(g, c, perm, 2, p)
            assert r.status == 0 and oracle.validate(g, r.colors) == (0, 0)
            rank = {int(x): s for s, x in enumerate(r.pi)}
            assert all(r.colors[v] <= rank[int(c[v])] + 1 for v in range(g.n))
            k = oracle.count(r.colors)
            assert k[0] == k[1] <= prev  # contiguous (Grundy) and never more colours
            prev = k[0]
            c = r.colors


def test_recolor_keeps_optimal():
    rng = np.random.default_rng(4)
    for _ in range(10):
        n = int(rng.integers(5, 12))
        g = _random_graph(n, 0.4, rng)
        chi = oracle.chromatic(g)
        # an optimal colouring from the best of many greedy orders
        best = min((oracle.greedy_seq(g, rng.permutation(n)) for _ in range(300)), key=lambda c: int(c.max()))
        if int(best.max()) != chi:
            continue
        for perm in range(4):
            r = oracle.recolor(g, best, perm, 5, 1)
            assert oracle.count(r.colors)[0] == chi


def test_recolor_rejects_bad_input():
    g = gen.path(3)
    assert oracle.recolor(g, np.array([1, 1, 2], np.int32)).status == oracle.ERR_COLORING
    assert oracle.recolor(g, np.array([1, 0, 1], np.int32)).status == oracle.ERR_COLORING


def test_schedules():
    ND, RAND = oracle.PERM_NONDEC, oracle.PERM_RANDOM
    assert [oracle.schedule_perm(1, 0, 5, t) for t in range(1, 11)] == [ND] * 4 + [RAND] + [ND] * 4 + [RAND]
    assert [oracle.schedule_perm(2, 0, 0, t) for t in range(1, 10)] == [ND, RAND, ND, RAND, ND, ND, ND, RAND, ND]
    assert oracle.schedule_perm(0, oracle.PERM_NONINC, 0, 3) == oracle.PERM_NONINC


# ---- asynchronous recoloring aRC (section 3) ----

def _ranks(colors, perm, seed, pass_):
    sizes = np.bincount(np.asarray(colors), minlength=int(np.max(colors)) + 1)
    pi = oracle.class_order(sizes, perm, seed, pass_)
    return {int(c): s for s, c in enumerate(pi)}


def test_arc_closed_forms():
    """aRC gives rank + 1 when every vertex touches every lower class: K_n
    from a one-class-per-vertex coloring (one vertex per round), the 3D mesh
    from its parity coloring, a path from its 2-coloring (section 3; the
    earlier old class wins every conflict)."""
    rng = np.random.default_rng(4)
    cases = [(gen.complete(9), (rng.permutation(9) + 1).astype(np.int32), 9),
             (gen.mesh27(6), None, 8),
             (gen.path(11), np.array([1 + (i & 1) for i in range(11)], np.int32), 2)]
    for g, c0, rounds in cases:
        if c0 is None:
            c0 = oracle.greedy_seq(g)  # 1 + (x&1) + 2(y&1) + 4(z&1)
        for perm, seed in ((oracle.PERM_REVERSE, 1), (oracle.PERM_NONINC, 1), (oracle.PERM_NONDEC, 1),
                           (oracle.PERM_RANDOM, 7)):
            r = oracle.arc_recolor(g, c0, perm, seed, 2)
            rank = _ranks(c0, perm, seed, 2)
            assert r.colors.tolist() == [rank[int(c)] + 1 for c in c0], (g.name, perm)
            assert r.stats["rounds"] == rounds


def test_arc_invariants():
    """Proper, every vertex colored, First Fit's Grundy bound C(v) <= deg(v) + 1."""
    for fam in range(len(FAMILIES)):
        g = FAMILIES[fam]()
        c0 = oracle.init_color(g, oracle.RANDOM_X, 3, 5).colors
        deg = g.degrees
        for perm in range(4):
            r = oracle.arc_recolor(g, c0, perm, 5, 1)
            assert r.status == 0
            assert oracle.validate(g, r.colors) == (0, 0)
            assert (r.colors <= deg + 1).all()


def test_arc_first_class_keeps_color_one():
    """Round 0 gives every vertex color 1 tentatively; a vertex of the first
    class in the order has no earlier neighbor, so it keeps color 1."""
    g = gen.er(300, 1500, 2)
    c0 = oracle.init_color(g, oracle.FIRST_FIT, 1, 3).colors
    for perm in range(4):
        rank = _ranks(c0, perm, 3, 0)
        first = [v for v in range(g.n) if rank[int(c0[v])] == 0]
        r = oracle.arc_recolor(g, c0, perm, 3, 0)
        assert all(r.colors[v] == 1 for v in first)


def test_arc_rejects_bad_input():
    g = gen.path(4)
    assert oracle.arc_recolor(g, [1, 0, 1, 2]).status == oracle.ERR_COLORING
    assert oracle.arc_recolor(g, [1, 1, 2, 1]).status == oracle.ERR_COLORING


# ---- ordering-derived priorities for the initial coloring (Largest First, Natural) ----

def test_priority_orders_closed_forms():
    FF = oracle.FIRST_FIT
    # LF: the star's center has the largest degree, so it keeps color 1 in round 0
    r = oracle.init_color(gen.star(30), FF, 1, 3, flags=oracle.PRIO_LF)
    assert r.colors.tolist() == [1] + [2] * 30 and r.stats["rounds"] == 2
    # Natural: K_n colors one vertex per round in id order
    r = oracle.init_color(gen.complete(10), FF, 1, 3, flags=oracle.PRIO_NATURAL)
    assert r.colors.tolist() == list(range(1, 11)) and r.stats["rounds"] == 10
    # Natural on paths, 2D grids and the 3D mesh: the natural-order greedy closed forms
    assert oracle.init_color(gen.path(13), FF, 1, 5, flags=oracle.PRIO_NATURAL).colors.tolist() == \
        [1 + (i & 1) for i in range(13)]
    nx, ny = 9, 7
    c = oracle.init_color(gen.grid5(nx, ny), FF, 1, 5, flags=oracle.PRIO_NATURAL).colors
    assert c.tolist() == [1 + ((x + y) & 1) for y in range(ny) for x in range(nx)]
    N = 5
    c = oracle.init_color(gen.mesh27(N), FF, 1, 5, flags=oracle.PRIO_NATURAL).colors
    assert c.tolist() == [1 + (x & 1) + 2 * (y & 1) + 4 * (z & 1) for z in range(N) for y in range(N) for x in range(N)]


def test_lf_on_regular_graphs_is_the_fixed_random_order():
    """All degrees equal: Largest First reduces to round 0's random order."""
    for g in (gen.complete(11), gen.cycle(20), gen.crown(6)):
        a = oracle.init_color(g, oracle.FIRST_FIT, 1, 9, flags=oracle.PRIO_LF)
        b = oracle.init_color(g, oracle.FIRST_FIT, 1, 9, flags=oracle.FIXED_PRIORITY)
        assert np.array_equal(a.colors, b.colors) and a.stats["rounds"] == b.stats["rounds"]


def test_priority_orders_invariants():
    for fam in range(len(FAMILIES)):
        g = FAMILIES[fam]()
        deg = g.degrees
        for flags in (oracle.PRIO_LF, oracle.PRIO_NATURAL):
            for sel, X in ((oracle.FIRST_FIT, 1), (oracle.RANDOM_X, 4)):
                r = oracle.init_color(g, sel, X, 6, flags=flags)
                assert oracle.validate(g, r.colors) == (0, 0)
                assert (r.colors <= deg + X).all()
    with pytest.raises(RuntimeError):  # the two orders exclude each other
        oracle.init_color(gen.path(3), oracle.FIRST_FIT, 1, 1, flags=oracle.PRIO_LF | oracle.PRIO_NATURAL)


# ---------------------------------------------------------------- distance-2 coloring

def _dist2_pairs_scipy(g):
    """Pairs u != w at graph distance 1 or 2, from scipy's shortest paths (an
    independent library routine)."""
    from scipy.sparse import csr_matrix
    from scipy.sparse.csgraph import shortest_path

    A = csr_matrix((np.ones(g.nnz), g.col, g.row_ptr), shape=(g.n, g.n))
    D = shortest_path(A, unweighted=True)
    return (D <= 2) & ~np.eye(g.n, dtype=bool)


D2_FAMILIES = [
    lambda: gen.path(11),
    lambda: gen.cycle(9),
    lambda: gen.star(7),
    lambda: gen.complete(6),
    lambda: gen.grid5(6, 5),
    lambda: gen.mesh27(4),
    lambda: gen.crown(5),
    lambda: gen.er(60, 130, seed=4),
    lambda: gen.er(80, 60, seed=5),
    lambda: gen.rmat(6, 4, seed=2),
    lambda: gen.empty(5),
]


@pytest.mark.parametrize("fam", range(len(D2_FAMILIES)))
def test_square_matches_shortest_paths(fam):
    g = D2_FAMILIES[fam]()
    s = oracle.square(g)
    ref = _dist2_pairs_scipy(g)
    got = np.zeros((g.n, g.n), bool)
    for v in range(g.n):
        row = s.col[s.row_ptr[v]:s.row_ptr[v + 1]]
        assert (np.diff(row) > 0).all(), "rows sorted, no duplicates"
        got[v, row] = True
    assert np.array_equal(got, ref)


def test_validate_d2_bruteforce_and_injected():
    rng = np.random.default_rng(8)
    for fam in range(len(D2_FAMILIES)):
        g = D2_FAMILIES[fam]()
        near = _dist2_pairs_scipy(g)
        c = rng.integers(1, 6, size=g.n).astype(np.int32)
        c[rng.random(g.n) < 0.1] = 0
        want = sum(1 for u in range(g.n) for w in range(u + 1, g.n) if near[u, w] and c[u] == c[w] > 0)
        assert oracle.validate_d2(g, c) == (want, int((c <= 0).sum()))
    # a proper distance-2 coloring, then one injected conflict at distance exactly 2 (path 0-1-2)
    g = gen.path(9)
    c = np.array([1 + i % 3 for i in range(9)], np.int32)
    assert oracle.validate_d2(g, c) == (0, 0)
    assert oracle.validate(g, c) == (0, 0)
    c[0] = c[2]  # vertices 0 and 2 are two edges apart; vertex 1 keeps them distance-1 proper
    assert oracle.validate_d2(g, c) == (1, 0) and oracle.validate(g, c) == (0, 0)


def _structurally_orthogonal(g, c):
    """Column compression view (sparse Jacobian / Hessian of the pattern A + I):
    within every row i, the columns {i} and N(i) carry pairwise different colors."""
    for i in range(g.n):
        cols = np.concatenate(([i], g.neighbors(i)))
        if len(set(c[cols].tolist())) != len(cols):
            return False
    return True


@pytest.mark.parametrize("fam", range(len(D2_FAMILIES)))
def test_init_d2_invariants(fam):
    g = D2_FAMILIES[fam]()
    s = oracle.square(g)
    d2deg = np.diff(s.row_ptr.astype(np.int64))
    for flags in (0, oracle.FIXED_PRIORITY, oracle.PRIO_NATURAL):
        for sel, X in ((oracle.FIRST_FIT, 1), (oracle.RANDOM_X, 3)):
            r = oracle.init_color_d2(g, sel, X, 7, flags=flags)
            c = r.colors
            assert oracle.validate_d2(g, c) == (0, 0)
            assert _structurally_orthogonal(g, c)
            # Grundy-type bound over the distance-2 neighborhood
            assert (c <= d2deg + X).all()
            # every closed neighborhood is a clique of G^2
            if g.n:
                assert r.stats["num_colors"] >= g.max_deg + 1
        # Random-X with X = 1 is First Fit, rounds included
        a = oracle.init_color_d2(g, oracle.RANDOM_X, 1, 7, flags=flags)
        b = oracle.init_color_d2(g, oracle.FIRST_FIT, 1, 7, flags=flags)
        assert np.array_equal(a.colors, b.colors) and a.rounds == b.rounds


def test_init_d2_closed_forms():
    FF = oracle.FIRST_FIT
    # star: its square is K_{m+1}; natural order colors one vertex per round
    r = oracle.init_color_d2(gen.star(9), FF, 1, 2, flags=oracle.PRIO_NATURAL)
    assert r.colors.tolist() == list(range(1, 11)) and r.rounds == 10
    # star with random priorities: m + 1 rounds, the largest remaining key takes color r + 1 in round r
    m, seed = 9, 4
    r = oracle.init_color_d2(gen.star(m), FF, 1, seed)
    assert r.rounds == m + 1 and sorted(r.colors.tolist()) == list(range(1, m + 2))
    left = set(range(m + 1))
    for rnd in range(m + 1):
        top = max(left, key=lambda v: oracle.key(seed, rnd, v))
        assert r.colors[top] == rnd + 1
        left.remove(top)
    # path, natural order: colors repeat with period 3
    assert oracle.init_color_d2(gen.path(14), FF, 1, 3, flags=oracle.PRIO_NATURAL).colors.tolist() == \
        [1 + i % 3 for i in range(14)]
    # 27-point mesh: distance 2 is Chebyshev distance <= 2; natural order gives
    # the product of the path's period-3 pattern over the three axes (27 colors,
    # the size of a 3x3x3 block, which is a clique of the square)
    N = 7
    c = oracle.init_color_d2(gen.mesh27(N), FF, 1, 3, flags=oracle.PRIO_NATURAL).colors
    assert c.tolist() == [1 + x % 3 + 3 * (y % 3) + 9 * (z % 3) for z in range(N) for y in range(N) for x in range(N)]
    # edgeless: distance 2 changes nothing
    r = oracle.init_color_d2(gen.empty(6), FF, 1, 1)
    assert r.colors.tolist() == [1] * 6 and r.rounds == 1
    with pytest.raises(ValueError):
        oracle.init_color_d2(gen.path(3), FF, 1, 1, flags=oracle.PRIO_LF)


def test_init_d2_vs_chromatic_exhaustive_small():
    """Never below the distance-2 chromatic number (brute force on tiny graphs)."""
    rng = np.random.default_rng(12)
    for _ in range(25):
        n = int(rng.integers(3, 9))
        pairs = [(u, w) for u in range(n) for w in range(u + 1, n) if rng.random() < 0.3]
        g = gen.from_pairs(n, pairs)
        near = _dist2_pairs_scipy(g)
        chi = None
        for k in range(1, n + 1):  # exhaustive search over all k^n assignments
            for c in itertools.product(range(k), repeat=n):
                if all(c[u] != c[w] for u in range(n) for w in range(u + 1, n) if near[u, w]):
                    chi = k
                    break
            if chi:
                break
        r = oracle.init_color_d2(g, oracle.FIRST_FIT, 1, int(rng.integers(1, 99)))
        assert r.stats["num_colors"] >= chi


def test_recolor_d2_closed_form_and_invariants():
    N = 6
    g = gen.mesh27(N)
    s = oracle.square(g)
    c0 = np.array([1 + x % 3 + 3 * (y % 3) + 9 * (z % 3) for z in range(N) for y in range(N) for x in range(N)],
                  np.int32)
    assert oracle.validate_d2(g, c0, sq=s) == (0, 0)
    for perm, seed in ((oracle.PERM_REVERSE, 1), (oracle.PERM_NONINC, 1), (oracle.PERM_RANDOM, 5)):
        r = oracle.recolor_d2(g, c0, perm, seed, 0, sq=s)
        rank = {int(c): i for i, c in enumerate(r.pi)}
        # every distance-2 neighborhood holds a 3x3x3 block, i.e. all 26 other classes
        assert r.colors.tolist() == [rank[int(c)] + 1 for c in c0]
    # general graphs: proper, never more colors, rank bound
    for fam in range(len(D2_FAMILIES)):
        g = D2_FAMILIES[fam]()
        c = oracle.init_color_d2(g, oracle.RANDOM_X, 4, 3).colors
        k0 = oracle.count(c)[0]
        for p, perm in enumerate((oracle.PERM_REVERSE, oracle.PERM_RANDOM, oracle.PERM_NONINC)):
            r = oracle.recolor_d2(g, c, perm, 3, p)
            assert oracle.validate_d2(g, r.colors) == (0, 0)
            assert r.stats["num_colors"] <= k0
            rank = {int(cc): i for i, cc in enumerate(r.pi)}
            assert all(r.colors[v] <= rank[int(c[v])] + 1 for v in range(g.n))
            c, k0 = r.colors, r.stats["num_colors"]
    # a distance-1 coloring that is not a distance-2 coloring is rejected
    g = gen.path(5)
    assert oracle.recolor_d2(g, np.array([1, 2, 1, 2, 1], np.int32)).status == oracle.ERR_COLORING


def test_checkpoint_resume_identity_oracle(tmp_path):
    """Ten recoloring passes equal five passes, a checkpoint of the colors to a
    text file, a restore from it and five more passes (pass indices 5..9): a
    pass depends only on its input coloring, the seed and the pass index."""
    g = gen.rmat(11, 16, seed=3)
    c0 = oracle.init_color(g, oracle.RANDOM_X, 4, 3).colors
    whole = c0
    for p in range(10):
        whole = oracle.recolor(g, whole, oracle.PERM_RANDOM, 3, p).colors
    half = c0
    for p in range(5):
        half = oracle.recolor(g, half, oracle.PERM_RANDOM, 3, p).colors
    f = tmp_path / "colors.txt"
    np.savetxt(f, half, fmt="%d")
    back = np.loadtxt(f, dtype=np.int32)
    for p in range(5, 10):
        back = oracle.recolor(g, back, oracle.PERM_RANDOM, 3, p).colors
    assert np.array_equal(back, whole)
    assert oracle.validate(g, whole) == (0, 0)
