"""Request server on the GPU: every request's colors are the same in a mix of
concurrent requests as alone (a one-slot server and the plain single-graph
calls with the request's seed), bit for bit; admission keeps the arena
within its budget; requests overlap on the device."""
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


@pytest.fixture(scope="module")
def pool():
    return gen.serve_pool(12, seed=3, small=True)


def plain_colors(gc, g, seed, X=4, passes=3, perm=0):
    d = torch.device("cuda:0")
    rp = torch.from_numpy(g.row_ptr).to(d)
    col = torch.from_numpy(g.col).to(d)
    c, _ = gc.init_color(rp, col, gc.RANDOM_X, X, seed, stats=False)
    for p in range(passes):
        c, _ = gc.recolor(rp, col, c, perm, seed, p, out=c, stats=False)
    return c.cpu().numpy()


def run_all(srv, pool, reqs):
    for tag, (gi, seed) in enumerate(reqs):
        g = pool[gi]
        srv.submit(g.row_ptr, g.col, seed=seed, tag=tag)
    out = {}
    while len(out) < len(reqs):
        for d in srv.poll(timeout_ms=20000):
            out[d["tag"]] = d
    return out


def test_mix_equals_alone(gc, pool):
    rng = np.random.default_rng(5)
    reqs = [(int(rng.integers(0, len(pool))), int(rng.integers(1, 2**62))) for _ in range(48)]
    biggest = max(gc.request_footprint(g.n, g.nnz) for g in pool)
    budget = int(2.5 * biggest)  # admission by footprint binds: at most two of the largest at once
    max_n = max(g.n for g in pool)
    max_nnz = max(g.nnz for g in pool)
    mix = gc.Server(slots=6, hbm_budget=budget, max_n=max_n, max_nnz=max_nnz)
    got = run_all(mix, pool, reqs)
    st = mix.stats()
    mix.close()
    assert st["completed"] == len(reqs) and st["waiting"] == 0 and st["running"] == 0
    assert st["arena_peak"] <= budget
    assert st["peak_running"] >= 2, "no two requests overlapped"
    alone = gc.Server(slots=1, hbm_budget=budget, max_n=max_n, max_nnz=max_nnz)
    ref = run_all(alone, pool, reqs)
    alone.close()
    for tag, (gi, seed) in enumerate(reqs):
        d, r = got[tag], ref[tag]
        assert d["status"] == 0 and r["status"] == 0
        assert np.array_equal(d["colors"], r["colors"]), f"request {tag}: mix != alone"
        assert (d["rounds"], d["colors_init"], d["colors_final"]) == (r["rounds"], r["colors_init"], r["colors_final"])
        assert d["t_submit"] <= d["t_admit"] <= d["t_done"]
    for tag in range(0, len(reqs), 6):
        gi, seed = reqs[tag]
        assert np.array_equal(got[tag]["colors"], plain_colors(gc, pool[gi], seed)), f"request {tag}: != plain calls"


def test_served_colors_match_oracle(gc, pool):
    srv = gc.Server(slots=3, hbm_budget=1 << 28, max_n=max(g.n for g in pool), max_nnz=max(g.nnz for g in pool))
    reqs = [(i, 1000 + i) for i in range(len(pool))]
    got = run_all(srv, pool, reqs)
    srv.close()
    for tag, (gi, seed) in enumerate(reqs):
        g = pool[gi]
        c = oracle.init_color(g, oracle.RANDOM_X, 4, seed).colors
        for p in range(3):
            c = oracle.recolor(g, c, oracle.PERM_REVERSE, seed, p).colors
        assert np.array_equal(got[tag]["colors"], c), g.name


def test_submit_rejects_out_of_range(gc, pool):
    g = pool[0]
    srv = gc.Server(slots=1, hbm_budget=1 << 20, max_n=g.n, max_nnz=g.nnz)
    big = gen.grid5(g.n + 5, 2)
    with pytest.raises(gc.GCError):
        srv.submit(big.row_ptr, big.col)
    with pytest.raises(gc.GCError):
        srv.submit(g.row_ptr, g.col, X=0)
    srv.close()
