"""Serving with compute-unit partitions: every slot's stream runs on its own
compute units, so the recoloring passes of different requests run on the
device at the same time (shown by the device timestamps of each request's
passes), and every result is still the plain single-graph result."""
import numpy as np
import pytest

import gen

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def gc():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1407_6745_amd as m

    m.lib()
    return m


def _plain(gc, g, seed, passes, perm):
    d = torch.device("cuda:0")
    rp = torch.from_numpy(g.row_ptr).to(d)
    col = torch.from_numpy(g.col).to(d)
    c, _ = gc.init_color(rp, col, gc.RANDOM_X, 4, seed, stats=False)
    for p in range(passes):
        c, _ = gc.recolor(rp, col, c, perm, seed, p, out=c, stats=False)
    return c.cpu().numpy()


@pytest.mark.parametrize("slots", [4, 8])
def test_partitioned_passes_overlap(gc, slots):
    graphs = [gen.mesh27(40), gen.rmat(15, 16, seed=3), gen.er(200000, 1600000, 5), gen.grid5(700, 700)]
    srv = gc.Server(slots=slots, hbm_budget=1 << 30, max_n=max(g.n for g in graphs),
                    max_nnz=max(g.nnz for g in graphs), cu_partition=1)
    st = srv.stats()
    assert st["cu_partition"] == 1 and st["slot_cus"] * slots <= 256 and st["slot_cus"] >= 8
    passes, perm = 6, gc.PERM_RANDOM
    reqs = [(k % len(graphs), 1000 + k) for k in range(3 * slots)]
    for tag, (gi, seed) in enumerate(reqs):
        srv.submit(graphs[gi].row_ptr, graphs[gi].col, gc.RANDOM_X, 4, perm, passes, seed, tag=tag)
    res = []
    while len(res) < len(reqs):
        res += srv.poll(timeout_ms=60000)
    srv.close()
    assert all(d["status"] == 0 for d in res)
    # passes of requests on different slots overlapping on the device
    spans = sorted((d["pass_start_ms"], d["pass_end_ms"], d["slot"]) for d in res)
    overlaps = sum(1 for i, a in enumerate(spans) for b in spans[i + 1:] if b[0] < a[1] and b[2] != a[2])
    print(f"[serve] {slots} slots x {st['slot_cus']} CUs: {overlaps} overlapping pass pairs", flush=True)
    assert overlaps >= slots // 2
    by_tag = {d["tag"]: d for d in res}
    for tag, (gi, seed) in enumerate(reqs):
        assert np.array_equal(by_tag[tag]["colors"], _plain(gc, graphs[gi], seed, passes, perm)), tag


def test_shared_device_mode_still_works(gc):
    g = gen.rmat(13, 16, seed=2)
    srv = gc.Server(slots=3, hbm_budget=1 << 28, max_n=g.n, max_nnz=g.nnz, cu_partition=0)
    assert srv.stats()["cu_partition"] == 0
    for k in range(6):
        srv.submit(g.row_ptr, g.col, gc.RANDOM_X, 4, gc.PERM_REVERSE, 3, 50 + k, tag=k)
    res = []
    while len(res) < 6:
        res += srv.poll(timeout_ms=60000)
    srv.close()
    for d in res:
        assert d["status"] == 0
        assert np.array_equal(d["colors"], _plain(gc, g, 50 + d["tag"], 3, gc.PERM_REVERSE))
