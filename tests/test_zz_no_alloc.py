"""The allocation-free entry point gc_count_colors_static against
gc_count_colors, through the C ABI, on consecutive calls that share its
static device array: a large input, then a smaller one whose colors would
pick up any bit the first call left, a color above the static limit
(GC_ERR_ARG), and a correct call after that."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def gc():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1407_6745_amd as m

    m.lib()
    return m


def _both(gc, c, ctx):
    return gc.count_colors_static(c), gc.count_colors(c, ctx=ctx)


def test_count_colors_static_matches_context_version(gc):
    rng = np.random.default_rng(11)
    ctx = gc.Context(1 << 21)
    # 1: two million vertices, colors with gaps up to 80,000 (LDS and global bitmap words)
    a = rng.integers(1, 80001, size=2_000_000).astype(np.int32)
    a[rng.random(a.size) < 0.01] = 0
    ca = torch.from_numpy(a).cuda()
    got, ref = _both(gc, ca, ctx)
    assert got == ref == (len(np.unique(a[a > 0])), int(a.max()))
    # 2: smaller input, three colors spread over the same bitmap words
    b = np.array([1, 2, 79_999] * 1667, np.int32)[:5000]
    got, ref = _both(gc, torch.from_numpy(b).cuda(), ctx)
    assert got == ref == (3, 79_999)
    # 3: a color above the static bitmap is refused; the context version counts it
    c = np.array([5, gc.STATIC_MAX_COLOR + 3, 7], np.int32)
    with pytest.raises(gc.GCError) as e:
        gc.count_colors_static(torch.from_numpy(c).cuda())
    assert e.value.status == gc.ERR_ARG
    assert gc.count_colors(torch.from_numpy(c).cuda(), ctx=ctx) == (3, gc.STATIC_MAX_COLOR + 3)
    # 4: still exact afterwards, including the largest color it takes, and the empty input
    d = np.array([gc.STATIC_MAX_COLOR, 1, 1, 64, 65_537, 0, -3], np.int32)
    got, ref = _both(gc, torch.from_numpy(d).cuda(), ctx)
    assert got == ref == (4, gc.STATIC_MAX_COLOR)
    e0 = torch.zeros(0, dtype=torch.int32, device="cuda")
    assert gc.count_colors_static(e0) == gc.count_colors(e0, ctx=ctx) == (0, 0)
    ctx.close()
