"""ctypes binding of the CPU oracle (``gc_oracle.c``).

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, by ``__graft_entry__.smoke()``
and by the CPU-baseline leg of ``bench.py``, never by the product package.
The oracle is a plain single-threaded C transcription of the method; it shares
no code with the HIP path.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))

# Builds of the same source: "plain" (gcc -O2) for the tests; "fast" (-O3,
# AVX2-level x86-64-v3 rather than -march=native, because the library is
# built on one host and may run on another) for the timed CPU baseline;
# "san" (AddressSanitizer + UndefinedBehaviorSanitizer, any report fatal) for
# a sanitizer run of the CPU suite, which needs the sanitizer runtimes
# preloaded into the Python process (see tests/test_oracle_sanitized.py).
VARIANTS = {
    "plain": ("liboracle.so", ["-O2"]),
    "fast": ("liboracle_o3.so", ["-O3", "-march=x86-64-v3"]),
    "san": ("liboracle_san.so", ["-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
                                 "-fno-sanitize-recover=undefined"]),
}
_variant = os.environ.get("ORACLE_VARIANT", "plain")
_lib = None


def use_variant(name: str) -> None:
    """Select the build that _load() opens (before the first oracle call)."""
    global _variant
    if name not in VARIANTS:
        raise ValueError(f"unknown oracle build {name!r}")
    if _lib is not None and name != _variant:
        raise RuntimeError(f"the {_variant!r} oracle build is already loaded")
    _variant = name


def variant() -> str:
    return _variant


def lib_path(name: str | None = None) -> str:
    return os.path.join(_HERE, VARIANTS[name or _variant][0])

OK, ERR_ARG, ERR_GRAPH, ERR_COLORING, ERR_OOM, ERR_NOT_CONVERGED = 0, 1, 2, 3, 4, 6
FIRST_FIT, RANDOM_X = 0, 1
PERM_REVERSE, PERM_NONINC, PERM_NONDEC, PERM_RANDOM = 0, 1, 2, 3
FIXED_PRIORITY = 1
PRIO_LF = 2
PRIO_NATURAL = 4


class Stats(ctypes.Structure):
    _fields_ = [("rounds", ctypes.c_int32), ("num_colors", ctypes.c_int32), ("max_color", ctypes.c_int32),
                ("_pad", ctypes.c_int32), ("losers_total", ctypes.c_int64)]

    def as_dict(self):
        return {"rounds": self.rounds, "num_colors": self.num_colors, "max_color": self.max_color,
                "losers_total": self.losers_total}


def build(verbose: bool = False, variants=("plain", "fast")) -> str:
    """Compile the oracle (plain C, single-threaded) into the requested builds;
    returns the path of the first."""
    src = os.path.join(_HERE, "gc_oracle.c")
    paths = []
    for name in variants:
        out = lib_path(name)
        tmp = out + ".tmp"
        cmd = ["gcc", *VARIANTS[name][1], "-fPIC", "-shared", "-std=c11", "-Wall", src, "-o", tmp]
        if verbose:
            print(" ".join(cmd))
        subprocess.run(cmd, check=True)
        os.replace(tmp, out)
        paths.append(out)
    return paths[0]


def _load():
    global _lib
    if _lib is not None:
        return _lib
    path = lib_path()
    if not os.path.exists(path):
        build(variants=(_variant,))
    lib = ctypes.CDLL(path)
    i32p = ctypes.POINTER(ctypes.c_int32)
    i64p = ctypes.POINTER(ctypes.c_int64)
    u64, u32, i32 = ctypes.c_uint64, ctypes.c_uint32, ctypes.c_int32
    sig = {
        "orc_mix64": (u64, [u64]),
        "orc_fmix32": (u32, [u32]),
        "orc_stream": (u32, [u64, u32, u32]),
        "orc_prio": (u32, [u64, u32, u32]),
        "orc_key": (u64, [u64, u32, u32]),
        "orc_pick": (u32, [u64, u32, u32, u32]),
        "orc_bounded": (u32, [u64, u32, u32, u32]),
        "orc_graph_seed": (u64, [u64, u32]),
        "orc_greedy_seq": (ctypes.c_int, [i32, i32p, i32p, i32p, i32p]),
        "orc_count": (ctypes.c_int, [i32, i32p, i32p, i32p]),
        "orc_validate": (ctypes.c_int, [i32, i32p, i32p, i32p, i64p, i64p]),
        "orc_check_csr": (ctypes.c_int, [i32, i32p, i32p]),
        "orc_init_color": (ctypes.c_int, [i32, i32p, i32p, i32, i32, u64, i32, u32, i32p,
                                          ctypes.POINTER(Stats), i64p, i64p, i32]),
        "orc_init_color_rounds": (ctypes.c_int, [i32, i32p, i32p, i32, i32, u64, i32, u32, i32p,
                                                 ctypes.POINTER(Stats), i64p, i64p, i32, i32p]),
        "orc_class_order": (i32, [i32, i64p, i32, u64, i32, i32p]),
        "orc_recolor": (ctypes.c_int, [i32, i32p, i32p, i32, u64, i32, i32p, i32p, i32p, i32p,
                                       ctypes.POINTER(Stats)]),
        "orc_arc_recolor": (ctypes.c_int, [i32, i32p, i32p, i32, u64, i32, i32p, i32p, i32p, ctypes.POINTER(Stats)]),
        "orc_schedule_perm": (i32, [i32, i32, i32, i32]),
        "orc_chromatic": (i32, [i32, i32p, i32p]),
        "orc_square_count": (ctypes.c_int64, [i32, i32p, i32p, i32p]),
        "orc_square_fill": (ctypes.c_int, [i32, i32p, i32p, i32p]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib


def _p32(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))


def _p64(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))


def _csr(g):
    rp = np.ascontiguousarray(g.row_ptr, dtype=np.int32)
    col = np.ascontiguousarray(g.col, dtype=np.int32)
    if col.size == 0:
        col = np.zeros(1, np.int32)
    return rp, col


# ---- hash ----
def mix64(z):
    return int(_load().orc_mix64(z & (2**64 - 1)))


def fmix32(h):
    return int(_load().orc_fmix32(h & 0xFFFFFFFF))


def stream(seed, tag, r):
    return int(_load().orc_stream(seed, tag, r))


def prio(seed, r, v):
    return int(_load().orc_prio(seed, r, v))


def key(seed, r, v):
    return int(_load().orc_key(seed, r, v))


def pick(seed, r, v, X):
    return int(_load().orc_pick(seed, r, v, X))


def bounded(seed, p, i, m):
    return int(_load().orc_bounded(seed, p, i, m))


def graph_seed(base, g):
    return int(_load().orc_graph_seed(base, g))


# ---- algorithms ----
def greedy_seq(g, order=None) -> np.ndarray:
    """Algorithm 1 (sequential greedy First Fit) over `order` (natural when None)."""
    rp, col = _csr(g)
    c = np.zeros(max(g.n, 1), np.int32)
    o = None if order is None else np.ascontiguousarray(order, dtype=np.int32)
    rc = _load().orc_greedy_seq(g.n, _p32(rp), _p32(col), None if o is None else _p32(o), _p32(c))
    if rc:
        raise RuntimeError(f"orc_greedy_seq: {rc}")
    return c[:g.n]


def count(colors) -> tuple[int, int]:
    c = np.ascontiguousarray(colors, dtype=np.int32)
    num, mx = ctypes.c_int32(), ctypes.c_int32()
    rc = _load().orc_count(c.size, _p32(c) if c.size else _p32(np.zeros(1, np.int32)), ctypes.byref(num),
                           ctypes.byref(mx))
    if rc:
        raise RuntimeError(f"orc_count: {rc}")
    return num.value, mx.value


def validate(g, colors) -> tuple[int, int]:
    rp, col = _csr(g)
    c = np.ascontiguousarray(colors, dtype=np.int32)
    if c.size == 0:
        c = np.zeros(1, np.int32)
    cf, un = ctypes.c_int64(), ctypes.c_int64()
    _load().orc_validate(g.n, _p32(rp), _p32(col), _p32(c), ctypes.byref(cf), ctypes.byref(un))
    return cf.value, un.value


def check_csr(g) -> int:
    rp, col = _csr(g)
    return int(_load().orc_check_csr(g.n, _p32(rp), _p32(col)))


class InitResult:
    def __init__(self, status, colors, stats, w_sizes, w_degsum):
        self.status = status
        self.colors = colors
        self.stats = stats
        self.w_sizes = w_sizes
        self.w_degsum = w_degsum

    @property
    def rounds(self):
        return self.stats["rounds"]


def init_color(g, select=FIRST_FIT, X=1, seed=1, max_rounds=0, flags=0, w_cap=None) -> InitResult:
    """Speculative round-synchronous initial coloring (section 2.2 framework)."""
    rp, col = _csr(g)
    c = np.zeros(max(g.n, 1), np.int32)
    cap = (g.n + 2) if w_cap is None else w_cap
    ws = np.zeros(max(cap, 1), np.int64)
    wd = np.zeros(max(cap, 1), np.int64)
    st = Stats()
    rc = _load().orc_init_color(g.n, _p32(rp), _p32(col), select, X, seed, max_rounds, flags, _p32(c),
                                ctypes.byref(st), _p64(ws), _p64(wd), cap)
    if rc not in (OK, ERR_NOT_CONVERGED):
        raise RuntimeError(f"orc_init_color: {rc}")
    r = min(st.rounds, cap)
    return InitResult(rc, c[:g.n], st.as_dict(), ws[:r].copy(), wd[:r].copy())


def init_color_rounds(g, select=FIRST_FIT, X=1, seed=1, max_rounds=0, flags=0):
    """init_color, plus the round in which each vertex kept its colour (-1:
    still uncoloured when max_rounds stopped it).  Returns (InitResult, rounds)."""
    rp, col = _csr(g)
    c = np.zeros(max(g.n, 1), np.int32)
    cr = np.zeros(max(g.n, 1), np.int32)
    cap = g.n + 2
    ws = np.zeros(max(cap, 1), np.int64)
    wd = np.zeros(max(cap, 1), np.int64)
    st = Stats()
    rc = _load().orc_init_color_rounds(g.n, _p32(rp), _p32(col), select, X, seed, max_rounds, flags, _p32(c),
                                       ctypes.byref(st), _p64(ws), _p64(wd), cap, _p32(cr))
    if rc not in (OK, ERR_NOT_CONVERGED):
        raise RuntimeError(f"orc_init_color_rounds: {rc}")
    r = min(st.rounds, cap)
    return InitResult(rc, c[:g.n], st.as_dict(), ws[:r].copy(), wd[:r].copy()), cr[:g.n].copy()


class RecolorResult:
    def __init__(self, status, colors, stats, pi):
        self.status = status
        self.colors = colors
        self.stats = stats
        self.pi = pi


def class_order(sizes_by_color, perm, seed=1, pass_=0) -> np.ndarray:
    """Class permutation pi for sizes_by_color[c] (index 0 ignored)."""
    s = np.ascontiguousarray(sizes_by_color, dtype=np.int64)
    maxc = s.size - 1
    pi = np.zeros(max(maxc, 1), np.int32)
    k = _load().orc_class_order(maxc, _p64(s), perm, seed, pass_, _p32(pi))
    return pi[:k].copy()


def recolor(g, colors, perm=PERM_REVERSE, seed=1, pass_=0) -> RecolorResult:
    """One Culberson recoloring pass over the color classes in order pi."""
    rp, col = _csr(g)
    c_old = np.ascontiguousarray(colors, dtype=np.int32)
    if c_old.size == 0:
        c_old = np.zeros(1, np.int32)
    c_new = np.zeros(max(g.n, 1), np.int32)
    maxc = int(c_old[:g.n].max()) if g.n > 0 else 0
    pi = np.zeros(max(maxc, 1), np.int32)
    k = ctypes.c_int32()
    st = Stats()
    rc = _load().orc_recolor(g.n, _p32(rp), _p32(col), perm, seed, pass_, _p32(c_old), _p32(c_new), _p32(pi),
                             ctypes.byref(k), ctypes.byref(st))
    if rc:
        return RecolorResult(rc, None, None, None)
    return RecolorResult(rc, c_new[:g.n], st.as_dict(), pi[:k.value].copy())


def arc_recolor(g, colors, perm=PERM_REVERSE, seed=1, pass_=0) -> RecolorResult:
    """Asynchronous recoloring aRC: speculative First Fit rounds in which the
    old class order decides conflicts (section 3)."""
    rp, col = _csr(g)
    c_old = np.ascontiguousarray(colors, dtype=np.int32)
    if c_old.size == 0:
        c_old = np.zeros(1, np.int32)
    c_new = np.zeros(max(g.n, 1), np.int32)
    rounds = ctypes.c_int32()
    st = Stats()
    rc = _load().orc_arc_recolor(g.n, _p32(rp), _p32(col), perm, seed, pass_, _p32(c_old), _p32(c_new),
                                 ctypes.byref(rounds), ctypes.byref(st))
    if rc:
        return RecolorResult(rc, None, None, None)
    return RecolorResult(rc, c_new[:g.n], st.as_dict(), None)


def schedule_perm(kind, base, x, t) -> int:
    return int(_load().orc_schedule_perm(kind, base, x, t))


def chromatic(g) -> int:
    rp, col = _csr(g)
    return int(_load().orc_chromatic(g.n, _p32(rp), _p32(col)))


# ---- distance-2 coloring ----
class Graph:
    """A CSR graph produced by the oracle (same fields as the generators' graphs)."""

    def __init__(self, n, row_ptr, col, name=""):
        self.n, self.row_ptr, self.col, self.name = n, row_ptr, col, name

    @property
    def nnz(self):
        return int(self.col.shape[0])


def square(g) -> Graph:
    """The square graph G^2: u != w adjacent iff G joins them by a path of one
    or two edges (section 1's distance-k condition with k = 2).  Rows sorted,
    no duplicates."""
    rp, col = _csr(g)
    rp2 = np.zeros(g.n + 1, np.int32)
    nnz2 = int(_load().orc_square_count(g.n, _p32(rp), _p32(col), _p32(rp2)))
    if nnz2 < 0:
        raise RuntimeError("orc_square_count: square graph too large")
    col2 = np.zeros(max(nnz2, 1), np.int32)
    rc = _load().orc_square_fill(g.n, _p32(rp), _p32(col), _p32(col2))
    if rc:
        raise RuntimeError(f"orc_square_fill: {rc}")
    return Graph(g.n, rp2, col2[:nnz2], getattr(g, "name", "") + "^2")


# A distance-2 coloring of G is a distance-1 coloring of G^2 (section 1), so
# the distance-2 routines are the distance-1 ones applied to the square.
# Largest First would need degrees in G^2 and is not offered.

def init_color_d2(g, select=FIRST_FIT, X=1, seed=1, max_rounds=0, flags=0, w_cap=None, sq=None) -> InitResult:
    """Speculative initial distance-2 coloring (w_degsum counts degrees in G^2)."""
    if flags & PRIO_LF:
        raise ValueError("Largest First is not defined for distance-2 coloring here")
    return init_color(square(g) if sq is None else sq, select, X, seed, max_rounds, flags, w_cap)


def recolor_d2(g, colors, perm=PERM_REVERSE, seed=1, pass_=0, sq=None) -> RecolorResult:
    """One recoloring pass of a distance-2 coloring (classes of a distance-2
    coloring are independent in G^2)."""
    return recolor(square(g) if sq is None else sq, colors, perm, seed, pass_)


def validate_d2(g, colors, sq=None) -> tuple[int, int]:
    """(pairs u < w within two edges of each other with equal positive colors,
    vertices with color <= 0).  Section 1's distance-k condition is stated per
    pair of vertices, so the check counts pairs, as the distance-1 check counts
    edges: it is the distance-1 check on the square graph.  A coloring is a
    distance-2 coloring iff both are 0."""
    return validate(square(g) if sq is None else sq, colors)


def run_pipeline(g, select, X, seed, perm_schedule, max_rounds=0):
    """Initial coloring followed by one recoloring pass per entry of perm_schedule.

    Returns (init_result, [recolor_result, ...]); pass p uses class order
    perm_schedule[p] and pass index p."""
    ini = init_color(g, select, X, seed, max_rounds)
    out = []
    c = ini.colors
    for p, perm in enumerate(perm_schedule):
        r = recolor(g, c, perm, seed, p)
        if r.status:
            raise RuntimeError(f"orc_recolor: {r.status}")
        out.append(r)
        c = r.colors
    return ini, out
