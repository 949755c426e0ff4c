"""Seeded synthetic graph inputs (host side).

This module builds the graphs that both the oracle and the HIP path are run
on.  It holds none of the coloring method's arithmetic: only graph
construction (C, ``gcgen.c``) and a few tiny textbook families written out in
Python for the oracle's closed-form tests.

Every graph is returned as a :class:`CSR` with int32 ``row_ptr`` (n+1) and
``col`` (nnz) numpy arrays: symmetric, no self-loops, no duplicates, rows
sorted ascending.
"""
from __future__ import annotations

import ctypes
import math
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libgcgen.so")
_lib = None


class _GenGraph(ctypes.Structure):
    _fields_ = [
        ("n", ctypes.c_int64),
        ("nnz", ctypes.c_int64),
        ("row_ptr", ctypes.POINTER(ctypes.c_int32)),
        ("col", ctypes.POINTER(ctypes.c_int32)),
        ("max_deg", ctypes.c_int32),
        ("status", ctypes.c_int32),
    ]


def build(verbose: bool = False) -> str:
    """Compile gcgen.c into libgcgen.so next to it (gcc, OpenMP)."""
    import subprocess

    src = os.path.join(_HERE, "gcgen.c")
    tmp = _LIB_PATH + ".tmp"
    cmd = ["gcc", "-O3", "-fopenmp", "-fPIC", "-shared", "-std=c11", "-D_DEFAULT_SOURCE",
           "-Wall", "-Wno-unused-function", src, "-o", tmp, "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        build()
    lib = ctypes.CDLL(_LIB_PATH)
    P = ctypes.POINTER(_GenGraph)
    i32p = ctypes.POINTER(ctypes.c_int32)
    i64p = ctypes.POINTER(ctypes.c_int64)
    f64p = ctypes.POINTER(ctypes.c_double)
    lib.gen_free.argtypes = [P]
    lib.gen_free.restype = None
    lib.gen_mesh27.argtypes = [ctypes.c_int32]
    lib.gen_mesh27.restype = P
    lib.gen_grid5.argtypes = [ctypes.c_int32, ctypes.c_int32]
    lib.gen_grid5.restype = P
    lib.gen_er.argtypes = [ctypes.c_int64, ctypes.c_int64, ctypes.c_uint64]
    lib.gen_er.restype = P
    lib.gen_rmat.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.c_double, ctypes.c_double,
                             ctypes.c_double, ctypes.c_uint64]
    lib.gen_rmat.restype = P
    lib.gen_rgg.argtypes = [ctypes.c_int64, ctypes.c_double, ctypes.c_uint64]
    lib.gen_rgg.restype = P
    lib.gen_from_pairs.argtypes = [ctypes.c_int64, ctypes.c_int64, i32p, i32p]
    lib.gen_from_pairs.restype = P
    lib.gen_rgg_batch_params.argtypes = [ctypes.c_int32, ctypes.c_uint64, ctypes.c_int32, ctypes.c_int32,
                                         ctypes.c_double, ctypes.c_double, i64p, f64p]
    lib.gen_rgg_batch_params.restype = None
    lib.gen_rgg_batch_fill.argtypes = [ctypes.c_int32, ctypes.c_uint64, i64p, f64p, i64p, i64p, i64p,
                                       i32p, i32p]
    lib.gen_rgg_batch_fill.restype = ctypes.c_int
    lib.gen_rgg_batch_one.argtypes = [ctypes.c_int32, ctypes.c_uint64, ctypes.c_int32, ctypes.c_int32, ctypes.c_double,
                                      ctypes.c_double]
    lib.gen_rgg_batch_one.restype = P
    lib.gen_threads.argtypes = []
    lib.gen_threads.restype = ctypes.c_int
    _lib = lib
    return lib


@dataclass
class CSR:
    """Undirected graph in compressed sparse rows (int32)."""

    n: int
    row_ptr: np.ndarray
    col: np.ndarray
    name: str = ""

    @property
    def nnz(self) -> int:
        return int(self.col.shape[0])

    @property
    def m(self) -> int:
        """Undirected edge count (nnz / 2 for a symmetric CSR)."""
        return self.nnz // 2

    @property
    def degrees(self) -> np.ndarray:
        return np.diff(self.row_ptr.astype(np.int64))

    @property
    def max_deg(self) -> int:
        return int(self.degrees.max()) if self.n > 0 else 0

    def neighbors(self, v: int) -> np.ndarray:
        return self.col[self.row_ptr[v]:self.row_ptr[v + 1]]


def _take(ptr, name: str) -> CSR:
    lib = _load()
    if not ptr:
        raise MemoryError("graph generator returned NULL")
    g = ptr.contents
    try:
        if g.status != 0:
            raise RuntimeError(f"graph generator failed for {name}: status {g.status}")
        n, nnz = int(g.n), int(g.nnz)
        rp = np.ctypeslib.as_array(g.row_ptr, shape=(n + 1,)).copy() if g.row_ptr else np.zeros(n + 1, np.int32)
        col = np.ctypeslib.as_array(g.col, shape=(nnz,)).copy() if nnz > 0 else np.zeros(0, np.int32)
    finally:
        lib.gen_free(ptr)
    return CSR(n, rp.astype(np.int32, copy=False), col.astype(np.int32, copy=False), name)


def mesh27(N: int) -> CSR:
    """3D 27-point stencil on N^3 vertices, id = x + N*(y + N*z)."""
    return _take(_load().gen_mesh27(N), f"mesh27_{N}")


def grid5(Nx: int, Ny: int | None = None) -> CSR:
    """2D 5-point grid, id = x + Nx*y."""
    Ny = Nx if Ny is None else Ny
    return _take(_load().gen_grid5(Nx, Ny), f"grid5_{Nx}x{Ny}")


def er(n: int, m: int, seed: int = 1) -> CSR:
    """Erdos-Renyi G(n, m): m distinct uniform undirected pairs."""
    return _take(_load().gen_er(n, m, seed), f"er_{n}_{m}_s{seed}")


def rmat(scale: int, ef: int = 16, a: float = 0.57, b: float = 0.19, c: float = 0.19, seed: int = 1) -> CSR:
    """Graph500-style RMAT (no noise, no relabeling), deduplicated and symmetrised."""
    return _take(_load().gen_rmat(scale, ef, a, b, c, seed), f"rmat{scale}_ef{ef}_s{seed}")


def rgg(n: int, r: float, seed: int = 1) -> CSR:
    """Random geometric graph: n points in the unit square, radius r, integer distance test."""
    return _take(_load().gen_rgg(n, r, seed), f"rgg_{n}_s{seed}")


def from_pairs(n: int, pairs) -> CSR:
    """CSR from undirected pairs (self-loops and duplicates removed, symmetrised)."""
    p = np.asarray(pairs, dtype=np.int32).reshape(-1, 2)
    u = np.ascontiguousarray(p[:, 0])
    v = np.ascontiguousarray(p[:, 1])
    i32p = ctypes.POINTER(ctypes.c_int32)
    return _take(_load().gen_from_pairs(n, len(u), u.ctypes.data_as(i32p), v.ctypes.data_as(i32p)), f"pairs_{n}")


# ---- tiny textbook families (closed-form tests) ----

def path(n: int) -> CSR:
    return from_pairs(n, [(i, i + 1) for i in range(n - 1)])


def cycle(n: int) -> CSR:
    return from_pairs(n, [(i, (i + 1) % n) for i in range(n)])


def complete(n: int) -> CSR:
    """K_n: row i lists every other vertex in increasing order."""
    if n < 2:
        return CSR(n, np.zeros(n + 1, np.int32), np.zeros(0, np.int32), f"pairs_{n}")
    col = np.tile(np.arange(n, dtype=np.int32), (n, 1))[~np.eye(n, dtype=bool)]
    rp = (np.arange(n + 1, dtype=np.int64) * (n - 1)).astype(np.int32)
    return CSR(n, rp, np.ascontiguousarray(col), f"pairs_{n}")


def star(n_leaves: int) -> CSR:
    """Center 0, leaves 1..n_leaves."""
    return from_pairs(n_leaves + 1, [(0, i) for i in range(1, n_leaves + 1)])


def empty(n: int) -> CSR:
    return CSR(n, np.zeros(n + 1, np.int32), np.zeros(0, np.int32), f"empty_{n}")


def crown(m: int, interleaved: bool = True) -> CSR:
    """Crown graph S_m^0: K_{m,m} minus a perfect matching.

    interleaved: ids u_i = 2i, v_i = 2i+1 (order u1 v1 u2 v2 ...);
    otherwise u_i = i, v_i = m + i (bipartite order).
    """
    def U(i):
        return 2 * i if interleaved else i

    def V(i):
        return 2 * i + 1 if interleaved else m + i

    return from_pairs(2 * m, [(U(i), V(j)) for i in range(m) for j in range(m) if i != j])


def grid9(N: int) -> CSR:
    """2D 9-point (king's move) grid, id = x + N*y."""
    pairs = []
    for y in range(N):
        for x in range(N):
            for dy in (-1, 0, 1):
                for dx in (-1, 0, 1):
                    if (dx or dy) and 0 <= x + dx < N and 0 <= y + dy < N:
                        pairs.append((x + N * y, x + dx + N * (y + dy)))
    return from_pairs(N * N, pairs)


def relabel(g: CSR, perm: np.ndarray) -> CSR:
    """Graph with vertex v renamed perm[v]."""
    perm = np.asarray(perm, dtype=np.int64)
    src = np.repeat(np.arange(g.n, dtype=np.int64), g.degrees)
    pairs = np.stack([perm[src], perm[g.col.astype(np.int64)]], axis=1)
    pairs = pairs[pairs[:, 0] < pairs[:, 1]]
    return from_pairs(g.n, pairs)


def shuffle_rows(g: CSR, seed: int) -> CSR:
    """Same graph with each adjacency row in a seeded random order."""
    rng = np.random.default_rng(seed)
    col = g.col.copy()
    for v in range(g.n):
        a, b = int(g.row_ptr[v]), int(g.row_ptr[v + 1])
        if b - a > 1:
            col[a:b] = rng.permutation(col[a:b])
    return CSR(g.n, g.row_ptr.copy(), col, g.name + "_shuf")


# ---- packed batch of random geometric graphs ----

@dataclass
class Batch:
    """Packed CSR of G graphs: graph g's local row_ptr (n_g+1 entries) starts
    at row_ptr[vtx_off[g] + g], its local col_idx at col[edge_off[g]], and its
    colors at colors[vtx_off[g]]."""

    num_graphs: int
    vtx_off: np.ndarray  # int64, G+1
    edge_off: np.ndarray  # int64, G+1
    row_ptr: np.ndarray  # int32, sum(n_g + 1)
    col: np.ndarray  # int32, sum(nnz_g)

    def graph(self, g: int) -> CSR:
        n = int(self.vtx_off[g + 1] - self.vtx_off[g])
        rp0 = int(self.vtx_off[g]) + g
        rp = self.row_ptr[rp0:rp0 + n + 1].copy()
        col = self.col[int(self.edge_off[g]):int(self.edge_off[g + 1])].copy()
        return CSR(n, rp, col, f"batch_g{g}")

    def n_of(self, g: int) -> int:
        return int(self.vtx_off[g + 1] - self.vtx_off[g])

    def nnz_of(self, g: int) -> int:
        return int(self.edge_off[g + 1] - self.edge_off[g])


def rgg_batch(G: int, seed: int = 1, n_lo: int = 500, n_hi: int = 50000,
              d_lo: float = 8.0, d_hi: float = 40.0) -> Batch:
    """G random geometric graphs with n_g ~ U{n_lo..n_hi}, target degree d_g ~ U[d_lo, d_hi]."""
    lib = _load()
    i64p = ctypes.POINTER(ctypes.c_int64)
    f64p = ctypes.POINTER(ctypes.c_double)
    i32p = ctypes.POINTER(ctypes.c_int32)
    ns = np.zeros(G, np.int64)
    rs = np.zeros(G, np.float64)
    lib.gen_rgg_batch_params(G, seed, n_lo, n_hi, d_lo, d_hi, ns.ctypes.data_as(i64p), rs.ctypes.data_as(f64p))
    nnz = np.zeros(G, np.int64)
    null32 = ctypes.POINTER(ctypes.c_int32)()
    null64 = ctypes.POINTER(ctypes.c_int64)()
    rc = lib.gen_rgg_batch_fill(G, seed, ns.ctypes.data_as(i64p), rs.ctypes.data_as(f64p), nnz.ctypes.data_as(i64p),
                                null64, null64, null32, null32)
    if rc:
        raise RuntimeError(f"rgg batch sizing failed: {rc}")
    vtx_off = np.zeros(G + 1, np.int64)
    vtx_off[1:] = np.cumsum(ns)
    edge_off = np.zeros(G + 1, np.int64)
    edge_off[1:] = np.cumsum(nnz)
    row_ptr = np.zeros(int(vtx_off[-1]) + G, np.int32)
    col = np.zeros(int(edge_off[-1]), np.int32)
    rc = lib.gen_rgg_batch_fill(G, seed, ns.ctypes.data_as(i64p), rs.ctypes.data_as(f64p), nnz.ctypes.data_as(i64p),
                                vtx_off.ctypes.data_as(i64p), edge_off.ctypes.data_as(i64p),
                                row_ptr.ctypes.data_as(i32p), col.ctypes.data_as(i32p))
    if rc:
        raise RuntimeError(f"rgg batch fill failed: {rc}")
    return Batch(G, vtx_off, edge_off, row_ptr, col)


def rgg_batch_graph(g: int, seed: int = 1, n_lo: int = 500, n_hi: int = 50000,
                    d_lo: float = 8.0, d_hi: float = 40.0) -> CSR:
    """Graph g of rgg_batch(G, seed, ...) on its own (for any G > g)."""
    return _take(_load().gen_rgg_batch_one(g, seed, n_lo, n_hi, d_lo, d_hi), f"rgg_batch_{seed}_g{g}")


def checksum(g: CSR) -> str:
    """SHA-256 of the CSR bytes (n, row_ptr, col; little-endian int32)."""
    import hashlib

    h = hashlib.sha256()
    h.update(np.int64(g.n).tobytes())
    h.update(np.ascontiguousarray(g.row_ptr, dtype="<i4").tobytes())
    h.update(np.ascontiguousarray(g.col, dtype="<i4").tobytes())
    return h.hexdigest()


def threads() -> int:
    return int(_load().gen_threads())


def mesh27_nnz(N: int) -> int:
    return (3 * N - 2) ** 3 - N ** 3 if N > 0 else 0


def log_uniform(rng: np.random.Generator, lo: float, hi: float) -> float:
    return float(math.exp(rng.uniform(math.log(lo), math.log(hi))))


# ---- serving workload: a pool of request graphs and a Poisson arrival trace ----

SERVE_FAMILIES = ("grid5", "er", "rmat")


def serve_graph_spec(rng: np.random.Generator, small: bool = False) -> tuple:
    """One request graph, family uniform over 2D 5-point grids (side
    log-uniform in [32, 2048]), Erdos-Renyi G(n, m) (n log-uniform in
    [10^3, 10^6], average degree uniform in [4, 32]) and RMAT (scale uniform in
    10..20, edge factor 16, Graph500 a, b, c).  small: the same families at
    test sizes (side 16..96, n 500..20000, scale 6..12)."""
    fam = SERVE_FAMILIES[int(rng.integers(0, 3))]
    seed = int(rng.integers(1, 2**31))
    if fam == "grid5":
        side = int(round(log_uniform(rng, 16, 96) if small else log_uniform(rng, 32, 2048)))
        return ("grid5", side)
    if fam == "er":
        n = int(round(log_uniform(rng, 500, 20000) if small else log_uniform(rng, 1e3, 1e6)))
        d = float(rng.uniform(4, 32))
        m = min(int(n * d / 2), n * (n - 1) // 2)
        return ("er", n, m, seed)
    scale = int(rng.integers(6, 13) if small else rng.integers(10, 21))
    return ("rmat", scale, seed)


def serve_graph(spec: tuple) -> CSR:
    if spec[0] == "grid5":
        return grid5(spec[1], spec[1])
    if spec[0] == "er":
        return er(spec[1], spec[2], spec[3])
    return rmat(spec[1], 16, 0.57, 0.19, 0.19, spec[2])


def serve_pool(count: int, seed: int = 1, small: bool = False) -> list:
    """`count` request graphs (specs drawn from one seeded stream)."""
    rng = np.random.default_rng(seed)
    specs = [serve_graph_spec(rng, small) for _ in range(count)]
    return [serve_graph(s) for s in specs]


def serve_trace(count: int, pool_size: int, rate: float, seed: int = 1):
    """Arrival times (seconds, Poisson process of `rate` per second), the pool
    graph of each request and its coloring seed."""
    rng = np.random.default_rng(seed + 7919)
    gaps = rng.exponential(1.0 / rate, count) if rate > 0 else np.zeros(count)
    t = np.cumsum(gaps) - (gaps[0] if count else 0.0)
    which = rng.integers(0, pool_size, count)
    seeds = rng.integers(1, 2**62, count, dtype=np.int64)
    return t, which, seeds
