"""Python binding of libgc (speculative graph coloring with iterated
recoloring on MI355X).  Argument marshalling only: every step of the method
runs in the HIP kernels of ``libgc.so``; torch provides device memory and
streams.  The binding refuses to run without the built library.
"""
from __future__ import annotations

import atexit
import ctypes
import os
import threading
import weakref

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libgc.so")

OK, ERR_ARG, ERR_GRAPH, ERR_COLORING, ERR_OOM, ERR_DEVICE, ERR_NOT_CONVERGED = 0, 1, 2, 3, 4, 5, 6
FIRST_FIT, RANDOM_X = 0, 1
PERM_REVERSE, PERM_NONINC, PERM_NONDEC, PERM_RANDOM = 0, 1, 2, 3
PERM_NAMES = {"RV": PERM_REVERSE, "NI": PERM_NONINC, "ND": PERM_NONDEC, "RAND": PERM_RANDOM}
FLAG_FIXED_PRIORITY = 1
FLAG_PRIO_LF = 2
FLAG_PRIO_NATURAL = 4
FLAG_DISTANCE2 = 8
MAX_X = 1024


class GCError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{msg} (status {status})")
        self.status = status


class CSRArgs(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("reserved", ctypes.c_int32), ("nnz", ctypes.c_int64),
                ("row_ptr", ctypes.c_void_p), ("col_idx", ctypes.c_void_p)]


class StatsArgs(ctypes.Structure):
    _fields_ = [("rounds", ctypes.c_int32), ("num_colors", ctypes.c_int32), ("max_color", ctypes.c_int32),
                ("k_classes", ctypes.c_int32), ("losers_total", ctypes.c_int64),
                ("round_sizes", ctypes.POINTER(ctypes.c_int64)), ("round_degsum", ctypes.POINTER(ctypes.c_int64)),
                ("round_cap", ctypes.c_int32), ("reserved", ctypes.c_int32)]


class Tuning(ctypes.Structure):
    _fields_ = [("block", ctypes.c_int32), ("deg_wave", ctypes.c_int32), ("group", ctypes.c_int32),
                ("grid_per_cu", ctypes.c_int32), ("walk_mode", ctypes.c_int32), ("xcd_chunks", ctypes.c_int32),
                ("check_resident", ctypes.c_int32), ("deg_split", ctypes.c_int32), ("split_len", ctypes.c_int32),
                ("hub_words", ctypes.c_int32), ("walk_group", ctypes.c_int32),
                ("d2_star", ctypes.c_int32), ("batch_wg_per_cu", ctypes.c_int32), ("batch_order", ctypes.c_int32),
                ("spin_limit", ctypes.c_int32), ("check_input", ctypes.c_int32), ("trace", ctypes.c_int32),
                ("tail_max", ctypes.c_int32), ("walk_flags", ctypes.c_int32), ("cu_count", ctypes.c_int32),
                ("compact_init", ctypes.c_int32), ("compact_sat", ctypes.c_int32)]

TUNING_FIELDS = ("block", "deg_wave", "group", "grid_per_cu", "walk_mode", "xcd_chunks", "check_resident", "deg_split",
                 "split_len", "hub_words", "walk_group", "d2_star", "batch_wg_per_cu", "batch_order", "spin_limit",
                 "check_input", "trace", "tail_max", "walk_flags", "cu_count", "compact_init", "compact_sat")


class BatchArgs(ctypes.Structure):
    _fields_ = [("num_graphs", ctypes.c_int32), ("reserved", ctypes.c_int32), ("vtx_off", ctypes.c_void_p),
                ("edge_off", ctypes.c_void_p), ("row_ptr", ctypes.c_void_p), ("col_idx", ctypes.c_void_p)]


_lib = None
_lib_lock = threading.Lock()

# name -> (restype, argtypes); every symbol the C header declares
_SIGS = {
    "gc_status_string": (ctypes.c_char_p, [ctypes.c_int]),
    "gc_ctx_create": (ctypes.c_int, [ctypes.c_int, ctypes.c_int64, ctypes.c_int64, ctypes.POINTER(ctypes.c_void_p)]),
    "gc_ctx_destroy": (None, [ctypes.c_void_p]),
    "gc_ctx_last_error": (ctypes.c_char_p, [ctypes.c_void_p]),
    "gc_ctx_status": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p]),
    "gc_ctx_get_trace": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_int64), ctypes.c_int64,
                                        ctypes.POINTER(ctypes.c_int64), ctypes.c_void_p]),
    "gc_ctx_get_tuning": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(Tuning)]),
    "gc_ctx_set_tuning": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(Tuning)]),
    "gc_check_csr": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(CSRArgs), ctypes.c_void_p]),
    "gc_init_color": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(CSRArgs), ctypes.c_int32, ctypes.c_int32,
                                     ctypes.c_uint64, ctypes.c_int32, ctypes.c_uint32, ctypes.c_void_p,
                                     ctypes.POINTER(StatsArgs), ctypes.c_void_p]),
    "gc_init_color_rounds": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(CSRArgs), ctypes.c_int32, ctypes.c_int32,
                                            ctypes.c_uint64, ctypes.c_int32, ctypes.c_uint32, ctypes.c_void_p,
                                            ctypes.c_void_p, ctypes.POINTER(StatsArgs), ctypes.c_void_p]),
    "gc_recolor": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(CSRArgs), ctypes.c_int32, ctypes.c_uint64,
                                  ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p, ctypes.POINTER(StatsArgs),
                                  ctypes.c_void_p]),
    "gc_recolor_passes": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(CSRArgs), ctypes.POINTER(ctypes.c_int32),
                                         ctypes.c_int32, ctypes.c_uint64, ctypes.c_int32, ctypes.c_void_p,
                                         ctypes.c_void_p, ctypes.POINTER(StatsArgs), ctypes.c_void_p]),
    "gc_recolor_d2": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(CSRArgs), ctypes.c_int32, ctypes.c_uint64,
                                     ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p, ctypes.POINTER(StatsArgs),
                                     ctypes.c_void_p]),
    "gc_validate": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(CSRArgs), ctypes.c_void_p,
                                   ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int64), ctypes.c_void_p]),
    "gc_validate_d2": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(CSRArgs), ctypes.c_void_p,
                                      ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int64), ctypes.c_void_p]),
    "gc_count_colors": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p, ctypes.POINTER(ctypes.c_int32),
                                       ctypes.POINTER(ctypes.c_int32), ctypes.c_void_p]),
    "gc_count_colors_static": (ctypes.c_int, [ctypes.c_int32, ctypes.c_void_p, ctypes.POINTER(ctypes.c_int32),
                                              ctypes.POINTER(ctypes.c_int32), ctypes.c_void_p]),
    "gc_batch_color": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(BatchArgs), ctypes.c_int32, ctypes.c_int32,
                                      ctypes.c_int32, ctypes.c_int32, ctypes.c_uint64, ctypes.c_int32, ctypes.c_int32,
                                      ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "gc_batch_graph_seed": (ctypes.c_uint64, [ctypes.c_uint64, ctypes.c_int32]),
    "gc_autotune": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(CSRArgs), ctypes.c_int32, ctypes.c_int32,
                                   ctypes.c_int32, ctypes.c_int32, ctypes.c_uint64, ctypes.c_void_p,
                                   ctypes.POINTER(Tuning), ctypes.POINTER(ctypes.c_double), ctypes.c_void_p]),
    "gc_autotune_batch": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(BatchArgs), ctypes.c_int32, ctypes.c_int32,
                                         ctypes.c_int32, ctypes.c_int32, ctypes.c_uint64, ctypes.c_int32,
                                         ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p, ctypes.POINTER(Tuning),
                                         ctypes.POINTER(ctypes.c_double), ctypes.c_void_p]),
    "gc_arc_recolor": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32, ctypes.c_uint64, ctypes.c_int32,
                                      ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "gc_schedule_perm": (ctypes.c_int32, [ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32]),
    "gc_color_preset": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32, ctypes.c_uint64,
                                       ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "gc_ctx_set_timing": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int]),
    "gc_ctx_get_info": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_int64), ctypes.c_int]),
    "gc_ctx_get_timing": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_int64),
                                         ctypes.POINTER(ctypes.c_double), ctypes.c_int]),
    # request server (include/gc_serve.h)
    "gc_server_create": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_void_p)]),
    "gc_server_submit": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p]),
    "gc_server_poll": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32,
                                      ctypes.POINTER(ctypes.c_int32), ctypes.c_int32]),
    "gc_server_get_stats": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p]),
    "gc_server_now": (ctypes.c_double, [ctypes.c_void_p]),
    "gc_server_destroy": (None, [ctypes.c_void_p]),
}

KERNEL_KINDS = ("round0", "assign", "detect", "hist", "order", "scatter", "walk", "count", "batch", "other")


def lib():
    """The loaded libgc.so (raises if it has not been built)."""
    global _lib
    with _lib_lock:
        if _lib is None:
            if not os.path.exists(LIB_PATH):
                raise ImportError(f"{LIB_PATH} is missing: build it with `python -c 'import __graft_entry__ as g; g.build()'`")
            L = ctypes.CDLL(LIB_PATH)
            for name, (res, args) in _SIGS.items():
                f = getattr(L, name)
                f.restype = res
                f.argtypes = args
            _lib = L
        return _lib


def status_string(s: int) -> str:
    return lib().gc_status_string(s).decode()


def _torch():
    import torch
    return torch


# Every live context and server, so that they are destroyed at interpreter
# exit while the HIP runtime is still up (before module teardown and the C
# library's exit handlers), servers first since their slots own contexts.
_live_contexts = weakref.WeakSet()
_live_servers = weakref.WeakSet()


def close_all():
    """Synchronize the device and destroy every live Server and Context of
    this process (they are unusable afterwards).  Registered with atexit."""
    servers, contexts = list(_live_servers), list(_live_contexts)
    if not servers and not contexts:
        return
    for srv in servers:
        try:
            srv.close()
        except Exception:
            pass
    try:
        import torch

        if torch.cuda.is_initialized():
            torch.cuda.synchronize()
    except Exception:
        pass
    for c in contexts:
        try:
            c.close()
        except Exception:
            pass
    _default_ctx.clear()


atexit.register(close_all)


def _stream_ptr(stream=None):
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


class Context:
    """Owns a gc_ctx (device workspace) for graphs up to max_n / max_nnz."""

    def __init__(self, max_n: int, max_nnz: int = 0, device: int | None = None):
        torch = _torch()
        self.device = torch.cuda.current_device() if device is None else device
        self.max_n = int(max_n)
        self.max_nnz = int(max_nnz)
        h = ctypes.c_void_p()
        rc = lib().gc_ctx_create(self.device, self.max_n, self.max_nnz, ctypes.byref(h))
        if rc:
            raise GCError(rc, f"gc_ctx_create(max_n={max_n}): {status_string(rc)}")
        self.handle = h
        _live_contexts.add(self)

    def close(self):
        if getattr(self, "handle", None):
            lib().gc_ctx_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def last_error(self) -> str:
        return lib().gc_ctx_last_error(self.handle).decode()

    def status(self, stream=None) -> int:
        """Synchronize the stream and return the context's sticky device status
        (gc_ctx_status): OK, or ERR_DEVICE once for a failure of earlier
        asynchronous work."""
        return lib().gc_ctx_status(self.handle, _stream_ptr(stream))

    def walk_trace(self, stream=None) -> dict:
        """Class-completion trace of the last traced walk (gc_ctx_get_trace), in
        nanoseconds since the walk started: {"end": t, "class_done": [..k],
        "split_done": [..k] (-1: no split row of that rank)}."""
        cnt = ctypes.c_int64()
        self.check(lib().gc_ctx_get_trace(self.handle, None, 0, ctypes.byref(cnt), _stream_ptr(stream)),
                   "gc_ctx_get_trace")
        buf = (ctypes.c_int64 * cnt.value)()
        self.check(lib().gc_ctx_get_trace(self.handle, buf, cnt.value, ctypes.byref(cnt), _stream_ptr(stream)),
                   "gc_ctx_get_trace")
        a = np.frombuffer(buf, dtype=np.int64).copy()
        return {"end": int(a[1]), "class_done": a[2::2].tolist(), "split_done": a[3::2].tolist()}

    def raise_status(self, stream=None):
        """status(), raising GCError on a device failure of earlier work."""
        self.check(self.status(stream), "gc_ctx_status")

    def check(self, rc, what):
        if rc not in (OK,):
            raise GCError(rc, f"{what}: {status_string(rc)}: {self.last_error()}")

    @property
    def tuning(self) -> dict:
        t = Tuning()
        self.check(lib().gc_ctx_get_tuning(self.handle, ctypes.byref(t)), "gc_ctx_get_tuning")
        return {f: getattr(t, f) for f in TUNING_FIELDS}

    def set_timing(self, enable: bool, kinds=None):
        """Turn per-kernel HIP-event timing on (clearing the sums) or off;
        `kinds` limits it to those kernel kinds (names of KERNEL_KINDS)."""
        if not enable:
            arg = 0
        elif kinds is None:
            arg = -1
        else:
            arg = sum(1 << KERNEL_KINDS.index(k) for k in kinds)
        self.check(lib().gc_ctx_set_timing(self.handle, arg), "gc_ctx_set_timing")

    def timing(self) -> dict:
        """{kind: (launches, total ms)} since timing was enabled (synchronizes the device)."""
        n = len(KERNEL_KINDS)
        la = (ctypes.c_int64 * n)()
        ms = (ctypes.c_double * n)()
        self.check(lib().gc_ctx_get_timing(self.handle, la, ms, n), "gc_ctx_get_timing")
        return {k: (int(la[i]), float(ms[i])) for i, k in enumerate(KERNEL_KINDS)}

    def info(self) -> dict:
        a = (ctypes.c_int64 * 5)()
        self.check(lib().gc_ctx_get_info(self.handle, a, 5), "gc_ctx_get_info")
        return {"num_cu": a[0], "walk_blocks": a[1], "walk_blocks_per_cu": a[2], "max_degree": a[3],
                "far_entries": a[4]}

    def set_tuning(self, **kw):
        t = Tuning()
        self.check(lib().gc_ctx_get_tuning(self.handle, ctypes.byref(t)), "gc_ctx_get_tuning")
        for k, v in kw.items():
            setattr(t, k, int(v))
        self.check(lib().gc_ctx_set_tuning(self.handle, ctypes.byref(t)), "gc_ctx_set_tuning")


_default_ctx: dict[int, Context] = {}


def default_context(n: int, nnz: int = 0) -> Context:
    """Per-device context, regrown when a larger graph arrives."""
    torch = _torch()
    dev = torch.cuda.current_device()
    c = _default_ctx.get(dev)
    if c is None or c.max_n < n or c.max_nnz < nnz:
        if c is not None:
            torch.cuda.synchronize()
            c.close()
        c = Context(max(n, 1024), max(nnz, 1024), dev)
        _default_ctx[dev] = c
    return c


def _check_i32_dev(t, name, numel=None):
    torch = _torch()
    if not isinstance(t, torch.Tensor) or t.dtype != torch.int32 or not t.is_cuda or not t.is_contiguous():
        raise TypeError(f"{name} must be a contiguous torch.int32 CUDA (HIP) tensor")
    if numel is not None and t.numel() != numel:
        raise ValueError(f"{name} must have {numel} elements, has {t.numel()}")


def _csr_args(row_ptr, col_idx) -> CSRArgs:
    _check_i32_dev(row_ptr, "row_ptr")
    _check_i32_dev(col_idx, "col_idx")
    n = row_ptr.numel() - 1
    if n < 0:
        raise ValueError("row_ptr needs n + 1 >= 1 entries")
    return CSRArgs(n, 0, col_idx.numel(), row_ptr.data_ptr(), col_idx.data_ptr() if col_idx.numel() else None)


def _stats_dict(st: StatsArgs, sizes=None, degsum=None) -> dict:
    d = {"rounds": st.rounds, "num_colors": st.num_colors, "max_color": st.max_color, "k_classes": st.k_classes,
         "losers_total": st.losers_total}
    if sizes is not None:
        r = min(st.rounds, len(sizes))
        d["round_sizes"] = sizes[:r].tolist()
        d["round_degsum"] = degsum[:r].tolist()
    return d


def init_color(row_ptr, col_idx, select=FIRST_FIT, X=1, seed=1, max_rounds=0, flags=0, out=None, stats=True,
               round_cap=4096, ctx: Context | None = None, stream=None, allow_not_converged=False):
    """Speculative initial coloring; returns (colors int32 tensor, stats dict or None)."""
    torch = _torch()
    g = _csr_args(row_ptr, col_idx)
    ctx = ctx or default_context(g.n, g.nnz)
    if out is None:
        out = torch.empty(max(g.n, 0), dtype=torch.int32, device=row_ptr.device)
    _check_i32_dev(out, "out", g.n)
    st = None
    sizes = degsum = None
    if stats:
        sizes = np.zeros(round_cap, np.int64)
        degsum = np.zeros(round_cap, np.int64)
        st = StatsArgs()
        st.round_sizes = sizes.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))
        st.round_degsum = degsum.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))
        st.round_cap = round_cap
    rc = lib().gc_init_color(ctx.handle, ctypes.byref(g), select, X, seed, max_rounds, flags,
                             out.data_ptr() if g.n else None, ctypes.byref(st) if st is not None else None,
                             _stream_ptr(stream))
    if not (rc == ERR_NOT_CONVERGED and allow_not_converged):
        ctx.check(rc, "gc_init_color")
    d = _stats_dict(st, sizes, degsum) if st is not None else None
    if d is not None:
        d["status"] = rc
    return out, d


def init_color_rounds(row_ptr, col_idx, select=FIRST_FIT, X=1, seed=1, max_rounds=0, flags=0, out=None,
                      ctx: Context | None = None, stream=None, allow_not_converged=False):
    """Initial coloring that also returns each vertex's commit round (-1:
    still uncolored).  Returns (colors, rounds int32 tensor, stats dict)."""
    torch = _torch()
    g = _csr_args(row_ptr, col_idx)
    ctx = ctx or default_context(g.n, g.nnz)
    if out is None:
        out = torch.empty(max(g.n, 0), dtype=torch.int32, device=row_ptr.device)
    _check_i32_dev(out, "out", g.n)
    vr = torch.empty(max(g.n, 0), dtype=torch.int32, device=row_ptr.device)
    st = StatsArgs()
    rc = lib().gc_init_color_rounds(ctx.handle, ctypes.byref(g), select, X, seed, max_rounds, flags,
                                    out.data_ptr() if g.n else None, vr.data_ptr() if g.n else None,
                                    ctypes.byref(st), _stream_ptr(stream))
    if not (rc == ERR_NOT_CONVERGED and allow_not_converged):
        ctx.check(rc, "gc_init_color_rounds")
    d = _stats_dict(st)
    d["status"] = rc
    return out, vr, d


def recolor(row_ptr, col_idx, colors, perm=PERM_REVERSE, seed=1, pass_=0, out=None, stats=True,
            ctx: Context | None = None, stream=None):
    """One recoloring pass; `out` may be `colors` (in place).  Returns (colors, stats or None)."""
    torch = _torch()
    g = _csr_args(row_ptr, col_idx)
    _check_i32_dev(colors, "colors", g.n)
    ctx = ctx or default_context(g.n, g.nnz)
    if out is None:
        out = torch.empty_like(colors)
    _check_i32_dev(out, "out", g.n)
    st = StatsArgs() if stats else None
    rc = lib().gc_recolor(ctx.handle, ctypes.byref(g), perm, seed, pass_, colors.data_ptr() if g.n else None,
                          out.data_ptr() if g.n else None, ctypes.byref(st) if st is not None else None,
                          _stream_ptr(stream))
    ctx.check(rc, "gc_recolor")
    return out, (_stats_dict(st) if st is not None else None)


def recolor_passes(row_ptr, col_idx, colors, perms, seed=1, pass0=0, out=None, stats=True,
                   ctx: Context | None = None, stream=None):
    """len(perms) recoloring passes in one call (pass p uses perms[p] and pass
    index pass0 + p); `out` may be `colors`.  Returns (colors, list of stats
    dicts or None)."""
    torch = _torch()
    g = _csr_args(row_ptr, col_idx)
    _check_i32_dev(colors, "colors", g.n)
    ctx = ctx or default_context(g.n, g.nnz)
    if out is None:
        out = torch.empty_like(colors)
    _check_i32_dev(out, "out", g.n)
    pa = (ctypes.c_int32 * max(len(perms), 1))(*[int(p) for p in perms])
    st = (StatsArgs * max(len(perms), 1))() if stats else None
    rc = lib().gc_recolor_passes(ctx.handle, ctypes.byref(g), pa, len(perms), seed, pass0,
                                 colors.data_ptr() if g.n else None, out.data_ptr() if g.n else None,
                                 st, _stream_ptr(stream))
    ctx.check(rc, "gc_recolor_passes")
    return out, ([_stats_dict(st[i]) for i in range(len(perms))] if st is not None else None)


def recolor_d2(row_ptr, col_idx, colors, perm=PERM_REVERSE, seed=1, pass_=0, out=None, stats=True,
               ctx: Context | None = None, stream=None):
    """One recoloring pass of a distance-2 coloring; `out` may be `colors`.
    Returns (colors, stats or None)."""
    torch = _torch()
    g = _csr_args(row_ptr, col_idx)
    _check_i32_dev(colors, "colors", g.n)
    ctx = ctx or default_context(g.n, g.nnz)
    if out is None:
        out = torch.empty_like(colors)
    _check_i32_dev(out, "out", g.n)
    st = StatsArgs() if stats else None
    rc = lib().gc_recolor_d2(ctx.handle, ctypes.byref(g), perm, seed, pass_, colors.data_ptr() if g.n else None,
                             out.data_ptr() if g.n else None, ctypes.byref(st) if st is not None else None,
                             _stream_ptr(stream))
    ctx.check(rc, "gc_recolor_d2")
    return out, (_stats_dict(st) if st is not None else None)


def arc_recolor(row_ptr, col_idx, colors, perm=PERM_REVERSE, seed=1, pass_=0, out=None, stats=True,
                ctx: Context | None = None, stream=None):
    """Asynchronous recoloring (aRC); `out` may be `colors`.  Returns (colors, stats or None)."""
    torch = _torch()
    g = _csr_args(row_ptr, col_idx)
    _check_i32_dev(colors, "colors", g.n)
    ctx = ctx or default_context(g.n, g.nnz)
    if out is None:
        out = torch.empty_like(colors)
    _check_i32_dev(out, "out", g.n)
    st = StatsArgs() if stats else None
    rc = lib().gc_arc_recolor(ctx.handle, ctypes.byref(g), perm, seed, pass_, colors.data_ptr() if g.n else None,
                              out.data_ptr() if g.n else None, ctypes.byref(st) if st is not None else None,
                              _stream_ptr(stream))
    ctx.check(rc, "gc_arc_recolor")
    return out, (_stats_dict(st) if st is not None else None)


def validate(row_ptr, col_idx, colors, ctx: Context | None = None, stream=None):
    """(conflicting edges, uncolored vertices)."""
    g = _csr_args(row_ptr, col_idx)
    _check_i32_dev(colors, "colors", g.n)
    ctx = ctx or default_context(g.n, g.nnz)
    cf, un = ctypes.c_int64(), ctypes.c_int64()
    rc = lib().gc_validate(ctx.handle, ctypes.byref(g), colors.data_ptr() if g.n else None, ctypes.byref(cf),
                           ctypes.byref(un), _stream_ptr(stream))
    ctx.check(rc, "gc_validate")
    return cf.value, un.value


def validate_d2(row_ptr, col_idx, colors, ctx: Context | None = None, stream=None):
    """(pairs of vertices within two edges of each other sharing a positive color, uncolored vertices)."""
    g = _csr_args(row_ptr, col_idx)
    _check_i32_dev(colors, "colors", g.n)
    ctx = ctx or default_context(g.n, g.nnz)
    cf, un = ctypes.c_int64(), ctypes.c_int64()
    rc = lib().gc_validate_d2(ctx.handle, ctypes.byref(g), colors.data_ptr() if g.n else None, ctypes.byref(cf),
                              ctypes.byref(un), _stream_ptr(stream))
    ctx.check(rc, "gc_validate_d2")
    return cf.value, un.value


def count_colors(colors, ctx: Context | None = None, stream=None):
    """(distinct positive colors, max color)."""
    _check_i32_dev(colors, "colors")
    n = colors.numel()
    ctx = ctx or default_context(n)
    num, mx = ctypes.c_int32(), ctypes.c_int32()
    rc = lib().gc_count_colors(ctx.handle, n, colors.data_ptr() if n else None, ctypes.byref(num), ctypes.byref(mx),
                               _stream_ptr(stream))
    ctx.check(rc, "gc_count_colors")
    return num.value, mx.value


STATIC_MAX_COLOR = 1 << 20


def count_colors_static(colors, stream=None):
    """(distinct positive colors, max color) through the allocation-free
    gc_count_colors_static (no context; colors up to STATIC_MAX_COLOR)."""
    _check_i32_dev(colors, "colors")
    n = colors.numel()
    num, mx = ctypes.c_int32(), ctypes.c_int32()
    rc = lib().gc_count_colors_static(n, colors.data_ptr() if n else None, ctypes.byref(num), ctypes.byref(mx),
                                      _stream_ptr(stream))
    if rc:
        raise GCError(rc, f"gc_count_colors_static: {status_string(rc)}")
    return num.value, mx.value


def check_csr(row_ptr, col_idx, ctx: Context | None = None, stream=None) -> int:
    """GC_OK (0) or GC_ERR_GRAPH (2)."""
    g = _csr_args(row_ptr, col_idx)
    ctx = ctx or default_context(g.n, g.nnz)
    rc = lib().gc_check_csr(ctx.handle, ctypes.byref(g), _stream_ptr(stream))
    if rc not in (OK, ERR_GRAPH):
        ctx.check(rc, "gc_check_csr")
    return rc


def batch_graph_seed(base_seed: int, g: int) -> int:
    return int(lib().gc_batch_graph_seed(base_seed, g))


GRAPH_STATS_FIELDS = ("rounds", "colors_init", "colors_final", "status")


def batch_color(vtx_off, edge_off, row_ptr, col_idx, select=RANDOM_X, X=4, perm=PERM_REVERSE, passes=5, base_seed=1,
                max_rounds=0, max_vertices_per_graph=None, out=None, per_graph=None, ctx: Context | None = None,
                stream=None):
    """Color every graph of a packed batch in one persistent launch (asynchronous).

    Returns (colors, per_graph int32 tensor of shape (G, 4): rounds, colors_init, colors_final, status)."""
    torch = _torch()
    for t, nm in ((vtx_off, "vtx_off"), (edge_off, "edge_off")):
        if t.dtype != torch.int64 or not t.is_cuda or not t.is_contiguous():
            raise TypeError(f"{nm} must be a contiguous torch.int64 CUDA tensor")
    _check_i32_dev(row_ptr, "row_ptr")
    _check_i32_dev(col_idx, "col_idx")
    G = vtx_off.numel() - 1
    total_v = row_ptr.numel() - G
    if max_vertices_per_graph is None:
        max_vertices_per_graph = int((vtx_off[1:] - vtx_off[:-1]).max().item()) if G > 0 else 0
    ctx = ctx or default_context(max(max_vertices_per_graph, 1))
    if out is None:
        out = torch.empty(max(total_v, 0), dtype=torch.int32, device=row_ptr.device)
    if per_graph is None:
        per_graph = torch.empty((max(G, 0), 4), dtype=torch.int32, device=row_ptr.device)
    b = BatchArgs(G, 0, vtx_off.data_ptr(), edge_off.data_ptr(), row_ptr.data_ptr(),
                  col_idx.data_ptr() if col_idx.numel() else None)
    rc = lib().gc_batch_color(ctx.handle, ctypes.byref(b), select, X, perm, passes, base_seed, max_rounds,
                              int(max_vertices_per_graph), out.data_ptr() if out.numel() else None,
                              per_graph.data_ptr() if G > 0 else None, _stream_ptr(stream))
    ctx.check(rc, "gc_batch_color")
    return out, per_graph


def _tuning_dict(t: Tuning) -> dict:
    return {f: getattr(t, f) for f in TUNING_FIELDS}


def autotune(row_ptr, col_idx, select=RANDOM_X, X=4, perm=PERM_NONINC, passes=3, seed=1, out=None,
             ctx: Context | None = None, stream=None):
    """Pick the fastest scheduling knobs for this graph and method (colors are
    checked identical under every candidate); the setting stays in ctx.
    Returns (tuning dict, ms of one run, colors)."""
    torch = _torch()
    g = _csr_args(row_ptr, col_idx)
    ctx = ctx or default_context(g.n, g.nnz)
    if out is None:
        out = torch.empty(max(g.n, 0), dtype=torch.int32, device=row_ptr.device)
    _check_i32_dev(out, "out", g.n)
    best, ms = Tuning(), ctypes.c_double()
    rc = lib().gc_autotune(ctx.handle, ctypes.byref(g), select, X, perm, passes, seed, out.data_ptr() if g.n else None,
                           ctypes.byref(best), ctypes.byref(ms), _stream_ptr(stream))
    ctx.check(rc, "gc_autotune")
    return _tuning_dict(best), ms.value, out


def autotune_batch(vtx_off, edge_off, row_ptr, col_idx, select=RANDOM_X, X=4, perm=PERM_REVERSE, passes=5,
                   base_seed=1, max_rounds=0, max_vertices_per_graph=None, out=None, per_graph=None,
                   ctx: Context | None = None, stream=None):
    """Pick batch_order and batch_wg_per_cu for gc_batch_color on this batch
    (colors and per-graph statistics checked identical under every candidate);
    the setting stays in ctx.  Returns (tuning dict, ms of one launch, colors, per_graph)."""
    torch = _torch()
    G = vtx_off.numel() - 1
    total_v = row_ptr.numel() - G
    if max_vertices_per_graph is None:
        max_vertices_per_graph = int((vtx_off[1:] - vtx_off[:-1]).max().item()) if G > 0 else 0
    ctx = ctx or default_context(max(max_vertices_per_graph, 1))
    if out is None:
        out = torch.empty(max(total_v, 0), dtype=torch.int32, device=row_ptr.device)
    if per_graph is None:
        per_graph = torch.empty((max(G, 0), 4), dtype=torch.int32, device=row_ptr.device)
    b = BatchArgs(G, 0, vtx_off.data_ptr(), edge_off.data_ptr(), row_ptr.data_ptr(),
                  col_idx.data_ptr() if col_idx.numel() else None)
    best, ms = Tuning(), ctypes.c_double()
    rc = lib().gc_autotune_batch(ctx.handle, ctypes.byref(b), select, X, perm, passes, base_seed, max_rounds,
                                 int(max_vertices_per_graph), out.data_ptr() if out.numel() else None,
                                 per_graph.data_ptr() if G > 0 else None, ctypes.byref(best), ctypes.byref(ms),
                                 _stream_ptr(stream))
    ctx.check(rc, "gc_autotune_batch")
    return _tuning_dict(best), ms.value, out, per_graph


SCHED_FIXED, SCHED_ND_RAND_X, SCHED_ND_RAND_POW2 = 0, 1, 2
PRESET_SPEED, PRESET_QUALITY = 0, 1


def schedule_perm(kind: int, base: int, x: int, t: int) -> int:
    """Class order of iteration t (1-based) under a hybrid schedule (gc_schedule_perm):
    kind 0 = `base` every time; 1 = ND-RAND%x; 2 = ND-RAND%2^i (RAND at t = 2, 4, 8, ...)."""
    p = int(lib().gc_schedule_perm(kind, base, x, t))
    if p < 0:
        raise ValueError(f"bad schedule arguments ({kind}, {base}, {x}, {t})")
    return p


def color_preset(row_ptr, col_idx, preset=PRESET_QUALITY, seed=1, out=None, stats=True, ctx: Context | None = None,
                 stream=None):
    """The paper's "speed" / "quality" parameter presets (gc_color_preset)."""
    torch = _torch()
    g = _csr_args(row_ptr, col_idx)
    ctx = ctx or default_context(g.n, g.nnz)
    if out is None:
        out = torch.empty(max(g.n, 0), dtype=torch.int32, device=row_ptr.device)
    _check_i32_dev(out, "out", g.n)
    st = StatsArgs() if stats else None
    rc = lib().gc_color_preset(ctx.handle, ctypes.byref(g), preset, seed, out.data_ptr() if g.n else None,
                               ctypes.byref(st) if st is not None else None, _stream_ptr(stream))
    ctx.check(rc, "gc_color_preset")
    return out, (_stats_dict(st) if st is not None else None)


def color(row_ptr, col_idx, select=RANDOM_X, X=4, seed=1, perms=(PERM_REVERSE,), ctx=None, stream=None, stats=True):
    """Initial coloring followed by one recoloring pass per entry of `perms` (pass p uses index p)."""
    c, s0 = init_color(row_ptr, col_idx, select, X, seed, ctx=ctx, stream=stream, stats=stats)
    hist = [s0]
    for p, perm in enumerate(perms):
        c, sp = recolor(row_ptr, col_idx, c, perm, seed, p, out=c, ctx=ctx, stream=stream, stats=stats)
        hist.append(sp)
    return c, hist


# ---------------------------------------------------------------------------
# request server (continuous batching of independent graphs on one GPU)
# ---------------------------------------------------------------------------

class ServerConfigArgs(ctypes.Structure):
    _fields_ = [("device", ctypes.c_int32), ("slots", ctypes.c_int32), ("hbm_budget", ctypes.c_int64),
                ("max_n", ctypes.c_int64), ("max_nnz", ctypes.c_int64), ("cu_partition", ctypes.c_int32),
                ("reserved", ctypes.c_int32)]


class RequestArgs(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("reserved", ctypes.c_int32), ("nnz", ctypes.c_int64),
                ("row_ptr", ctypes.c_void_p), ("col_idx", ctypes.c_void_p), ("colors", ctypes.c_void_p),
                ("select", ctypes.c_int32), ("X", ctypes.c_int32), ("perm", ctypes.c_int32), ("passes", ctypes.c_int32),
                ("seed", ctypes.c_uint64), ("tag", ctypes.c_uint64)]


class RequestDoneArgs(ctypes.Structure):
    _fields_ = [("tag", ctypes.c_uint64), ("status", ctypes.c_int32), ("slot", ctypes.c_int32),
                ("rounds", ctypes.c_int32), ("colors_init", ctypes.c_int32), ("colors_final", ctypes.c_int32),
                ("running_at_admit", ctypes.c_int32), ("footprint", ctypes.c_int64), ("t_submit", ctypes.c_double),
                ("t_admit", ctypes.c_double), ("t_done", ctypes.c_double), ("device_ms", ctypes.c_double),
                ("pass_start_ms", ctypes.c_double), ("pass_end_ms", ctypes.c_double)]


class ServerStatsArgs(ctypes.Structure):
    _fields_ = [(k, ctypes.c_int64) for k in ("submitted", "completed", "waiting", "running", "peak_running",
                                              "arena_size", "arena_used", "arena_peak", "cu_partition", "slot_cus")]


def request_footprint(n: int, nnz: int) -> int:
    """Arena bytes a request holds: row_ptr, col_idx and colors, each rounded up to 256 bytes."""
    a = lambda x: (x + 255) // 256 * 256
    return a(4 * (n + 1)) + a(4 * nnz) + a(4 * n)


class Server:
    """Continuous-batching request server of libgc (gc_serve.h).  Requests are
    host CSR graphs (numpy int32); results come back as host color arrays."""

    def __init__(self, slots=4, hbm_budget=16 << 30, max_n=1 << 22, max_nnz=1 << 26, device=0, cu_partition=1):
        cfg = ServerConfigArgs(device, slots, hbm_budget, max_n, max_nnz, cu_partition, 0)
        h = ctypes.c_void_p()
        rc = lib().gc_server_create(ctypes.byref(cfg), ctypes.byref(h))
        if rc:
            raise GCError(rc, f"gc_server_create: {status_string(rc)}")
        self.handle = h
        _live_servers.add(self)
        self._live = {}
        self._lock = threading.Lock()
        self._next = 0

    def submit(self, row_ptr, col, select=RANDOM_X, X=4, perm=PERM_REVERSE, passes=3, seed=1, tag=None) -> int:
        rp = np.ascontiguousarray(row_ptr, dtype=np.int32)
        cl = np.ascontiguousarray(col, dtype=np.int32)
        n = rp.shape[0] - 1
        out = np.zeros(max(n, 0), np.int32)
        with self._lock:
            if tag is None:
                tag = self._next
            self._next = max(self._next, tag + 1)
            self._live[tag] = (rp, cl, out)
        r = RequestArgs(n, 0, cl.shape[0], rp.ctypes.data, cl.ctypes.data if cl.size else None,
                        out.ctypes.data if n else None, select, X if select == RANDOM_X else 1, perm, passes,
                        seed, tag)
        rc = lib().gc_server_submit(self.handle, ctypes.byref(r))
        if rc:
            with self._lock:
                self._live.pop(tag, None)
            raise GCError(rc, f"gc_server_submit: {status_string(rc)}")
        return tag

    def poll(self, timeout_ms=-1, cap=256) -> list:
        buf = (RequestDoneArgs * cap)()
        cnt = ctypes.c_int32()
        rc = lib().gc_server_poll(self.handle, buf, cap, ctypes.byref(cnt), timeout_ms)
        if rc:
            raise GCError(rc, f"gc_server_poll: {status_string(rc)}")
        res = []
        for i in range(cnt.value):
            d = {k: getattr(buf[i], k) for k, _ in RequestDoneArgs._fields_}
            with self._lock:
                d["colors"] = self._live.pop(d["tag"])[2]
            res.append(d)
        return res

    def stats(self) -> dict:
        st = ServerStatsArgs()
        lib().gc_server_get_stats(self.handle, ctypes.byref(st))
        return {k: getattr(st, k) for k, _ in ServerStatsArgs._fields_}

    def now(self) -> float:
        return lib().gc_server_now(self.handle)

    def close(self):
        if self.handle:
            lib().gc_server_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
