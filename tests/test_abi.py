"""Host-side checks of the C ABI library (no GPU needed): it loads, exports
every symbol include/gc.h declares, and its host helpers agree with the
oracle's definitions."""
import ctypes
import os
import re
import subprocess

import pytest

import oracle

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_1407_6745_amd", "libgc.so")
HEADERS = [os.path.join(ROOT, "include", h) for h in ("gc.h", "gc_serve.h")]


def declared_functions():
    names = set()
    for h in HEADERS:
        src = re.sub(r"/\*.*?\*/", "", open(h).read(), flags=re.S)
        names |= set(re.findall(r"\b(gc_[a-z_0-9]+)\s*\(", src))
    return sorted(names)


def test_header_declares_the_boundary():
    names = declared_functions()
    for must in ("gc_init_color", "gc_recolor", "gc_validate", "gc_count_colors", "gc_batch_color", "gc_check_csr",
                 "gc_ctx_create", "gc_ctx_destroy", "gc_status_string", "gc_server_create", "gc_server_submit",
                 "gc_server_poll", "gc_server_destroy"):
        assert must in names


def test_library_exports_every_declared_symbol():
    assert os.path.exists(LIB), "libgc.so not built"
    out = subprocess.run(["nm", "-D", "--defined-only", LIB], capture_output=True, text=True, check=True).stdout
    exported = set(re.findall(r"\bT (gc_[a-z_0-9]+)\b", out))
    missing = [n for n in declared_functions() if n not in exported]
    assert not missing, missing
    L = ctypes.CDLL(LIB)
    for n in declared_functions():
        getattr(L, n)


def test_binding_binds_every_symbol():
    import paper_1407_6745_amd as gc

    assert set(gc._SIGS) == set(declared_functions())
    gc.lib()


def test_status_strings():
    import paper_1407_6745_amd as gc

    texts = {s: gc.status_string(s) for s in range(7)}
    assert texts[0] == "ok" and len(set(texts.values())) == 7
    assert gc.status_string(99) == "unknown status"


def test_batch_graph_seed_matches_oracle_definition():
    import paper_1407_6745_amd as gc

    for base in (1, 12345, 2**63 + 5):
        for g in (0, 1, 7, 4095):
            assert gc.batch_graph_seed(base, g) == oracle.graph_seed(base, g)


def test_ctx_create_fails_cleanly_without_gpu():
    import torch

    import paper_1407_6745_amd as gc

    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    h = ctypes.c_void_p()
    rc = gc.lib().gc_ctx_create(0, 1000, 1000, ctypes.byref(h))
    assert rc == gc.ERR_DEVICE and not h.value
    assert gc.lib().gc_ctx_create(0, -1, 0, ctypes.byref(h)) == gc.ERR_ARG


def test_no_oracle_in_product_path():
    # the package never imports or loads the oracle
    pkg = os.path.join(ROOT, "paper_1407_6745_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".h", ".cpp")):
                text = open(os.path.join(dirpath, f)).read()
                assert "import oracle" not in text and "liboracle" not in text and "gc_oracle" not in text, f


def test_server_struct_layouts():
    """The binding's ctypes mirrors of the server structs have the C sizes."""
    import paper_1407_6745_amd as gc

    assert ctypes.sizeof(gc.ServerConfigArgs) == 40
    assert ctypes.sizeof(gc.RequestArgs) == 72
    assert ctypes.sizeof(gc.RequestDoneArgs) == 88
    assert ctypes.sizeof(gc.ServerStatsArgs) == 80
    assert gc.request_footprint(0, 0) == 256 + 0 + 0
    assert gc.request_footprint(100, 1000) == 512 + 4096 + 512


def test_server_create_rejects_bad_config_without_gpu():
    import torch

    import paper_1407_6745_amd as gc

    h = ctypes.c_void_p()
    for cfg in (gc.ServerConfigArgs(0, 0, 1 << 20, 10, 10), gc.ServerConfigArgs(0, 65, 1 << 20, 10, 10),
                gc.ServerConfigArgs(0, 2, 0, 10, 10), gc.ServerConfigArgs(0, 2, 1 << 20, -1, 10)):
        assert gc.lib().gc_server_create(ctypes.byref(cfg), ctypes.byref(h)) == gc.ERR_ARG and not h.value
    if not torch.cuda.is_available():
        cfg = gc.ServerConfigArgs(0, 2, 1 << 20, 10, 10)
        rc = gc.lib().gc_server_create(ctypes.byref(cfg), ctypes.byref(h))
        assert rc in (gc.ERR_DEVICE, gc.ERR_OOM) and not h.value


def test_schedule_perm_matches_oracle():
    """The library's schedule helper against the oracle's definition (section 4.2.1)."""
    import paper_1407_6745_amd as gc

    for t in range(1, 70):
        for x in range(1, 13):
            assert gc.schedule_perm(gc.SCHED_ND_RAND_X, 0, x, t) == oracle.schedule_perm(1, 0, x, t)
        assert gc.schedule_perm(gc.SCHED_ND_RAND_POW2, 0, 0, t) == oracle.schedule_perm(2, 0, 0, t)
        for base in range(4):
            assert gc.schedule_perm(gc.SCHED_FIXED, base, 0, t) == oracle.schedule_perm(0, base, 0, t)
    lib = gc.lib()
    for bad in ((3, 0, 1, 1), (-1, 0, 1, 1), (0, 4, 0, 1), (0, 0, 0, 0), (1, 0, 0, 5)):
        assert lib.gc_schedule_perm(*bad) == -1


def _struct_members(header, name):
    """Member names, in order, of `typedef struct name { ... } name;` in a header."""
    src = re.sub(r"/\*.*?\*/", "", open(header).read(), flags=re.S)
    body = re.search(r"typedef struct %s \{(.*?)\} %s;" % (name, name), src, flags=re.S).group(1)
    names = []
    for decl in body.split(";"):
        for part in decl.split(","):  # the last identifier of each declarator is the member
            ids = re.findall(r"[A-Za-z_]\w*", part.split("[")[0])
            if ids:
                names.append(ids[-1])
    return names


def test_tuning_struct_matches_header():
    """The binding's gc_tuning mirror has the header's members in the header's
    order (all int32), and every knob is one the binding can set by name."""
    import paper_1407_6745_amd as gc

    members = _struct_members(HEADERS[0], "gc_tuning")
    assert [f[0] for f in gc.Tuning._fields_] == members
    assert all(t is ctypes.c_int32 for _, t in gc.Tuning._fields_)
    assert ctypes.sizeof(gc.Tuning) == 4 * len(members)
    assert list(gc.TUNING_FIELDS) == members


def test_stats_and_batch_structs_match_header():
    import paper_1407_6745_amd as gc

    assert [f[0] for f in gc.CSRArgs._fields_] == _struct_members(HEADERS[0], "gc_csr")
    assert [f[0] for f in gc.BatchArgs._fields_] == _struct_members(HEADERS[0], "gc_batch_csr")


def test_server_structs_match_header():
    import paper_1407_6745_amd as gc

    for cls, name in ((gc.ServerConfigArgs, "gc_server_config"), (gc.RequestArgs, "gc_request"),
                      (gc.RequestDoneArgs, "gc_request_done"), (gc.ServerStatsArgs, "gc_server_stats")):
        assert [f[0] for f in cls._fields_] == _struct_members(HEADERS[1], name), name
