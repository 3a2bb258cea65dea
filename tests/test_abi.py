"""The C-ABI library loads and exports every entry point include/lsh.h declares
(no GPU work: only dlopen and symbol lookup)."""
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "lsh.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(lsh_[a-z0-9_]+)\s*\(", src)))


def test_header_declares_boundary():
    names = _declared()
    for want in ("lsh_hash_cs", "lsh_hash_hcs", "lsh_hash_dense", "lsh_build_index", "lsh_query"):
        assert want in names


def test_library_exports_every_declared_symbol():
    from paper_2503_06737_amd import lsh
    if not os.path.exists(lsh.LIB_PATH):
        pytest.skip("liblsh.so not built (run __graft_entry__.build())")
    L = lsh.lib()
    missing = [n for n in _declared() if not hasattr(L, n)]
    assert not missing, missing
    assert set(lsh.EXPORTS) <= set(_declared())


def test_library_argument_errors_need_no_gpu():
    """Host-side validation rejects bad arguments before touching the device."""
    import ctypes as C
    from paper_2503_06737_amd import lsh
    if not os.path.exists(lsh.LIB_PATH):
        pytest.skip("liblsh.so not built")
    L = lsh.lib()
    pts = lsh.Points(None, 0, None, 10, 0, 0)           # d = 0
    disc = lsh.Disc(0, 8, 4, 2, 1.0, None, 0)
    out = lsh.Out(None, 0, None, None, None)
    st = L.lsh_hash_cs(C.byref(pts), C.c_void_p(1), C.c_void_p(1), C.byref(disc), C.byref(out),
                       None, 0, None)
    assert st == -1 and b"shape" in L.lsh_last_error()
    pts = lsh.Points(C.c_void_p(16), 0, None, 10, 4, 4)
    disc = lsh.Disc(0, 9, 4, 2, 1.0, C.c_void_p(16), 0)  # m != K*L
    st = L.lsh_hash_cs(C.byref(pts), C.c_void_p(1), C.c_void_p(1), C.byref(disc), C.byref(out),
                       None, 0, None)
    assert st == -1 and b"m = K*L" in L.lsh_last_error()
    disc = lsh.Disc(0, 8, 4, 2, 1.0, C.c_void_p(16), 3)  # recheck outside 0..2
    st = L.lsh_hash_cs(C.byref(pts), C.c_void_p(1), C.c_void_p(1), C.byref(disc), C.byref(out),
                       None, 0, None)
    assert st == -1 and b"recheck" in L.lsh_last_error()
    disc = lsh.Disc(0, 8, 4, 2, 1.0, C.c_void_p(16), 2)  # reuse needs the caller's workspace
    st = L.lsh_hash_cs_noalloc(C.byref(pts), C.c_void_p(1), C.c_void_p(1), C.byref(disc),
                               C.byref(out), None)
    assert st == -1 and b"recheck = 2" in L.lsh_last_error()
    h = C.c_void_p()
    st = L.lsh_build_index(C.c_void_p(256), 0, 10, 2, (1 << 32) - 5, C.c_void_p(256), 1 << 20,
                           C.c_void_p(256), 1 << 20, C.byref(h), None, None)
    assert st == -5
    assert L.lsh_index_bytes(1000, 4) >= 1000 * 4 * 16


def test_query_workspace_sizes_need_no_gpu():
    """lsh_query_workspace_bytes: the shares' top-k lists and counts for 1..1024
    queries (four shares at most), 0 outside that range or for k outside 1..64."""
    from paper_2503_06737_amd import lsh
    if not os.path.exists(lsh.LIB_PATH):
        pytest.skip("liblsh.so not built")
    L = lsh.lib()
    assert L.lsh_query_workspace_bytes(1, 10) == 4 * (10 * 8 + 4)
    assert L.lsh_query_workspace_bytes(1024, 64) == 1024 * 4 * (64 * 8 + 4)
    for nq, k in ((0, 10), (1025, 10), (10, 0), (10, 65), (-1, 10)):
        assert L.lsh_query_workspace_bytes(nq, k) == 0, (nq, k)
