"""Python binding of liblsh (ctypes).  Argument marshalling only.

Every step of hashing, indexing and querying runs in the HIP kernels of
``liblsh.so``; this module turns torch tensors (device memory) and torch's
current stream into the C ABI's plain pointers, allocates output and
workspace tensors of the sizes the library asks for, and raises
``LshError`` with the library's message on any non-OK status.  There is no
other execution path: without the built library every call raises.
"""
from __future__ import annotations

import ctypes as C
import math
import os

import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liblsh.so")

E2LSH, SRP = 0, 1
F32, BF16, FP8 = 0, 1, 2
STATUS = {0: "LSH_OK", -1: "LSH_EINVAL", -2: "LSH_ENOMEM", -3: "LSH_EHIP", -5: "LSH_ERANGE"}

EXPORTS = ("lsh_hash_dense_bf16", "lsh_hash_cs_tables", "lsh_hash_hcs_tables", "lsh_quantize_rows", "lsh_build_check_async", "lsh_hash_workspace_bytes", "lsh_hash_cs", "lsh_hash_cs_noalloc", "lsh_hash_hcs", "lsh_hash_dense",
           "lsh_index_bytes", "lsh_build_workspace_bytes", "lsh_build_index",
           "lsh_index_get_view", "lsh_index_free", "lsh_query", "lsh_query_workspace_bytes",
           "lsh_last_error", "lsh_version")


class LshError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


class Points(C.Structure):
    _fields_ = [("x", C.c_void_p), ("dtype", C.c_int32), ("row_scale", C.c_void_p),
                ("n", C.c_int64), ("d", C.c_int32), ("ld", C.c_int64)]


class Disc(C.Structure):
    _fields_ = [("family", C.c_int32), ("m", C.c_int32), ("K", C.c_int32), ("L", C.c_int32),
                ("w", C.c_float), ("b", C.c_void_p), ("recheck", C.c_int32),
                ("comp_slot", C.c_void_p)]


class Out(C.Structure):
    _fields_ = [("keys", C.c_void_p), ("key_ld", C.c_int64), ("codes", C.c_void_p),
                ("proj", C.c_void_p), ("counters", C.c_void_p)]


class IndexView(C.Structure):
    _fields_ = [("n", C.c_int64), ("L", C.c_int32), ("id_base", C.c_int64),
                ("sorted_ids", C.c_void_p), ("ukeys", C.c_void_p), ("offs", C.c_void_p),
                ("nuniq", C.c_void_p)]


_lib = None


def lib() -> C.CDLL:
    """Load liblsh.so (built in-tree by paper_2503_06737_amd.build); raise if absent."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with "
                              "`python -m paper_2503_06737_amd.build` (there is no fallback)")
        L = C.CDLL(LIB_PATH)
        vp, i32, i64, sz = C.c_void_p, C.c_int32, C.c_int64, C.c_size_t
        L.lsh_hash_workspace_bytes.argtypes = [i32, i32, i32]
        L.lsh_hash_workspace_bytes.restype = sz
        L.lsh_hash_cs.argtypes = [vp, vp, vp, vp, vp, vp, sz, vp]
        L.lsh_hash_cs_noalloc.argtypes = [vp, vp, vp, vp, vp, vp]
        L.lsh_hash_hcs.argtypes = [vp, i32, vp, vp, vp, vp, vp, vp, vp, sz, vp]
        L.lsh_hash_dense.argtypes = [vp, vp, vp, vp, vp]
        L.lsh_hash_cs_tables.argtypes = [vp, vp, vp, vp, vp, vp]
        L.lsh_hash_dense_bf16.argtypes = [vp, vp, i64, vp, vp, vp]
        L.lsh_hash_hcs_tables.argtypes = [vp, i32, vp, vp, vp, vp, vp, vp, vp]
        L.lsh_index_bytes.argtypes = [i64, i32]
        L.lsh_index_bytes.restype = sz
        L.lsh_build_workspace_bytes.argtypes = [i64, i32]
        L.lsh_build_workspace_bytes.restype = sz
        L.lsh_build_index.argtypes = [vp, i64, i64, i32, i64, vp, sz, vp, sz, vp, vp, vp]
        L.lsh_index_get_view.argtypes = [vp, vp]
        L.lsh_index_free.argtypes = [vp]
        L.lsh_index_free.restype = None
        L.lsh_build_check.argtypes = [vp, sz, i64, i32, vp, vp]
        L.lsh_build_check_async.argtypes = [vp, sz, i64, i32, vp, vp]
        L.lsh_quantize_rows.argtypes = [vp, i64, i32, i64, i32, vp, i64, vp, vp]
        L.lsh_query.argtypes = [vp, i32, vp, vp, vp, i64, i32, i64, i32, vp, vp, vp, vp, sz, vp]
        L.lsh_query_workspace_bytes.argtypes = [i64, i32]
        L.lsh_query_workspace_bytes.restype = sz
        L.lsh_last_error.restype = C.c_char_p
        L.lsh_version.restype = i32
        for fn in ("lsh_hash_cs", "lsh_hash_cs_noalloc", "lsh_hash_hcs", "lsh_hash_cs_tables",
                   "lsh_hash_hcs_tables", "lsh_hash_dense_bf16", "lsh_hash_dense", "lsh_build_index",
                   "lsh_index_get_view", "lsh_query", "lsh_build_check", "lsh_build_check_async",
                   "lsh_quantize_rows"):
            getattr(L, fn).restype = i32
        _lib = L
    return _lib


def _check(st: int):
    if st != 0:
        raise LshError(st, lib().lsh_last_error().decode())


def _stream():
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


def points(x: torch.Tensor, scale: torch.Tensor | None = None) -> Points:
    """Describe a 2-D device tensor of points (rows contiguous)."""
    assert x.dim() == 2 and (x.stride(1) == 1 or x.shape[1] == 1), \
        "points must be a row-major 2-D tensor"
    if x.dtype == torch.float32:
        dt = F32
    elif x.dtype in (torch.bfloat16, torch.int16, torch.uint16):
        dt = BF16
    elif x.dtype in (torch.float8_e4m3fn, torch.uint8):
        dt = FP8
    else:
        raise TypeError(f"unsupported point dtype {x.dtype}")
    if scale is not None:
        assert scale.dtype == torch.float32 and scale.is_contiguous()
    return Points(x.data_ptr() if x.numel() else 0, dt, None if scale is None else scale.data_ptr(),
                  x.shape[0], x.shape[1], x.stride(0) if x.shape[0] > 1 else x.shape[1])


def lsh_quantize_rows(x: torch.Tensor, kind: str, q: torch.Tensor | None = None,
                      scale: torch.Tensor | None = None):
    """FP32 rows -> (codes, scale) on the device: kind "bf16" (int16 bit
    patterns) or "fp8" (uint8 bit patterns), one float32 scale per row.
    q / scale may be given (views into resident storage) to write in place."""
    assert x.dtype == torch.float32 and x.dim() == 2 and x.stride(1) == 1
    n, d = x.shape
    dt = {"bf16": BF16, "fp8": FP8}[kind]
    if q is None:
        q = torch.empty((n, d), dtype=torch.int16 if dt == BF16 else torch.uint8, device=x.device)
    if scale is None:
        scale = torch.empty(n, dtype=torch.float32, device=x.device)
    assert q.shape == (n, d) and q.stride(1) == 1 and scale.shape == (n,) and scale.is_contiguous()
    _check(lib().lsh_quantize_rows(_ptr(x), n, d, x.stride(0) if n > 1 else d, dt, _ptr(q),
                                   q.stride(0) if n > 1 else d, _ptr(scale), _stream()))
    return q, scale


def _disc(family, K, L, w, b, recheck, comp_slot=None):
    return Disc(family, K * L, K, L, float(w), None if b is None else b.data_ptr(), int(recheck),
                None if comp_slot is None else comp_slot.data_ptr())


def _outputs(n, m, L, device, keys, codes, proj, counters):
    o = {}
    o["keys"] = torch.empty((L, n), dtype=torch.int64, device=device) if keys else None
    o["codes"] = torch.empty((n, m), dtype=torch.int32, device=device) if codes else None
    o["proj"] = torch.empty((n, m), dtype=torch.float32, device=device) if proj else None
    o["counters"] = counters
    out = Out(_ptr(o["keys"]), n, _ptr(o["codes"]), _ptr(o["proj"]), _ptr(counters))
    return o, out


def _hash_ws(x, m, recheck, ws):
    """The recheck's workspace: the caller's (recheck = 2 reuses the table an
    earlier call built in it) or a new one."""
    wsb = lib().lsh_hash_workspace_bytes(x.shape[1], m, int(recheck))
    if ws is None:
        ws = torch.empty(max(wsb, 1), dtype=torch.uint8, device=x.device)
    elif ws.numel() < wsb:
        raise ValueError(f"hash workspace needs {wsb} bytes, got {ws.numel()}")
    return ws, wsb


def lsh_hash_cs(x, h, s, *, family, K, L, w=1.0, b=None, scale=None, recheck=False, keys=True,
                codes=False, proj=False, counters=None, comp_slot=None, ws=None):
    """CS-E2LSH / CS-SRP of the rows of x.  Returns dict(keys [L][n] int64 bit
    patterns of the u64 keys, codes [n][m], proj [n][m], counters).
    comp_slot: optional [m] device tensor, the code position of each sketch
    component (a permutation of range(m)).  recheck: 0, 1 or 2 (2: reuse the
    recheck table a call with recheck = 1 built in ws for the same h, d, m)."""
    pts = points(x, scale)
    m = K * L
    o, out = _outputs(x.shape[0], m, L, x.device, keys, codes, proj, counters)
    ws, wsb = _hash_ws(x, m, recheck, ws)
    disc = _disc(family, K, L, w, b, recheck, comp_slot)
    _check(lib().lsh_hash_cs(C.byref(pts), _ptr(h), _ptr(s), C.byref(disc), C.byref(out),
                             _ptr(ws), wsb, _stream()))
    return o


def lsh_hash_cs_noalloc(x, h, s, out, *, family, K, L, w=1.0, b=None, scale=None, recheck=False,
                        comp_slot=None):
    """lsh_hash_cs without a workspace: the recheck table lives in the library's
    static device array.  out: dict of caller-allocated device tensors (keys
    [L][n] int64, codes [n][m] int32, proj [n][m] float32, counters [4] int64;
    any may be absent or None); this call allocates nothing."""
    pts = points(x, scale)
    o = {k: out.get(k) for k in ("keys", "codes", "proj", "counters")}
    c = Out(_ptr(o["keys"]), x.shape[0] if o["keys"] is None else o["keys"].stride(0),
            _ptr(o["codes"]), _ptr(o["proj"]), _ptr(o["counters"]))
    disc = _disc(family, K, L, w, b, recheck, comp_slot)
    _check(lib().lsh_hash_cs_noalloc(C.byref(pts), _ptr(h), _ptr(s), C.byref(disc), C.byref(c),
                                     _stream()))
    return o


def lsh_hash_hcs(x, dk, mk, hk, sk, *, family, K, L, w=1.0, b=None, scale=None, recheck=False,
                 keys=True, codes=False, proj=False, counters=None, comp_slot=None, ws=None):
    """HCS-E2LSH / HCS-SRP.  hk/sk: device tensors with the per-mode tables back
    to back; comp_slot as for lsh_hash_cs."""
    pts = points(x, scale)
    m = K * L
    assert math.prod(mk) == m
    o, out = _outputs(x.shape[0], m, L, x.device, keys, codes, proj, counters)
    N = len(dk)
    dka = (C.c_int32 * N)(*dk)
    mka = (C.c_int32 * N)(*mk)
    ws, wsb = _hash_ws(x, m, recheck, ws)
    disc = _disc(family, K, L, w, b, recheck, comp_slot)
    _check(lib().lsh_hash_hcs(C.byref(pts), N, dka, mka, _ptr(hk), _ptr(sk), C.byref(disc),
                              C.byref(out), _ptr(ws), wsb, _stream()))
    return o


def lsh_hash_cs_tables(x, h, s, *, family, K, L, w=1.0, b=None, scale=None, keys=True,
                       codes=False, proj=False, counters=None):
    """Independent per-table count sketches: h, s are [L][d] device tensors
    (table t's bins in [0, K) and signs).  Returns the dict of lsh_hash_cs."""
    pts = points(x, scale)
    o, out = _outputs(x.shape[0], K * L, L, x.device, keys, codes, proj, counters)
    disc = _disc(family, K, L, w, b, 0)
    _check(lib().lsh_hash_cs_tables(C.byref(pts), _ptr(h), _ptr(s), C.byref(disc), C.byref(out),
                                    _stream()))
    return o


def lsh_hash_hcs_tables(x, dk, mk, hk, sk, *, family, K, L, w=1.0, b=None, scale=None,
                        keys=True, codes=False, proj=False, counters=None):
    """Independent per-table higher-order count sketches: hk, sk are
    [L][sum dk] device tensors (table t's per-mode tables back to back)."""
    pts = points(x, scale)
    assert math.prod(mk) == K
    o, out = _outputs(x.shape[0], K * L, L, x.device, keys, codes, proj, counters)
    N = len(dk)
    dka = (C.c_int32 * N)(*dk)
    mka = (C.c_int32 * N)(*mk)
    disc = _disc(family, K, L, w, b, 0)
    _check(lib().lsh_hash_hcs_tables(C.byref(pts), N, dka, mka, _ptr(hk), _ptr(sk),
                                     C.byref(disc), C.byref(out), _stream()))
    return o


def lsh_hash_dense(x, R, *, family, K, L, w=1.0, b=None, keys=True, codes=False, proj=False):
    """Dense E2LSH / SRP (y = x R on FP32 matrix cores)."""
    pts = points(x)
    m = K * L
    o, out = _outputs(x.shape[0], m, L, x.device, keys, codes, proj, None)
    disc = _disc(family, K, L, w, b, 0)
    _check(lib().lsh_hash_dense(C.byref(pts), _ptr(R), C.byref(disc), C.byref(out), _stream()))
    return o


def lsh_hash_dense_bf16(x, scale, Rt, *, family, K, L, w=1.0, b=None, keys=True, codes=False,
                        proj=False):
    """Dense E2LSH / SRP with BF16 operands: x [n][d] BF16 bits (int16) with
    float32 row scales, Rt [m][d] BF16 bits (row l = projection vector r_l)."""
    pts = points(x, scale)
    # (a size-1 dimension's stride is arbitrary: torch keeps the transposed one)
    assert Rt.dim() == 2 and (Rt.stride(1) == 1 or Rt.shape[1] == 1) and Rt.shape[0] == K * L
    o, out = _outputs(x.shape[0], K * L, L, x.device, keys, codes, proj, None)
    disc = _disc(family, K, L, w, b, 0)
    _check(lib().lsh_hash_dense_bf16(C.byref(pts), _ptr(Rt), Rt.stride(0), C.byref(disc),
                                     C.byref(out), _stream()))
    return o


class Index:
    """A built index: its device storage tensor and the library's descriptor."""

    def __init__(self, handle, mem, n, L, id_base, ws=None):
        self.handle, self.mem, self.n, self.L, self.id_base = handle, mem, n, L, id_base
        self.ws = ws  # the build workspace (kept for check())

    def check(self):
        """(big-sort stack overflows, run-head waits given up) of this build:
        both zero unless the build went wrong.  Waits for the build."""
        if self.ws is None:
            raise ValueError("the build workspace was not kept")
        c = (C.c_uint32 * 2)()
        _check(lib().lsh_build_check(_ptr(self.ws), self.ws.numel(), self.n, self.L, c,
                                     _stream()))
        return int(c[0]), int(c[1])

    def check_async(self, counts: torch.Tensor):
        """Enqueue the copy of this build's two consistency counters into
        counts (int32 [2], pinned host or device) on the current stream."""
        if self.ws is None:
            raise ValueError("the build workspace was not kept")
        assert counts.dtype == torch.int32 and counts.numel() == 2 and counts.is_contiguous()
        _check(lib().lsh_build_check_async(_ptr(self.ws), self.ws.numel(), self.n, self.L,
                                           _ptr(counts), _stream()))

    def view(self):
        v = IndexView()
        _check(lib().lsh_index_get_view(self.handle, C.byref(v)))
        return v

    def arrays(self):
        """Device tensors (sorted_ids [L][n], ukeys [L][n], offs [L][n+1], nuniq [L])."""
        n, L = self.n, self.L
        base = self.mem.data_ptr()
        v = self.view()

        def sub(ptr, count, dtype, shape):
            off = ptr - base
            es = torch.empty((), dtype=dtype).element_size()
            return self.mem[off:off + count * es].view(dtype).view(*shape)

        return (sub(v.sorted_ids, L * n, torch.int32, (L, n)),
                sub(v.ukeys, L * n, torch.int64, (L, n)),
                sub(v.offs, L * (n + 1), torch.int32, (L, n + 1)),
                sub(v.nuniq, L, torch.int64, (L,)))

    def __del__(self):
        if getattr(self, "handle", None) and _lib is not None:
            _lib.lsh_index_free(self.handle)
            self.handle = None


def lsh_build_index(keys: torch.Tensor, id_base: int = 0, mem: torch.Tensor | None = None,
                    ws: torch.Tensor | None = None,
                    side_stream: torch.cuda.Stream | None = None) -> Index:
    """Bucket the points of every table.  keys: [L][n] (int64 bit patterns of u64 keys).
    side_stream: a second stream for the heavy-bucket kernels (joined back to
    the current stream), or None to run the whole build on the current stream."""
    L, n = keys.shape
    ib = lib().lsh_index_bytes(n, L)
    wb = lib().lsh_build_workspace_bytes(n, L)
    if mem is None:
        mem = torch.empty(ib, dtype=torch.uint8, device=keys.device)
    if ws is None:
        ws = torch.empty(max(wb, 1), dtype=torch.uint8, device=keys.device)
    h = C.c_void_p()
    _check(lib().lsh_build_index(_ptr(keys) if n else None, keys.stride(0) if n else 0, n, L,
                                 id_base, _ptr(mem), mem.numel(), _ptr(ws), ws.numel(),
                                 C.byref(h), _stream(),
                                 None if side_stream is None else C.c_void_p(side_stream.cuda_stream)))
    return Index(h, mem, n, L, id_base, ws)


# Query workspaces, one per (device, stream): calls on one stream run one
# after another, so they never overlap on theirs.
_QUERY_WS: dict = {}


def _query_ws(dev, stream_ptr: int) -> torch.Tensor:
    key = (str(dev), stream_ptr)
    ws = _QUERY_WS.get(key)
    if ws is None:
        ws = _QUERY_WS[key] = torch.zeros(lib().lsh_query_workspace_bytes(1024, 64),
                                          dtype=torch.uint8, device=dev)
    return ws


def lsh_query(segs, base, Q, qkeys, *, k, watermark=None, metric=E2LSH, base_scale=None,
              q_scale=None, ncand=True, split=True):
    """Top-k of every query row; returns (ids [nq][k] int64, score [nq][k] f32, ncand [nq]).
    split: let a small batch score each query with several workgroups (through
    a workspace kept per device and stream); the answers are the same."""
    segs = list(segs)
    nq = Q.shape[0]
    ids = torch.empty((nq, k), dtype=torch.int64, device=Q.device)
    score = torch.empty((nq, k), dtype=torch.float32, device=Q.device)
    nc = torch.empty(nq, dtype=torch.int32, device=Q.device) if ncand else None
    arr = (C.c_void_p * len(segs))(*[s.handle.value for s in segs])
    pb, pq = points(base, base_scale), points(Q, q_scale)
    wm = (1 << 62) if watermark is None else int(watermark)
    st = _stream()
    ws = _query_ws(Q.device, st.value or 0) if split and 0 < nq <= 1024 else None
    _check(lib().lsh_query(arr, len(segs), C.byref(pb), C.byref(pq), _ptr(qkeys),
                           qkeys.stride(0) if nq else 0, k, wm, metric, _ptr(ids), _ptr(score),
                           _ptr(nc), _ptr(ws), 0 if ws is None else ws.numel(), st))
    return ids, score, nc
