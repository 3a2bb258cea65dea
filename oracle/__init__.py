"""FP64 CPU oracle for the LSH indexing path -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The product (the HIP library and its
Python binding) never does.  The arithmetic lives in ``lsh_oracle.c`` (plain
C, FP64, no floating-point contraction); this module marshals NumPy arrays
through ctypes and strings the steps together in the paper's order:
project (count sketch / higher-order count sketch / dense), discretise
(E2LSH floor or SRP sign), concatenate K codes per table into a bucket key,
group the points by key per table, and answer queries by the union of the
probed buckets re-ranked by exact distance.

Parity pins for every function here are in ``tests/test_oracle_pins.py``.
"""
from __future__ import annotations

import ctypes as C
import math
import os

import numpy as np

from .build import LIB_PATH, build as _build

E2LSH, SRP = 0, 1
F32, BF16, FP8 = 0, 1, 2

_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            _build()
        _lib = C.CDLL(LIB_PATH)
        _declare(_lib)
    return _lib


def _p(a):
    return a.ctypes.data_as(C.c_void_p)


def _declare(L):
    vp, i64, i32, f32, f64 = C.c_void_p, C.c_int64, C.c_int32, C.c_float, C.c_double
    L.orc_decode.argtypes = [vp, C.c_int, vp, i64, i32, i64, vp]
    L.orc_quantise_rows.argtypes = [vp, i64, i32, C.c_int, vp, vp]
    L.orc_cs_sketch.argtypes = [vp, i64, i32, vp, vp, i32, vp]
    L.orc_hcs_sketch.argtypes = [vp, i64, i32, i32, vp, vp, vp, vp, vp]
    L.orc_dense_proj.argtypes = [vp, i64, i32, vp, i32, vp]
    L.orc_disc_e2lsh.argtypes = [vp, i64, i32, vp, f32, f64, vp, vp]
    L.orc_disc_srp.argtypes = [vp, vp, i64, i32, vp, vp]
    L.orc_row_norms.argtypes = [vp, i64, i32, vp]
    L.orc_assign_components.argtypes = [vp, i64, i32, vp, vp]
    L.orc_keys_e2lsh.argtypes = [vp, i64, i32, i32, i32, vp]
    L.orc_keys_srp.argtypes = [vp, i64, i32, i32, i32, vp]
    L.orc_set_threads.argtypes = [C.c_int]
    L.orc_max_threads.restype = C.c_int
    L.orc_mix64.argtypes = [C.c_uint64]
    L.orc_mix64.restype = C.c_uint64
    L.orc_fp8_e4m3fn_value.argtypes = [C.c_uint8]
    L.orc_fp8_e4m3fn_value.restype = f64
    L.orc_build_index.argtypes = [vp, i64, i32, i64, vp, vp, vp, vp, vp]
    L.orc_query_one.argtypes = [i32, vp, i32, vp, vp, vp, vp, vp, i32, vp, vp, i64, i32, i64,
                                C.c_int, vp, vp]
    L.orc_query_one.restype = i64


# ----------------------------------------------------------------------------
# step 1: decode
# ----------------------------------------------------------------------------

def decode(q: np.ndarray, scale: np.ndarray | None = None) -> np.ndarray:
    """Stored values -> FP64: float32 as is; uint16 = BF16 bits; uint8 = FP8-E4M3FN bits."""
    q = np.ascontiguousarray(q)
    n, d = q.shape
    if q.dtype == np.float32:
        dt = F32
    elif q.dtype == np.uint16:
        dt = BF16
    elif q.dtype == np.uint8:
        dt = FP8
    else:
        raise TypeError(q.dtype)
    sc = None if scale is None else np.ascontiguousarray(scale, dtype=np.float32)
    x = np.empty((n, d), np.float64)
    lib().orc_decode(_p(q), dt, None if sc is None else _p(sc), n, d, d, _p(x))
    return x


def quantise_rows(x: np.ndarray, kind: str):
    """FP32 rows -> (codes, scale): BF16 (uint16 bits, scale = max|x|) or
    FP8-E4M3FN (uint8 bits, scale = max|x| / 448); each value x / scale
    rounded to the nearest code, ties to even (the low-precision storage)."""
    x = np.ascontiguousarray(x, np.float32)
    n, d = x.shape
    dt = {"bf16": BF16, "fp8": FP8}[kind]
    q = np.empty((n, d), np.uint16 if dt == BF16 else np.uint8)
    sc = np.empty(n, np.float32)
    lib().orc_quantise_rows(_p(x), n, d, dt, _p(q), _p(sc))
    return q, sc


def set_threads(n: int) -> None:
    """OpenMP threads the oracle's loops use from now on."""
    lib().orc_set_threads(int(n))


def max_threads() -> int:
    return int(lib().orc_max_threads())


def fp8_value(bits: int) -> float:
    return lib().orc_fp8_e4m3fn_value(bits)


def mix64(z: int) -> int:
    return lib().orc_mix64(z & 0xFFFFFFFFFFFFFFFF)


# ----------------------------------------------------------------------------
# step 2: projections
# ----------------------------------------------------------------------------

def cs_sketch(x: np.ndarray, h: np.ndarray, s: np.ndarray, m: int) -> np.ndarray:
    x = np.ascontiguousarray(x, np.float64)
    n, d = x.shape
    h = np.ascontiguousarray(h, np.uint32)
    s = np.ascontiguousarray(s, np.int8)
    assert h.shape == (d,) and s.shape == (d,) and (h < m).all()
    y = np.empty((n, m), np.float64)
    lib().orc_cs_sketch(_p(x), n, d, _p(h), _p(s), m, _p(y))
    return y


def hcs_sketch(x: np.ndarray, dk, mk, hk, sk) -> np.ndarray:
    x = np.ascontiguousarray(x, np.float64)
    n, d = x.shape
    N = len(dk)
    assert int(np.prod(dk)) >= d
    dk_a = np.ascontiguousarray(dk, np.int32)
    mk_a = np.ascontiguousarray(mk, np.int32)
    hk_a = np.ascontiguousarray(np.concatenate([np.asarray(a, np.uint32) for a in hk]))
    sk_a = np.ascontiguousarray(np.concatenate([np.asarray(a, np.int8) for a in sk]))
    m = int(np.prod(mk))
    y = np.empty((n, m), np.float64)
    lib().orc_hcs_sketch(_p(x), n, d, N, _p(dk_a), _p(mk_a), _p(hk_a), _p(sk_a), _p(y))
    return y


def dense_proj(x: np.ndarray, R: np.ndarray) -> np.ndarray:
    x = np.ascontiguousarray(x, np.float64)
    R = np.ascontiguousarray(R, np.float32)
    n, d = x.shape
    m = R.shape[1]
    y = np.empty((n, m), np.float64)
    lib().orc_dense_proj(_p(x), n, d, _p(R), m, _p(y))
    return y


def assign_components(y: np.ndarray, slot: np.ndarray) -> np.ndarray:
    """Code position slot[l] receives sketch component l (a permutation of range(m))."""
    y = np.ascontiguousarray(y, np.float64)
    n, m = y.shape
    slot = np.ascontiguousarray(slot, np.uint32)
    assert slot.shape == (m,) and (slot < m).all()
    out = np.empty((n, m), np.float64)
    lib().orc_assign_components(_p(y), n, m, _p(slot), _p(out))
    return out


def row_norms(x: np.ndarray) -> np.ndarray:
    x = np.ascontiguousarray(x, np.float64)
    out = np.empty(x.shape[0], np.float64)
    lib().orc_row_norms(_p(x), x.shape[0], x.shape[1], _p(out))
    return out


# ----------------------------------------------------------------------------
# step 3: discretise
# ----------------------------------------------------------------------------

def disc_e2lsh(y: np.ndarray, b: np.ndarray, w: float, alpha: float):
    y = np.ascontiguousarray(y, np.float64)
    n, m = y.shape
    b = np.ascontiguousarray(b, np.float32)
    codes = np.empty((n, m), np.int32)
    near = np.empty((n, m), np.uint8)
    lib().orc_disc_e2lsh(_p(y), n, m, _p(b), float(w), float(alpha), _p(codes), _p(near))
    return codes, near.astype(bool)


def disc_srp(y: np.ndarray, xnorm: np.ndarray):
    y = np.ascontiguousarray(y, np.float64)
    n, m = y.shape
    xnorm = np.ascontiguousarray(xnorm, np.float64)
    bits = np.empty((n, m), np.int32)
    near = np.empty((n, m), np.uint8)
    lib().orc_disc_srp(_p(y), _p(xnorm), n, m, _p(bits), _p(near))
    return bits, near.astype(bool)


# ----------------------------------------------------------------------------
# step 4: keys
# ----------------------------------------------------------------------------

def keys_e2lsh(codes: np.ndarray, K: int, L: int) -> np.ndarray:
    codes = np.ascontiguousarray(codes, np.int32)
    n, m = codes.shape
    assert K * L <= m
    keys = np.empty((L, n), np.uint64)
    lib().orc_keys_e2lsh(_p(codes), n, m, K, L, _p(keys))
    return keys


def keys_srp(bits: np.ndarray, K: int, L: int) -> np.ndarray:
    bits = np.ascontiguousarray(bits, np.int32)
    n, m = bits.shape
    assert K * L <= m and K <= 64
    keys = np.empty((L, n), np.uint64)
    lib().orc_keys_srp(_p(bits), n, m, K, L, _p(keys))
    return keys


# ----------------------------------------------------------------------------
# steps 2-4 together
# ----------------------------------------------------------------------------

def hash_points(x: np.ndarray, family: int, K: int, L: int, *, kind: str, w: float = 1.0,
                b: np.ndarray | None = None, h=None, s=None, m: int | None = None, dk=None,
                mk=None, hk=None, sk=None, R=None, comp_slot=None) -> dict:
    """Project (kind in {"cs", "hcs", "dense"}), assign the components to code
    positions (comp_slot, identity when None), discretise and key FP64 points x.

    Returns y (projection before scaling, in code-position order), codes
    (E2LSH codes or SRP bits), near (near-edge flags), keys [L][n].
    """
    x = np.ascontiguousarray(x, np.float64)
    if kind == "cs":
        y = cs_sketch(x, h, s, K * L if m is None else m)
    elif kind == "hcs":
        y = hcs_sketch(x, dk, mk, hk, sk)
    elif kind == "dense":
        y = dense_proj(x, R)
    else:
        raise ValueError(kind)
    if comp_slot is not None:
        y = assign_components(y, comp_slot)
    m = y.shape[1]
    if family == E2LSH:
        alpha = 1.0 if kind == "dense" else math.sqrt(m)
        codes, near = disc_e2lsh(y, b, w, alpha)
        keys = keys_e2lsh(codes, K, L)
    else:
        codes, near = disc_srp(y, row_norms(x))
        keys = keys_srp(codes, K, L)
    return {"y": y, "codes": codes, "near": near, "keys": keys}


# ----------------------------------------------------------------------------
# step 5: index
# ----------------------------------------------------------------------------

def hash_points_tables(x: np.ndarray, family: int, K: int, L: int, *, kind: str,
                       w: float = 1.0, b: np.ndarray | None = None, h=None, s=None, dk=None,
                       mk=None, hk=None, sk=None) -> dict:
    """Independent tables, the protocol of Section 6: table t has a sketch of
    its own with K components (kind "cs": h[t], s[t] over the d coordinates;
    kind "hcs": per-mode tables hk[t][k], sk[t][k] with prod mk = K),
    discretised with scale sqrt(K) (the sketch length, Definition
    CS_Eucl_LSH) and shifts b[tK:(t+1)K]; its K codes form its key.

    Returns y [n][K L] (table t at columns tK..tK+K-1), codes, near, keys [L][n].
    """
    x = np.ascontiguousarray(x, np.float64)
    ys = []
    for t in range(L):
        if kind == "cs":
            ys.append(cs_sketch(x, h[t], s[t], K))
        elif kind == "hcs":
            assert int(np.prod(mk)) == K
            ys.append(hcs_sketch(x, dk, mk, hk[t], sk[t]))
        else:
            raise ValueError(kind)
    y = np.ascontiguousarray(np.concatenate(ys, axis=1))
    if family == E2LSH:
        codes, near = disc_e2lsh(y, b, w, math.sqrt(K))
        keys = keys_e2lsh(codes, K, L)
    else:
        codes, near = disc_srp(y, row_norms(x))
        keys = keys_srp(codes, K, L)
    return {"y": y, "codes": codes, "near": near, "keys": keys}


def build_index(keys: np.ndarray, id_base: int = 0) -> dict:
    keys = np.ascontiguousarray(keys, np.uint64)
    L, n = keys.shape
    sorted_ids = np.empty((L, n), np.uint32)
    sorted_keys = np.empty((L, n), np.uint64)
    ukeys = np.zeros((L, n), np.uint64)
    offs = np.zeros((L, n + 1), np.uint32)
    nuniq = np.zeros(L, np.int64)
    lib().orc_build_index(_p(keys), n, L, id_base, _p(sorted_ids), _p(sorted_keys), _p(ukeys),
                          _p(offs), _p(nuniq))
    return {"n": n, "L": L, "id_base": id_base, "sorted_ids": sorted_ids,
            "sorted_keys": sorted_keys, "ukeys": ukeys, "offs": offs, "nuniq": nuniq}


# ----------------------------------------------------------------------------
# step 6: query
# ----------------------------------------------------------------------------

def query(segments: list, base: np.ndarray, Q: np.ndarray, qkeys: np.ndarray, k: int,
          watermark: int, metric: int):
    """Union-of-buckets candidates, exact FP64 re-rank, top-k by (score, id).

    segments: dicts from build_index; base: FP64 points by global id;
    Q: FP64 queries [nq][d]; qkeys: [L][nq].  Returns ids [nq][k] int64,
    scores [nq][k] float64, ncand [nq] int64.
    """
    base = np.ascontiguousarray(base, np.float64)
    Q = np.ascontiguousarray(Q, np.float64)
    qkeys = np.ascontiguousarray(qkeys, np.uint64)
    L, nq = qkeys.shape
    d = base.shape[1]
    nseg = len(segments)
    seg_n = np.array([s["n"] for s in segments], np.int64)
    arrs = {f: [np.ascontiguousarray(s[f]) for s in segments]
            for f in ("sorted_ids", "ukeys", "offs", "nuniq")}
    ptrs = {f: (C.c_void_p * max(1, nseg))(*[a.ctypes.data for a in arrs[f]]) for f in arrs}
    ids = np.empty((nq, k), np.int64)
    sc = np.empty((nq, k), np.float64)
    nc = np.empty(nq, np.int64)
    for i in range(nq):
        qrow = Q[i]
        out_i = ids[i]
        out_s = sc[i]
        nc[i] = lib().orc_query_one(nseg, _p(seg_n), L, ptrs["sorted_ids"], ptrs["ukeys"],
                                    ptrs["offs"], ptrs["nuniq"], _p(base), d, _p(qrow),
                                    qkeys[:, i:].ctypes.data_as(C.c_void_p), nq, k, watermark,
                                    metric, _p(out_i), _p(out_s))
    return ids, sc, nc
