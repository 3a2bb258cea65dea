"""Parity of the timed hash call at full size.

The benchmark hashes with keys only (no codes, no projection, no recheck) and
a grid capped at what the GPU holds at once, so each workgroup loops over many
32-row blocks: the next block's first row is prefetched across the block
boundary and the LDS key staging is reused after barriers.  These tests run
exactly that call on enough rows that every workgroup takes several blocks
(n well above 32 rows x the resident workgroups), compare every key with the
FP64 oracle's (a table whose K codes include an oracle near-edge component,
|v - w round(v/w)| < 1e-4 w or |y| < 1e-6 ||x||, is exempt and counted), then
build the index from the GPU keys as the benchmark does and compare it
bit-exactly with the oracle's index of the same keys (Section 3.1: every
point in the bucket of its key, per table).
"""
import numpy as np
import pytest
import torch

import oracle
from paper_2503_06737_amd import lsh, synth
from gpu_util import dev, to_dev, to_host

pytestmark = pytest.mark.gpu


def _oracle_keys(x, family, K, L, chunk=50_000, **kw):
    """Oracle keys [L][n] and per-table near-edge flags, hashed in row chunks."""
    n = x.shape[0]
    scale = kw.pop("scale_all", None)   # low-precision codes: decode with the row scales
    keys = np.empty((L, n), np.uint64)
    tab_near = np.zeros((L, n), bool)
    for lo in range(0, n, chunk):
        xs = x[lo:lo + chunk]
        x64 = xs.astype(np.float64) if scale is None else oracle.decode(xs, scale[lo:lo + chunk])
        out = oracle.hash_points(x64, family, K, L, **kw)
        keys[:, lo:lo + chunk] = out["keys"]
        tab_near[:, lo:lo + chunk] = out["near"].reshape(-1, L, K).any(axis=2).T
    return keys, tab_near


def _check_keys(kg, rk, tab_near, what):
    diff = kg != rk
    outside = diff & ~tab_near
    assert not outside.any(), (f"{what}: {int(outside.sum())} keys differ outside the near-edge "
                               f"band, first (table, row) {np.argwhere(outside)[:3].tolist()}")
    print(f"{what}: {int(diff.sum())} keys differ, all in {int(tab_near.sum())} exempt "
          f"(table, row) pairs", flush=True)


def _check_index(keys_dev, kg, what):
    """Index of the GPU keys (caller memory, as timed) == oracle index of the same keys."""
    L, n = keys_dev.shape
    mem = torch.empty(lsh.lib().lsh_index_bytes(n, L), dtype=torch.uint8, device=keys_dev.device)
    ws = torch.empty(lsh.lib().lsh_build_workspace_bytes(n, L), dtype=torch.uint8,
                     device=keys_dev.device)
    idx = lsh.lsh_build_index(keys_dev, mem=mem, ws=ws)
    assert idx.check() == (0, 0), what
    ref = oracle.build_index(kg)
    sid, uk, of, nu = idx.arrays()
    nu = to_host(nu)
    assert (nu == ref["nuniq"]).all(), f"{what}: distinct key counts"
    assert (to_host(sid, np.uint32) == ref["sorted_ids"]).all(), f"{what}: sorted ids"
    uk, of = to_host(uk, np.uint64), to_host(of, np.uint32)
    for t in range(L):
        u = int(nu[t])
        assert (uk[t, :u] == ref["ukeys"][t, :u]).all(), f"{what}: ukeys of table {t}"
        assert (of[t, :u + 1] == ref["offs"][t, :u + 1]).all(), f"{what}: offsets of table {t}"


CS_CASES = [
    # name, n, d, K, L, data, w
    ("image-like d784 m1024", 100_003, 784, 16, 64, "sparse", 4.0),
    ("clusters d1024 m128 (K=8)", 200_001, 1024, 8, 16, "clusters", 4.0),
    ("clusters d1024 non-narrow rows", 100_001, 1024, 8, 16, "clusters", 0.25),
    ("clusters d256 K=12", 300_007, 256, 12, 8, "clusters", 4.0),
    ("clusters d784 K=32 (SRP words)", 100_003, 784, 32, 16, "clusters", 4.0),
]


@pytest.mark.parametrize("family", [oracle.E2LSH, oracle.SRP])
@pytest.mark.parametrize("name,n,d,K,L,data,w", CS_CASES)
def test_keys_only_many_blocks_per_workgroup(name, n, d, K, L, data, w, family):
    dev()
    what = f"{name} fam={family} n={n}"
    print(f"case {what}", flush=True)
    m = K * L
    if data == "sparse":
        x = synth.sparse_uniform(n, d, 0.2, 9000 + d)
    else:
        x = synth.gaussian_clusters(n, d, 50, 0.1, 9000 + d)
    h, s = synth.cs_state(d, m, 9001 + d)
    b = synth.shifts(m, w, 9002 + d)
    xd = to_dev(x)
    out = lsh.lsh_hash_cs(xd, to_dev(h), to_dev(s), family=family, K=K, L=L, w=w, b=to_dev(b))
    kg = to_host(out["keys"], np.uint64)
    rk, tab_near = _oracle_keys(x, family, K, L, kind="cs", w=w, b=b, h=h, s=s)
    _check_keys(kg, rk, tab_near, what)
    del xd
    _check_index(out["keys"], kg, what)


@pytest.mark.parametrize("family", [oracle.E2LSH, oracle.SRP])
@pytest.mark.parametrize("dk,mk", [((64, 64), (32, 32)), ((16, 16, 16), (8, 8, 16))])
def test_hcs_keys_only_many_blocks(dk, mk, family):
    """HCS at the 4096-dimensional tensor-reshape shape, keys only."""
    dev()
    n, d, K, L = 60_001, 4096, 16, 64
    what = f"hcs {dk} fam={family} n={n}"
    print(f"case {what}", flush=True)
    x = synth.gaussian_clusters(n, d, 200, 0.2, 9100)
    hk, sk = synth.hcs_state(dk, mk, 9101)
    b = synth.shifts(K * L, 4.0, 9102)
    out = lsh.lsh_hash_hcs(to_dev(x), dk, mk, to_dev(np.concatenate(hk)),
                           to_dev(np.concatenate(sk)), family=family, K=K, L=L, w=4.0,
                           b=to_dev(b))
    kg = to_host(out["keys"], np.uint64)
    rk, tab_near = _oracle_keys(x, family, K, L, chunk=20_000, kind="hcs", w=4.0, b=b, dk=dk,
                                mk=mk, hk=hk, sk=sk)
    _check_keys(kg, rk, tab_near, what)
    _check_index(out["keys"], kg, what)


@pytest.mark.parametrize("kind", ["bf16", "fp8"])
def test_low_precision_long_rows_many_blocks(kind):
    """d = 16384 stored BF16 / FP8 with row scales (rows read in pieces), with
    and without the FP64 recheck: with it every key equals the oracle's on the
    dequantised points."""
    dev()
    n, d, K, L = 40_003, 16384, 16, 32
    what = f"{kind} d={d} n={n}"
    print(f"case {what}", flush=True)
    x = synth.gaussian_clusters(n, d, 50, 0.1, 9200)
    q, sc = synth.quantise_rows(x, kind)
    del x
    h, s = synth.cs_state(d, K * L, 9201)
    b = synth.shifts(K * L, 4.0, 9202)
    qd, scd = to_dev(q), to_dev(sc)
    kw = dict(family=oracle.E2LSH, K=K, L=L, w=4.0, b=to_dev(b), scale=scd)
    fast = to_host(lsh.lsh_hash_cs(qd, to_dev(h), to_dev(s), **kw)["keys"], np.uint64)
    cnt = to_dev(np.zeros(4, np.uint64))
    exact = lsh.lsh_hash_cs(qd, to_dev(h), to_dev(s), recheck=True, counters=cnt, **kw)["keys"]
    rk, tab_near = _oracle_keys(q, oracle.E2LSH, K, L, chunk=10_000, kind="cs", w=4.0, b=b, h=h,
                                s=s, scale_all=sc)
    _check_keys(fast, rk, tab_near, what + " fast")
    assert (to_host(exact, np.uint64) == rk).all(), f"{what}: recheck keys differ"
    c = to_host(cnt, np.uint64)
    assert c[1] <= c[0] and c[2] == 0
    _check_index(exact, rk, what)


def test_headline_workload_full():
    """The benchmark's own workload and call: 1,000,000 image-like rows,
    d = 784, K = 16, L = 64, w = 4, CS-E2LSH keys only, then the index build
    in caller memory."""
    dev()
    wl = synth.C2
    print(f"case {wl.name} full", flush=True)
    x = wl.points()
    h, s = wl.cs()
    b = wl.b()
    xd = to_dev(x)
    out = lsh.lsh_hash_cs(xd, to_dev(h), to_dev(s), family=oracle.E2LSH, K=wl.K, L=wl.L, w=wl.w,
                          b=to_dev(b))
    kg = to_host(out["keys"], np.uint64)
    del xd
    rk, tab_near = _oracle_keys(x, oracle.E2LSH, wl.K, wl.L, chunk=100_000, kind="cs", w=wl.w,
                                b=b, h=h, s=s)
    del x
    _check_keys(kg, rk, tab_near, wl.name)
    _check_index(out["keys"], kg, wl.name)
