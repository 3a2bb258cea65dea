"""A seeded sweep of random shapes through the whole path, each stage against
the FP64 oracle: the hash (count sketch or higher-order count sketch, E2LSH or
SRP, FP32 / BF16 / FP8-E4M3FN storage, with and without the FP64 recheck),
the index built from the GPU keys (bit-exact), and a top-10 query over it.
The draws reach the kernels' edges: d not a multiple of the 16-byte chunk,
rows longer than one register load (read in pieces), a single point, K other
than 8 and 16, m not a multiple of 64."""
import math

import numpy as np
import pytest

import oracle
from paper_2503_06737_amd import lsh, recall, synth
from gpu_util import compare_hash, dev, to_dev, to_host

pytestmark = pytest.mark.gpu

N_CASES = 64


def _draw(i):
    g = np.random.default_rng([0x5EED, i])
    c = dict(
        n=int(g.choice([1, 2, 31, 33, 257, 1000, 2049, 3001])),
        d=int(g.choice([1, 3, 8, 17, 64, 100, 333, 784, 1024, 1025, 2500, 4096, 5000])),
        family=int(g.integers(0, 2)),
        K=int(g.choice([1, 3, 7, 8, 12, 16, 24, 32])),
        L=int(g.integers(1, 41)),
        storage=str(g.choice(["f32", "bf16", "fp8"])),
        recheck=bool(g.integers(0, 2)),
        hcs=int(g.choice([0, 0, 2, 3])),
        seed=1000 + i,
    )
    c["L"] = max(1, min(c["L"], 2048 // c["K"]))
    return c


def _points(c):
    x = synth.gaussian_clusters(c["n"], c["d"], 5, 0.1, c["seed"])
    if c["storage"] == "f32":
        return x, None, x.astype(np.float64)
    q, sc = synth.quantise_rows(x, c["storage"])
    return q, sc, oracle.decode(q, sc)


def _hash(c, xs, sc, st, x64, recheck):
    """GPU hash of stored rows xs (scale sc) and the oracle's of x64."""
    K, L, fam = c["K"], c["L"], c["family"]
    okw = dict(w=4.0, b=st["b"])
    gkw = dict(family=fam, K=K, L=L, w=4.0, b=to_dev(st["b"]), recheck=recheck, codes=True,
               scale=None if sc is None else to_dev(sc))
    if c["hcs"]:
        ref = oracle.hash_points(x64, fam, K, L, kind="hcs", dk=st["dk"], mk=st["mk"],
                                 hk=st["hk"], sk=st["sk"], **okw)
        out = lsh.lsh_hash_hcs(to_dev(xs), st["dk"], st["mk"], to_dev(np.concatenate(st["hk"])),
                               to_dev(np.concatenate(st["sk"])), proj=not recheck, **gkw)
    else:
        ref = oracle.hash_points(x64, fam, K, L, kind="cs", h=st["h"], s=st["s"], **okw)
        out = lsh.lsh_hash_cs(to_dev(xs), to_dev(st["h"]), to_dev(st["s"]), proj=not recheck,
                              **gkw)
    return out, ref


@pytest.mark.parametrize("i", range(N_CASES))
def test_random_shape_hash_index_query(i):
    dev()
    c = _draw(i)
    n, d, K, L, fam = c["n"], c["d"], c["K"], c["L"], c["family"]
    m = K * L
    print(f"random shape {i}: {c}", flush=True)
    st = {"b": synth.shifts(m, 4.0, c["seed"] + 1)}
    if c["hcs"]:
        st["dk"], st["mk"] = recall.hcs_modes(d, m, c["hcs"])
        st["hk"], st["sk"] = synth.hcs_state(st["dk"], st["mk"], c["seed"] + 2)
        assert math.prod(st["dk"]) >= d and math.prod(st["mk"]) == m
    else:
        st["h"], st["s"] = synth.cs_state(d, m, c["seed"] + 2)
    xs, sc, x64 = _points(c)

    # 1. hash: exact with the recheck, else codes equal outside the near-edge band
    out, ref = _hash(c, xs, sc, st, x64, c["recheck"])
    compare_hash(out, ref, x64, K, L, exact=c["recheck"], what=f"case {i}")

    # 2. index of the GPU keys: bit-exact against the oracle's grouping of the same keys
    keys = to_host(out["keys"], np.uint64)
    ri = oracle.build_index(keys)
    idx = lsh.lsh_build_index(out["keys"])
    assert idx.check() == (0, 0)
    sid, uk, of, nu = idx.arrays()
    assert to_host(nu).tolist() == ri["nuniq"].tolist()
    assert (to_host(sid, np.uint32) == ri["sorted_ids"]).all()
    uk, of = to_host(uk, np.uint64), to_host(of, np.uint32)
    for t in range(L):
        u = int(ri["nuniq"][t])
        assert (uk[t, :u] == ri["ukeys"][t, :u]).all()
        assert (of[t, :u + 1] == ri["offs"][t, :u + 1]).all()

    # 3. query: the first rows as queries (FP32), hashed with the recheck so
    # that their keys are the oracle's; candidates and top-10 over the index
    nq = min(n, 20)
    Q = x64[:nq].astype(np.float32)
    qo, qref = _hash(c, Q, None, st, Q.astype(np.float64), True)
    qk = to_host(qo["keys"], np.uint64)
    assert (qk == qref["keys"]).all()
    base = to_dev(xs)
    ids, sc_g, nc = lsh.lsh_query([idx], base, to_dev(Q), qo["keys"], k=10, metric=fam,
                                  base_scale=None if sc is None else to_dev(sc))
    rids, rsc, rnc = oracle.query([ri], x64, Q.astype(np.float64), qk, 10, n, fam)
    assert (to_host(nc) == rnc).all(), f"case {i}: candidate counts"
    np.testing.assert_allclose(to_host(sc_g), rsc, rtol=1e-5, atol=1e-5)
    gids = to_host(ids)
    for r in range(nq):
        fin = np.isfinite(rsc[r])
        kth = rsc[r][fin][-1] if fin.any() else np.inf
        strict = rsc[r] < kth * (1 - 1e-5) - 1e-5
        assert set(gids[r][strict]) == set(rids[r][strict]), f"case {i}: query {r}"
        assert (gids[r][~fin] == -1).all()


def _draw_tables(i):
    g = np.random.default_rng([0x7AB1E5, i])
    c = dict(
        n=int(g.choice([1, 2, 33, 1000, 3001])),
        d=int(g.choice([1, 5, 17, 64, 300, 784, 1025, 1500])),
        family=int(g.integers(0, 2)),
        K=int(g.choice([1, 2, 3, 4, 7, 8, 12, 16])),
        L=int(g.integers(1, 65)),
        storage=str(g.choice(["f32", "bf16", "fp8"])),
        hcs=int(g.choice([0, 0, 2, 3])),
        seed=5000 + i,
    )
    c["L"] = max(1, min(c["L"], 100_000 // c["d"]))   # the per-table state stays small in LDS
    return c


@pytest.mark.parametrize("i", range(32))
def test_random_shape_per_table_sketches(i):
    """Per-table sketches (L independent sketches of K) at random shapes:
    codes and keys against the oracle's L separate sketches, and the index
    of the GPU keys bit-exact."""
    dev()
    c = _draw_tables(i)
    n, d, K, L, fam = c["n"], c["d"], c["K"], c["L"], c["family"]
    print(f"random per-table shape {i}: {c}", flush=True)
    b = synth.shifts(K * L, 4.0, c["seed"] + 1)
    xs, sc, x64 = _points(c)
    gkw = dict(family=fam, K=K, L=L, w=4.0, b=to_dev(b) if fam == 0 else None, codes=True,
               proj=True, scale=None if sc is None else to_dev(sc))
    if c["hcs"]:
        dk, mk = recall.hcs_modes(d, K, c["hcs"])
        hk, sk = synth.hcs_tables_state(dk, mk, L, c["seed"] + 2)
        splits = np.cumsum(dk)[:-1]
        ref = oracle.hash_points_tables(x64, fam, K, L, kind="hcs", w=4.0, b=b, dk=dk, mk=mk,
                                        hk=[np.split(hk[t], splits) for t in range(L)],
                                        sk=[np.split(sk[t], splits) for t in range(L)])
        out = lsh.lsh_hash_hcs_tables(to_dev(xs), dk, mk, to_dev(hk), to_dev(sk), **gkw)
    else:
        h, s = synth.cs_tables_state(d, K, L, c["seed"] + 2)
        ref = oracle.hash_points_tables(x64, fam, K, L, kind="cs", w=4.0, b=b, h=h, s=s)
        out = lsh.lsh_hash_cs_tables(to_dev(xs), to_dev(h), to_dev(s), **gkw)
    compare_hash(out, ref, x64, K, L, what=f"per-table case {i}")
    keys = to_host(out["keys"], np.uint64)
    ri = oracle.build_index(keys)
    idx = lsh.lsh_build_index(out["keys"])
    assert idx.check() == (0, 0)
    assert (to_host(idx.arrays()[0], np.uint32) == ri["sorted_ids"]).all()


def _draw_dense(i):
    g = np.random.default_rng([0xDE15E, i])
    c = dict(
        n=int(g.choice([1, 2, 127, 129, 1000, 3001])),
        d=int(g.choice([1, 3, 7, 8, 9, 16, 100, 129, 784, 1025])),
        family=int(g.integers(0, 2)),
        K=int(g.choice([1, 3, 7, 8, 12, 16, 24, 32])),
        L=int(g.integers(1, 41)),
        bf16=bool(g.integers(0, 2)),
        seed=9000 + i,
    )
    c["L"] = max(1, min(c["L"], 2048 // c["K"]))
    return c


@pytest.mark.parametrize("i", range(32))
def test_random_shape_dense(i):
    """The dense baselines (FP32 and BF16-operand matrix cores) at random
    shapes, rows and columns off the 128 x 128 tile and d off the 16-value
    step: projections within the dense band, codes equal outside the
    near-edge band, keys equal wherever a table has no near-edge code."""
    dev()
    c = _draw_dense(i)
    n, d, K, L, fam = c["n"], c["d"], c["K"], c["L"], c["family"]
    m = K * L
    print(f"random dense shape {i}: {c}", flush=True)
    x = synth.gaussian_clusters(n, d, 5, 0.1, c["seed"])
    R = synth.gaussian_matrix(d, m, c["seed"] + 1)
    b = synth.shifts(m, 4.0, c["seed"] + 2)
    kw = dict(family=fam, K=K, L=L, w=4.0, b=to_dev(b) if fam == 0 else None, codes=True,
              proj=True)
    if c["bf16"]:
        import torch
        q, sc = synth.quantise_rows(x, "bf16")
        x64 = oracle.decode(q, sc)
        Rb = torch.from_numpy(R).to(torch.bfloat16)
        R = Rb.to(torch.float32).numpy()                    # the BF16 values, exactly
        Rt = Rb.T.contiguous().view(torch.int16).to(dev())  # [m][d] bits
        out = lsh.lsh_hash_dense_bf16(to_dev(q), to_dev(sc), Rt, **kw)
    else:
        x64 = x.astype(np.float64)
        out = lsh.lsh_hash_dense(to_dev(x), to_dev(R), **kw)
    ref = oracle.hash_points(x64, fam, K, L, kind="dense", w=4.0, b=b, R=R)
    compare_hash(out, ref, x64, K, L, weight_max=float(np.abs(R).max()),
                 what=f"dense case {i}")


def _draw_query(i):
    g = np.random.default_rng([0x9E41, i])
    c = dict(
        n=int(g.choice([1, 40, 3000, 9000])),
        d=int(g.choice([1, 3, 17, 64, 200, 960])),
        family=int(g.integers(0, 2)),
        K=int(g.choice([2, 4, 8])),
        L=int(g.choice([1, 3, 8, 16])),
        w=float(g.choice([0.5, 4.0, 64.0])),
        nseg=int(g.integers(1, 5)),
        nq=int(g.choice([1, 7, 300, 1100])),
        k=int(g.choice([1, 3, 10, 33, 64])),
        storage=str(g.choice(["f32", "bf16", "fp8"])),
        seed=12000 + i,
    )
    c["cuts"] = sorted(int(v) for v in g.integers(0, c["n"] + 1, c["nseg"] - 1))
    c["watermark"] = int(g.integers(0, c["n"] + 1))
    if c["w"] >= 64.0 and c["nq"] * c["n"] * c["d"] > 3e8:   # huge buckets: keep the oracle quick
        c["nq"] = 7
    return c


@pytest.mark.parametrize("i", range(32))
def test_random_shape_query(i):
    """Queries at random shapes: 1-4 index segments of contiguous ids (some
    may be empty), a random watermark, batches of 1 to 1100 queries (both
    workgroup shapes), k up to 64, buckets wide enough to need several
    candidate windows, FP32 / BF16 / FP8 bases; candidate counts exact,
    scores and top-k against the FP64 oracle."""
    dev()
    c = _draw_query(i)
    n, d, K, L, fam, w = c["n"], c["d"], c["K"], c["L"], c["family"], c["w"]
    m = K * L
    print(f"random query shape {i}: {c}", flush=True)
    h, s = synth.cs_state(d, m, c["seed"] + 1)
    b = synth.shifts(m, w, c["seed"] + 2)
    hd, sd, bd = to_dev(h), to_dev(s), to_dev(b)
    xs, sc, x64 = _points(c)
    kw = dict(family=fam, K=K, L=L, w=w, b=bd if fam == 0 else None, recheck=True)
    keys = lsh.lsh_hash_cs(to_dev(xs), hd, sd, scale=None if sc is None else to_dev(sc),
                           **kw)["keys"]
    okw = dict(kind="cs", w=w, b=b, h=h, s=s)
    rk = oracle.hash_points(x64, fam, K, L, **okw)["keys"]
    assert (to_host(keys, np.uint64) == rk).all()
    bounds = [0] + c["cuts"] + [n]
    segs, rsegs = [], []
    for lo, hi in zip(bounds[:-1], bounds[1:]):
        segs.append(lsh.lsh_build_index(keys[:, lo:hi].contiguous(), id_base=lo))
        rsegs.append(oracle.build_index(np.ascontiguousarray(rk[:, lo:hi]), lo))
    g = np.random.default_rng([c["seed"], 1])
    own = x64[g.integers(0, n, (c["nq"] + 1) // 2)]
    fresh = synth.gaussian_clusters(c["nq"] // 2, d, 5, 0.1, c["seed"], stream=1)
    Q = np.concatenate([own, fresh.astype(np.float64)]).astype(np.float32)
    qk = lsh.lsh_hash_cs(to_dev(Q), hd, sd, **kw)["keys"]
    rqk = oracle.hash_points(Q.astype(np.float64), fam, K, L, **okw)["keys"]
    assert (to_host(qk, np.uint64) == rqk).all()
    ids, scg, nc = lsh.lsh_query(segs, to_dev(xs), to_dev(Q), qk, k=c["k"],
                                 watermark=c["watermark"], metric=fam,
                                 base_scale=None if sc is None else to_dev(sc))
    rids, rsc, rnc = oracle.query(rsegs, x64, Q.astype(np.float64), rqk, c["k"], c["watermark"],
                                  fam)
    assert (to_host(nc) == rnc).all(), f"case {i}: candidate counts"
    np.testing.assert_allclose(to_host(scg), rsc, rtol=1e-5, atol=1e-5)
    gids = to_host(ids)
    for r in range(Q.shape[0]):
        fin = np.isfinite(rsc[r])
        kth = rsc[r][fin][-1] if fin.any() else np.inf
        strict = rsc[r] < kth * (1 - 1e-5) - 1e-5
        assert set(gids[r][strict]) == set(rids[r][strict]), f"case {i}: query {r}"
        assert (gids[r][~fin] == -1).all()
