"""Indexing quality of the sketched hash families against dense E2LSH / SRP.

Section 6 compares the recall of E2LSH with CS-E2LSH and HCS-E2LSH (and of SRP
with CS-SRP and HCS-SRP) as the number of tables grows, and finds them nearly
identical.  This module repeats that protocol on a synthetic stand-in (the
paper's datasets are not available): clustered points, k = 50 nearest
neighbours, K = 8 components per table, L = 1..50 tables, fresh hash state
per repetition.  Recall of a query = |returned ids ∩ exact top-k| / k, where
the exact top-k is a brute-force FP64 search on the GPU (Euclidean distance
for the E2LSH families, 1 - cos for SRP).  Every hash, index and query call
is the library's.

Two ways of forming the L tables are measured:
  shared     one sketch of m = K·L components per point, split into the L
             tables (this library's design: O(d) work per point for all
             tables together); HCS components are assigned to tables by a
             seeded permutation;
  per_table  L independent sketches of K components, one per table (the
             experiments' protocol: O(L·d) work per point), hashed in one
             pass over the points by lsh_hash_cs_tables / lsh_hash_hcs_tables.

It also reports the bytes of each family's projection state (the space
comparison of Section 6): dense m·d FP32 weights, CS d bins + d signs, HCS
Σ_k d_k bins + signs.

    python -m paper_2503_06737_amd.recall [--reps R] [--L 1,2,4,...] [--nq Q]
"""
from __future__ import annotations

import argparse
import json
import math
import time

import numpy as np
import torch

from . import lsh, synth

FAMILIES = ("dense", "cs", "hcs2", "hcs3")


def hcs_modes(d: int, m: int, N: int):
    """Mode sizes for HCS of order N = 2 or 3: d_k are near-equal powers of
    two with product >= d, and the prime factors of m (largest first) go one
    by one to the mode with the most indices per bin, so the smallest
    d_k / m_k is as large as the totals allow."""
    e = math.ceil(math.log2(d))
    base, extra = divmod(e, N)
    dk = [1 << (base + (1 if i < extra else 0)) for i in range(N)]
    primes, r, p = [], m, 2
    while r > 1:
        while r % p == 0:
            primes.append(p)
            r //= p
        p += 1
    mk = [1] * N
    for f in sorted(primes, reverse=True):
        i = max(range(N), key=lambda k: (dk[k] / mk[k], -mk[k]))
        mk[i] *= f
    assert N in (2, 3) and math.prod(mk) == m and math.prod(dk) >= d
    return dk, mk


def hash_state(fam: str, protocol: str, d: int, K: int, L: int, w: float, seed: int) -> dict:
    """The random state of one repetition, as host arrays (the same arrays the
    oracle takes).  shared: one sketch of m = K L components (a seeded
    permutation assigns the HCS components to tables, so that no table sits
    inside one mode slice); per_table: L independent sketches of K."""
    m = K * L
    st = {"fam": fam, "protocol": protocol, "K": K, "L": L, "w": w,
          "b": synth.shifts(m, w, seed)}
    if fam == "dense":  # independent columns: L tables of K columns are L dense tables
        st["R"] = synth.gaussian_matrix(d, m, seed)
    elif protocol == "shared" and fam == "cs":
        st["h"], st["s"] = synth.cs_state(d, m, seed)
    elif protocol == "shared":
        st["dk"], st["mk"] = hcs_modes(d, m, 2 if fam == "hcs2" else 3)
        hk, sk = synth.hcs_state(st["dk"], st["mk"], seed)
        st["hk"], st["sk"] = np.concatenate(hk), np.concatenate(sk)
        st["slot"] = synth.component_slots(m, seed)
    elif fam == "cs":
        st["h"], st["s"] = synth.cs_tables_state(d, K, L, seed)
    else:
        st["dk"], st["mk"] = hcs_modes(d, K, 2 if fam == "hcs2" else 3)
        st["hk"], st["sk"] = synth.hcs_tables_state(st["dk"], st["mk"], L, seed)
    return st


def table_keys(st: dict, metric: int, dev: str):
    """A function returning the [L][rows] keys of a point set under state st
    (device-resident copies of the state, every hash a library call)."""
    K, L, w = st["K"], st["L"], st["w"]
    t = lambda a: torch.from_numpy(np.ascontiguousarray(
        a.view(np.int32) if a.dtype == np.uint32 else a)).to(dev)
    b = t(st["b"]) if metric == lsh.E2LSH else None
    kw = dict(family=metric, K=K, L=L, w=w, b=b)
    if st["fam"] == "dense":
        R = t(st["R"])
        return lambda A: lsh.lsh_hash_dense(A, R, **kw)["keys"]
    if st["fam"] == "cs":
        h, s = t(st["h"]), t(st["s"])
        if st["protocol"] == "shared":
            return lambda A: lsh.lsh_hash_cs(A, h, s, **kw)["keys"]
        return lambda A: lsh.lsh_hash_cs_tables(A, h, s, **kw)["keys"]
    hk, sk, dk, mk = t(st["hk"]), t(st["sk"]), st["dk"], st["mk"]
    if st["protocol"] == "shared":
        slot = t(st["slot"])
        return lambda A: lsh.lsh_hash_hcs(A, dk, mk, hk, sk, comp_slot=slot, **kw)["keys"]
    return lambda A: lsh.lsh_hash_hcs_tables(A, dk, mk, hk, sk, **kw)["keys"]


def exact_topk(X: torch.Tensor, Q: torch.Tensor, k: int, metric: int) -> torch.Tensor:
    """Brute-force top-k ids per query in FP64 (ties by id)."""
    x, q = X.double(), Q.double()
    if metric == lsh.E2LSH:
        s = (q * q).sum(1, keepdim=True) + (x * x).sum(1)[None, :] - 2.0 * (q @ x.T)
    else:
        xn, qn = x.norm(dim=1), q.norm(dim=1)
        s = 1.0 - (q @ x.T) / (qn[:, None] * xn[None, :]).clamp_min(1e-300)
    # a stable sort keeps equal scores in id order: (score, id) order
    order = torch.argsort(s, dim=1, stable=True)
    return order[:, :k]


def run(nq: int = 100, reps: int = 20, Ls=(1, 2, 4, 8, 16, 32, 50), k: int = 50, K: int = 8,
        w: float = 18.0, dev: str = "cuda", protocols=("shared", "per_table")) -> dict:
    wl = synth.C1
    X = torch.from_numpy(wl.points()).to(dev)
    Q = torch.from_numpy(wl.queries(nq)).to(dev)
    n, d = X.shape
    out = {"workload": wl.name, "n": n, "d": d, "nq": nq, "k": k, "K": K, "w": w,
           "reps": reps, "results": {}, "state_bytes": {}}
    truth = {f: exact_topk(X, Q, k, f) for f in (lsh.E2LSH, lsh.SRP)}
    for protocol in protocols:
        for metric, mname in ((lsh.E2LSH, "e2lsh"), (lsh.SRP, "srp")):
            tk = truth[metric]
            for fam in FAMILIES:
                rows = []
                for L in Ls:
                    rec, qt, cand = [], [], []
                    for r in range(reps):
                        st = hash_state(fam, protocol, d, K, L, w, 7000 + 97 * r + L)
                        keys_of = table_keys(st, metric, dev)
                        idx = lsh.lsh_build_index(keys_of(X))
                        torch.cuda.synchronize()
                        t0 = time.perf_counter()
                        ids, _, nc = lsh.lsh_query([idx], X, Q, keys_of(Q), k=k, metric=metric)
                        torch.cuda.synchronize()
                        qt.append(time.perf_counter() - t0)
                        hit = (ids[:, :, None] == tk[:, None, :]).any(2).sum(1).double() / k
                        rec.append(float(hit.mean()))
                        cand.append(float(nc.double().mean()))
                    rows.append({"L": L, "recall": round(float(np.mean(rec)), 4),
                                 "recall_sd": round(float(np.std(rec)), 4),
                                 "candidates": round(float(np.mean(cand)), 1),
                                 "query_ms": round(1e3 * float(np.median(qt)), 3)})
                out["results"][f"{protocol}/{mname}-{fam}"] = rows
    m = K * max(Ls)
    out["state_bytes"] = {"m": m, "dense": 4 * d * m, "cs": 4 * d + d,
                          "hcs2": sum(hcs_modes(d, m, 2)[0]) * 5,
                          "hcs3": sum(hcs_modes(d, m, 3)[0]) * 5}
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--reps", type=int, default=20)
    ap.add_argument("--nq", type=int, default=100)
    ap.add_argument("--L", default="1,2,4,8,16,32,50")
    ap.add_argument("--w", type=float, default=18.0)
    ap.add_argument("--protocols", default="shared,per_table")
    args = ap.parse_args()
    res = run(nq=args.nq, reps=args.reps, Ls=tuple(int(v) for v in args.L.split(",")), w=args.w,
              protocols=tuple(args.protocols.split(",")))
    print(json.dumps(res))


if __name__ == "__main__":
    main()
