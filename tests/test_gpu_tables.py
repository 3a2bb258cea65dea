"""Independent per-table sketches (lsh_hash_cs_tables / lsh_hash_hcs_tables,
the protocol of Section 6) against the oracle's L separate sketches of K
components each: projections within 1e-5 * ||x||, codes equal outside the
oracle's near-edge band, keys equal wherever a table has no near-edge code.
Shapes span one and several lane groups per table (L = 64, 50, 16, 5), many
rows per wave, ragged d, BF16 / FP8 rows with scales."""
import numpy as np
import pytest
import torch

import oracle
from paper_2503_06737_amd import lsh, synth
from gpu_util import compare_hash, dev, to_dev, to_host

pytestmark = pytest.mark.gpu

CASES = [  # n, d, K, L, data
    (20001, 784, 16, 64, "sparse"),     # the image-like shape, one group
    (5003, 1024, 8, 16, "clusters"),    # the recall protocol's K, four groups
    (3001, 1024, 8, 50, "clusters"),    # L not a power of two
    (777, 37, 3, 5, "clusters"),        # ragged d, odd K
    (1, 64, 4, 4, "clusters"),
]


def _data(n, d, kind, seed):
    if kind == "sparse":
        return synth.sparse_uniform(n, d, 0.2, seed)
    return synth.gaussian_clusters(n, d, 20, 0.1, seed)


@pytest.mark.parametrize("family", [oracle.E2LSH, oracle.SRP])
@pytest.mark.parametrize("n,d,K,L,kind", CASES)
def test_cs_tables_parity(n, d, K, L, kind, family):
    dev()
    x = _data(n, d, kind, 500 + d + L)
    h, s = synth.cs_tables_state(d, K, L, 501)
    b = synth.shifts(K * L, 4.0, 502)
    x64 = x.astype(np.float64)
    ref = oracle.hash_points_tables(x64, family, K, L, kind="cs", w=4.0, b=b, h=h, s=s)
    cnt = to_dev(np.zeros(4, np.uint64))
    out = lsh.lsh_hash_cs_tables(to_dev(x), to_dev(h), to_dev(s), family=family, K=K, L=L,
                                 w=4.0, b=to_dev(b) if family == 0 else None, codes=True,
                                 proj=True, counters=cnt)
    near = compare_hash(out, ref, x64, K, L, what=f"tables n={n} d={d} K={K} L={L}")
    assert to_host(cnt)[3] == 0
    print(f"tables n={n} d={d} K={K} L={L} family={family}: {near} near-edge codes", flush=True)


@pytest.mark.parametrize("family", [oracle.E2LSH, oracle.SRP])
@pytest.mark.parametrize("dk,mk,d,L", [((32, 32), (2, 4), 1024, 12),
                                       ((16, 8, 8), (2, 2, 2), 1000, 20)])
def test_hcs_tables_parity(dk, mk, d, L, family):
    dev()
    K = int(np.prod(mk))
    n = 4001
    x = synth.gaussian_clusters(n, d, 20, 0.1, 510)
    hk, sk = synth.hcs_tables_state(dk, mk, L, 511)
    b = synth.shifts(K * L, 4.0, 512)
    x64 = x.astype(np.float64)
    splits = np.cumsum(dk)[:-1]
    ref = oracle.hash_points_tables(x64, family, K, L, kind="hcs", w=4.0, b=b, dk=dk, mk=mk,
                                    hk=[np.split(hk[t], splits) for t in range(L)],
                                    sk=[np.split(sk[t], splits) for t in range(L)])
    out = lsh.lsh_hash_hcs_tables(to_dev(x), dk, mk, to_dev(hk), to_dev(sk), family=family, K=K,
                                  L=L, w=4.0, b=to_dev(b) if family == 0 else None, codes=True,
                                  proj=True)
    compare_hash(out, ref, x64, K, L, what=f"hcs tables dk={dk}")


@pytest.mark.parametrize("kind", ["bf16", "fp8"])
def test_cs_tables_low_precision(kind):
    dev()
    n, d, K, L = 3000, 2048, 8, 32
    x = synth.gaussian_clusters(n, d, 10, 0.1, 520)
    q, sc = synth.quantise_rows(x, kind)
    x64 = oracle.decode(q, sc)
    h, s = synth.cs_tables_state(d, K, L, 521)
    b = synth.shifts(K * L, 4.0, 522)
    ref = oracle.hash_points_tables(x64, oracle.E2LSH, K, L, kind="cs", w=4.0, b=b, h=h, s=s)
    out = lsh.lsh_hash_cs_tables(to_dev(q), to_dev(h), to_dev(s), family=0, K=K, L=L, w=4.0,
                                 b=to_dev(b), scale=to_dev(sc), codes=True, proj=True)
    compare_hash(out, ref, x64, K, L, what=f"tables {kind}")


def test_one_table_equals_shared_sketch():
    """Special case: L = 1 independent table is the shared sketch of m = K."""
    dev()
    n, d, K = 3000, 500, 16
    x = synth.gaussian_clusters(n, d, 10, 0.1, 530)
    h, s = synth.cs_tables_state(d, K, 1, 531)
    b = synth.shifts(K, 4.0, 532)
    a = lsh.lsh_hash_cs_tables(to_dev(x), to_dev(h), to_dev(s), family=0, K=K, L=1, w=4.0,
                               b=to_dev(b), codes=True)
    c = lsh.lsh_hash_cs(to_dev(x), to_dev(h[0]), to_dev(s[0]), family=0, K=K, L=1, w=4.0,
                        b=to_dev(b), codes=True, recheck=True)
    ref = oracle.hash_points(x.astype(np.float64), 0, K, 1, kind="cs", w=4.0, b=b, h=h[0], s=s[0])
    diff = (to_host(a["codes"]) != to_host(c["codes"])) & ~ref["near"]
    assert not diff.any()
