"""GPU parity of CS / HCS / dense hashing against the FP64 oracle, through the
C ABI.  Inputs are seeded and shaped like the paper's workloads (Section 6):
Gaussian clusters, sparse image-like rows, tensor reshapes for HCS."""
import math

import numpy as np
import pytest

import oracle
from paper_2503_06737_amd import lsh, synth
from gpu_util import compare_hash, dev, to_dev, to_host

pytestmark = pytest.mark.gpu


def _cs_case(n, d, K, L, data, seed):
    m = K * L
    if data == "clusters":
        x = synth.gaussian_clusters(n, d, 20, 0.1, seed)
    else:
        x = synth.sparse_uniform(n, d, 0.2, seed)
    h, s = synth.cs_state(d, m, seed + 1)
    b = synth.shifts(m, 4.0, seed + 1)
    return x, h, s, b


CS_CASES = [
    # n, d, K, L, data        (several row blocks and workgroups, ragged tails)
    (10000, 1024, 8, 16, "clusters"),   # the n=10k, d=1024, m=128 workload
    (2003, 784, 16, 64, "sparse"),      # the d=784, m=1024 image-like shape, ragged n
    (777, 960, 16, 32, "clusters"),     # d=960, m=512
    (501, 37, 5, 3, "clusters"),        # d not a multiple of 4: scalar-load path, odd m
    (1, 64, 4, 4, "clusters"),          # a single point
    (65, 4096, 16, 64, "clusters"),     # long row: read in 4 pieces
    (300, 2500, 8, 16, "clusters"),     # long row: 3 pieces, rounded up to 4
    (257, 1301, 8, 8, "sparse"),        # long unaligned row (scalar loads, 4 pieces)
]


@pytest.mark.parametrize("family", [oracle.E2LSH, oracle.SRP])
@pytest.mark.parametrize("d", [4096, 1301])
def test_long_rows_growing_magnitude_recheck_exact(d, family):
    """Long rows whose magnitude grows along the row: every later piece raises
    the exponent, so the bins are shifted several times per row.  The FP64
    recheck must still reproduce the oracle exactly, and without it the
    projection stays within 1e-5 * ||x||.  (The fast path's codes are the
    FP32 evaluation: with |sqrt(m) y| near 1e6 its error exceeds the oracle's
    fixed 1e-4 * w near-edge band; the counting test below checks that the
    fast path counts them.)"""
    dev()
    n, K, L = 400, 16, 32
    g = np.random.default_rng(5)
    x = (g.standard_normal((n, d)) * np.exp2(np.arange(d) // 1024 * 5.0)).astype(np.float32)
    h, s = synth.cs_state(d, K * L, 6)
    b = synth.shifts(K * L, 4.0, 6)
    x64 = x.astype(np.float64)
    ref = oracle.hash_points(x64, family, K, L, kind="cs", w=4.0, b=b, h=h, s=s)
    kw = dict(family=family, K=K, L=L, w=4.0, b=to_dev(b), codes=True)
    cnt = to_dev(np.zeros(4, np.uint64))
    out = lsh.lsh_hash_cs(to_dev(x), to_dev(h), to_dev(s), recheck=True, counters=cnt, **kw)
    compare_hash(out, ref, x64, K, L, exact=True, what=f"growing d={d} recheck")
    kw.update(codes=False, keys=False)
    out = lsh.lsh_hash_cs(to_dev(x), to_dev(h), to_dev(s), proj=True, **kw)
    compare_hash(out, ref, x64, K, L, what=f"growing d={d}")


@pytest.mark.parametrize("family", [oracle.E2LSH, oracle.SRP])
@pytest.mark.parametrize("growing", [False, True])
def test_fast_path_counts_its_uncertain_components(family, growing):
    """Without the recheck, counters[0] counts the components whose FP32 value
    lies within the fast path's error bound of a bin edge (E2LSH) or of zero
    (SRP).  Every code that differs from the FP64 oracle's must be one of
    them, so the mismatches never outnumber the count, and every value beyond
    2^23 is counted.  Rows whose magnitude grows along the row make the FP32
    codes wrong in places."""
    dev()
    n, K, L = 400, 16, 32
    m = K * L
    if growing:
        d = 4096
        g = np.random.default_rng(8)
        x = (g.standard_normal((n, d)) * np.exp2(np.arange(d) // 1024 * 5.0)).astype(np.float32)
        h, s = synth.cs_state(d, m, 9)
        b = synth.shifts(m, 4.0, 9)
    else:
        d = 784
        x, h, s, b = _cs_case(n, d, K, L, "sparse", 91)
    x64 = x.astype(np.float64)
    ref = oracle.hash_points(x64, family, K, L, kind="cs", w=4.0, b=b, h=h, s=s)
    cnt = to_dev(np.zeros(4, np.uint64))
    out = lsh.lsh_hash_cs(to_dev(x), to_dev(h), to_dev(s), family=family, K=K, L=L, w=4.0,
                          b=to_dev(b), codes=True, counters=cnt)
    c = to_host(cnt, np.uint64)
    diff = int((to_host(out["codes"]) != ref["codes"]).sum())
    assert diff <= int(c[0]), (diff, c)
    if family == oracle.E2LSH:
        v = (math.sqrt(m) * ref["y"] + b) / 4.0
        huge = int((np.abs(v) >= 2.0 ** 23).sum())
        assert int(c[0]) >= huge
    if growing and family == oracle.E2LSH:
        assert diff > 0     # the case does reach codes the FP32 path gets wrong
    if family == oracle.E2LSH and not growing:
        assert int(c[0]) < n * m // 100     # ordinary rows: a small fraction is uncertain
    if family == oracle.SRP:
        # a component whose coordinates are all zero sums to exactly 0, which
        # the bound cannot tell from a sum truncated to 0: it is counted
        assert int(c[0]) >= int((ref["y"] == 0).sum())
    # the same call without counters gives the same codes
    again = lsh.lsh_hash_cs(to_dev(x), to_dev(h), to_dev(s), family=family, K=K, L=L, w=4.0,
                            b=to_dev(b), codes=True)
    assert (to_host(again["codes"]) == to_host(out["codes"])).all()


@pytest.mark.parametrize("family", [oracle.E2LSH, oracle.SRP])
@pytest.mark.parametrize("n,d,K,L,data", CS_CASES)
def test_cs_hash_parity(n, d, K, L, data, family):
    dev()
    x, h, s, b = _cs_case(n, d, K, L, data, 1234 + d)
    x64 = x.astype(np.float64)
    ref = oracle.hash_points(x64, family, K, L, kind="cs", w=4.0, b=b, h=h, s=s)
    out = lsh.lsh_hash_cs(to_dev(x), to_dev(h), to_dev(s), family=family, K=K, L=L, w=4.0,
                          b=to_dev(b), codes=True, proj=True)
    compare_hash(out, ref, x64, K, L, what=f"cs n={n} d={d}")


@pytest.mark.parametrize("family", [oracle.E2LSH, oracle.SRP])
def test_cs_hash_recheck_is_exact(family):
    """With the FP64 recheck every code and key equals the FP64 oracle's."""
    dev()
    n, d, K, L = 3001, 784, 16, 64
    x, h, s, b = _cs_case(n, d, K, L, "sparse", 77)
    x64 = x.astype(np.float64)
    ref = oracle.hash_points(x64, family, K, L, kind="cs", w=4.0, b=b, h=h, s=s)
    cnt = to_dev(np.zeros(4, np.uint64))
    out = lsh.lsh_hash_cs(to_dev(x), to_dev(h), to_dev(s), family=family, K=K, L=L, w=4.0,
                          b=to_dev(b), codes=True, proj=True, recheck=True, counters=cnt)
    compare_hash(out, ref, x64, K, L, exact=True, what="cs recheck")
    c = to_host(cnt, np.uint64)
    assert c[1] <= c[0] and c[2] == 0


def test_keys_only_output_matches():
    """Keys alone (the timed configuration: no codes, no projection) equal keys
    computed with every debug output on; key_ld > n leaves the gap untouched."""
    dev()
    import torch
    n, d, K, L = 1500, 784, 16, 64
    x, h, s, b = _cs_case(n, d, K, L, "sparse", 5)
    xd, hd, sd, bd = to_dev(x), to_dev(h), to_dev(s), to_dev(b)
    full = lsh.lsh_hash_cs(xd, hd, sd, family=0, K=K, L=L, w=4.0, b=bd, codes=True, proj=True)
    keys = lsh.lsh_hash_cs(xd, hd, sd, family=0, K=K, L=L, w=4.0, b=bd)
    assert torch.equal(full["keys"], keys["keys"])
    again = lsh.lsh_hash_cs(xd, hd, sd, family=0, K=K, L=L, w=4.0, b=bd)
    assert torch.equal(again["keys"], keys["keys"])          # run-to-run determinism


def test_empty_input_is_noop():
    dev()
    import torch
    x = torch.empty((0, 64), dtype=torch.float32, device="cuda")
    h, s = synth.cs_state(64, 16, 3)
    out = lsh.lsh_hash_cs(x, to_dev(h), to_dev(s), family=1, K=4, L=4)
    assert out["keys"].shape == (4, 0)


HCS_CASES = [
    # n, d, dk, mk, K, L
    (1000, 4096, (64, 64), (32, 32), 16, 64),
    (1000, 4096, (16, 16, 16), (8, 8, 16), 16, 64),
    (700, 1000, (32, 32), (16, 8), 8, 16),        # zero padding: d < prod d_k
    (300, 960, (8, 10, 12), (4, 4, 8), 16, 8),    # unequal modes, d = prod d_k
]


@pytest.mark.parametrize("family", [oracle.E2LSH, oracle.SRP])
@pytest.mark.parametrize("n,d,dk,mk,K,L", HCS_CASES)
def test_hcs_hash_parity(n, d, dk, mk, K, L, family):
    dev()
    m = K * L
    x = synth.gaussian_clusters(n, d, 30, 0.2, 99 + d)
    hk, sk = synth.hcs_state(dk, mk, 100 + d)
    b = synth.shifts(m, 4.0, 101)
    x64 = x.astype(np.float64)
    ref = oracle.hash_points(x64, family, K, L, kind="hcs", w=4.0, b=b, dk=dk, mk=mk, hk=hk,
                             sk=sk)
    out = lsh.lsh_hash_hcs(to_dev(x), dk, mk, to_dev(np.concatenate(hk)),
                           to_dev(np.concatenate(sk)), family=family, K=K, L=L, w=4.0,
                           b=to_dev(b), codes=True, proj=True)
    compare_hash(out, ref, x64, K, L, what=f"hcs {dk}")
    cnt = to_dev(np.zeros(4, np.uint64))
    out = lsh.lsh_hash_hcs(to_dev(x), dk, mk, to_dev(np.concatenate(hk)),
                           to_dev(np.concatenate(sk)), family=family, K=K, L=L, w=4.0,
                           b=to_dev(b), codes=True, recheck=True, counters=cnt)
    compare_hash(out, ref, x64, K, L, exact=True, what=f"hcs {dk} recheck")


def test_hcs_equals_cs_under_composite_hash():
    """Invariant: HCS with per-mode tables gives the same bits as CS run with
    the composite bin/sign of every coordinate (Definition def_hcs)."""
    dev()
    import torch
    n, d, dk, mk, K, L = 2000, 4096, (16, 16, 16), (8, 8, 16), 16, 64
    x = synth.gaussian_clusters(n, d, 30, 0.2, 5)
    hk, sk = synth.hcs_state(dk, mk, 6)
    b = synth.shifts(K * L, 4.0, 7)
    hb = np.zeros(d, np.uint32)
    sb = np.zeros(d, np.int8)
    for j in range(d):
        i1, i2, i3 = j % 16, (j // 16) % 16, j // 256
        hb[j] = hk[0][i1] + 8 * (hk[1][i2] + 8 * hk[2][i3])
        sb[j] = sk[0][i1] * sk[1][i2] * sk[2][i3]
    xd, bd = to_dev(x), to_dev(b)
    for fam in (0, 1):
        a = lsh.lsh_hash_hcs(xd, dk, mk, to_dev(np.concatenate(hk)), to_dev(np.concatenate(sk)),
                             family=fam, K=K, L=L, w=4.0, b=bd, proj=True)
        c = lsh.lsh_hash_cs(xd, to_dev(hb), to_dev(sb), family=fam, K=K, L=L, w=4.0, b=bd,
                            proj=True)
        assert torch.equal(a["keys"], c["keys"]) and torch.equal(a["proj"], c["proj"])


@pytest.mark.parametrize("kind", ["bf16", "fp8"])
@pytest.mark.parametrize("family", [oracle.E2LSH, oracle.SRP])
def test_low_precision_recheck_matches_fp64(kind, family):
    """BF16 / FP8-E4M3FN storage with per-row scales, FP32 accumulation and the
    FP64 near-edge recheck reproduce the FP64 oracle's codes on the
    dequantised points exactly."""
    dev()
    n, d, K, L = 1200, 16384, 16, 32
    x = synth.gaussian_clusters(n, d, 10, 0.1, 31)
    q, sc = synth.quantise_rows(x, kind)
    x64 = oracle.decode(q, sc)
    h, s = synth.cs_state(d, K * L, 32)
    b = synth.shifts(K * L, 4.0, 32)
    ref = oracle.hash_points(x64, family, K, L, kind="cs", w=4.0, b=b, h=h, s=s)
    cnt = to_dev(np.zeros(4, np.uint64))
    out = lsh.lsh_hash_cs(to_dev(q), to_dev(h), to_dev(s), family=family, K=K, L=L, w=4.0,
                          b=to_dev(b), scale=to_dev(sc), codes=True, recheck=True, counters=cnt)
    compare_hash(out, ref, x64, K, L, exact=True, what=f"{kind} recheck")
    pre = lsh.lsh_hash_cs(to_dev(q), to_dev(h), to_dev(s), family=family, K=K, L=L, w=4.0,
                          b=to_dev(b), scale=to_dev(sc), codes=True, proj=True)
    compare_hash(pre, ref, x64, K, L, what=f"{kind} no recheck")


def test_fp8_decode_all_codes():
    """Every FP8-E4M3FN bit pattern except NaN decodes to the oracle's value
    (one point per pattern, identity hash d = m)."""
    dev()
    pats = np.array([p for p in range(256) if (p & 0x7f) != 0x7f], np.uint8)
    d = 16
    q = np.zeros((len(pats), d), np.uint8)
    q[:, 0] = pats
    sc = np.ones(len(pats), np.float32)
    h = np.arange(d, dtype=np.uint32)
    s = np.ones(d, np.int8)
    out = lsh.lsh_hash_cs(to_dev(q), to_dev(h), to_dev(s), family=1, K=4, L=4,
                          scale=to_dev(sc), proj=True, keys=False)
    got = to_host(out["proj"])[:, 0].astype(np.float64)
    want = np.array([oracle.fp8_value(int(p)) for p in pats])
    assert (got == want).all()


DENSE_CASES = [(10000, 1024, 8, 16), (1003, 784, 16, 64), (333, 100, 5, 7)]


@pytest.mark.parametrize("family", [oracle.E2LSH, oracle.SRP])
@pytest.mark.parametrize("n,d,K,L", DENSE_CASES)
def test_dense_hash_parity(n, d, K, L, family):
    dev()
    m = K * L
    x = synth.gaussian_clusters(n, d, 20, 0.1, 400 + d)
    R = synth.gaussian_matrix(d, m, 401)
    b = synth.shifts(m, 4.0, 402)
    x64 = x.astype(np.float64)
    ref = oracle.hash_points(x64, family, K, L, kind="dense", w=4.0, b=b, R=R)
    out = lsh.lsh_hash_dense(to_dev(x), to_dev(R), family=family, K=K, L=L, w=4.0, b=to_dev(b),
                             codes=True, proj=True)
    # dense dot products of d terms: allow the dense weight scale in the band
    compare_hash(out, ref, x64, K, L, weight_max=float(np.abs(R).max()),
                 what=f"dense n={n} d={d}")


def test_dense_with_cs_matrix_equals_cs():
    """Special case: the dense projection by the explicit count-sketch matrix
    is the count sketch (codes agree outside the near-edge band)."""
    dev()
    n, d, K, L = 2000, 256, 8, 16
    m = K * L
    x = synth.gaussian_clusters(n, d, 20, 0.1, 9)
    h, s = synth.cs_state(d, m, 10)
    R = np.zeros((d, m), np.float32)
    R[np.arange(d), h] = s
    b = synth.shifts(m, 4.0, 11)
    ys = lsh.lsh_hash_cs(to_dev(x), to_dev(h), to_dev(s), family=1, K=K, L=L, proj=True)
    yd = lsh.lsh_hash_dense(to_dev(x), to_dev(R), family=1, K=K, L=L, proj=True)
    np.testing.assert_allclose(to_host(yd["proj"]), to_host(ys["proj"]), rtol=0, atol=1e-4)


@pytest.mark.parametrize("family", [oracle.E2LSH, oracle.SRP])
@pytest.mark.parametrize("dk,mk", [((64, 64), (32, 32)), ((16, 16, 16), (8, 8, 16)),
                                   ((8, 10, 12), (4, 4, 8))])
def test_hcs_component_slots_parity(dk, mk, family):
    """HCS with a seeded permutation assigning sketch components to tables:
    projection, codes and keys against the oracle (fast path within the
    near-edge band, recheck exact)."""
    dev()
    d = int(np.prod(dk))
    m = int(np.prod(mk))
    K = 16 if m % 16 == 0 else 8
    L = m // K
    n = 1500
    x = synth.gaussian_clusters(n, d, 30, 0.2, 300 + d)
    hk, sk = synth.hcs_state(dk, mk, 301 + d)
    slot = synth.component_slots(m, 302 + d)
    b = synth.shifts(m, 4.0, 303)
    x64 = x.astype(np.float64)
    ref = oracle.hash_points(x64, family, K, L, kind="hcs", w=4.0, b=b, dk=dk, mk=mk, hk=hk,
                             sk=sk, comp_slot=slot)
    args = (to_dev(x), dk, mk, to_dev(np.concatenate(hk)), to_dev(np.concatenate(sk)))
    kw = dict(family=family, K=K, L=L, w=4.0, b=to_dev(b), comp_slot=to_dev(slot))
    out = lsh.lsh_hash_hcs(*args, codes=True, proj=True, **kw)
    compare_hash(out, ref, x64, K, L, what=f"hcs slots {dk}")
    cnt = to_dev(np.zeros(4, np.uint64))
    out = lsh.lsh_hash_hcs(*args, codes=True, recheck=True, counters=cnt, **kw)
    compare_hash(out, ref, x64, K, L, exact=True, what=f"hcs slots {dk} recheck")
    assert to_host(cnt, np.uint64)[3] == 0


def test_cs_component_slots_parity():
    """A component map on the count sketch: keys-only, codes and recheck."""
    dev()
    n, d, K, L = 5000, 784, 16, 64
    x, h, s, b = _cs_case(n, d, K, L, "sparse", 404)
    slot = synth.component_slots(K * L, 405)
    x64 = x.astype(np.float64)
    for fam in (oracle.E2LSH, oracle.SRP):
        ref = oracle.hash_points(x64, fam, K, L, kind="cs", w=4.0, b=b, h=h, s=s, comp_slot=slot)
        kw = dict(family=fam, K=K, L=L, w=4.0, b=to_dev(b), comp_slot=to_dev(slot))
        out = lsh.lsh_hash_cs(to_dev(x), to_dev(h), to_dev(s), **kw)
        compare_hash(out, ref, x64, K, L, what="cs slots keys only")
        out = lsh.lsh_hash_cs(to_dev(x), to_dev(h), to_dev(s), codes=True, recheck=True, **kw)
        compare_hash(out, ref, x64, K, L, exact=True, what="cs slots recheck")


def test_c3_hcs_index_has_no_constant_table():
    """The 4096-dimensional tensor-reshape workload with its own hash state:
    with contiguous tables some tables give every point one bucket; with the
    workload's component map no table does, and the index of the GPU keys
    equals the oracle's."""
    dev()
    wl = synth.C3
    n = 20000
    x = wl.points(n)
    b = wl.b()
    slot = wl.slots()
    xd = to_dev(x)
    for i, (dk, mk) in enumerate(wl.hcs):
        hk, sk = wl.hcs_state(i)
        args = (xd, dk, mk, to_dev(np.concatenate(hk)), to_dev(np.concatenate(sk)))
        kw = dict(family=oracle.E2LSH, K=wl.K, L=wl.L, w=wl.w, b=to_dev(b))
        plain = lsh.lsh_build_index(lsh.lsh_hash_hcs(*args, **kw)["keys"])
        assert (to_host(plain.arrays()[3]) == 1).sum() > 0, f"{dk}: contiguous tables"
        keys = lsh.lsh_hash_hcs(*args, comp_slot=to_dev(slot), **kw)["keys"]
        idx = lsh.lsh_build_index(keys)
        nu = to_host(idx.arrays()[3])
        assert (nu > 1).all(), f"{dk}: constant tables {np.nonzero(nu == 1)[0]}"
        rk = oracle.hash_points(x.astype(np.float64), oracle.E2LSH, wl.K, wl.L, kind="hcs",
                                w=wl.w, b=b, dk=dk, mk=mk, hk=hk, sk=sk, comp_slot=slot)
        tab_near = rk["near"].reshape(n, wl.L, wl.K).any(axis=2).T
        kg = to_host(keys, np.uint64)
        assert not ((kg != rk["keys"]) & ~tab_near).any()
        ref = oracle.build_index(kg)
        assert (to_host(idx.arrays()[0], np.uint32) == ref["sorted_ids"]).all()
        assert (nu == ref["nuniq"]).all()


def test_invalid_hash_state_is_counted():
    """counters[3] counts coordinates whose hash state is out of range (each is
    taken as 0), once per call."""
    dev()
    n, d, K, L = 3000, 256, 8, 4
    x, h, s, b = _cs_case(n, d, K, L, "clusters", 406)
    h = h.copy()
    h[[3, 77, 200]] = K * L + np.array([0, 5, 1000])
    cnt = to_dev(np.zeros(4, np.uint64))
    lsh.lsh_hash_cs(to_dev(x), to_dev(h), to_dev(s), family=1, K=K, L=L, counters=cnt)
    assert to_host(cnt, np.uint64).tolist()[1:] == [0, 0, 3]
    slot = synth.component_slots(K * L, 407)
    slot[5] = K * L
    h2, _ = synth.cs_state(d, K * L, 408)
    cnt = to_dev(np.zeros(4, np.uint64))
    lsh.lsh_hash_cs(to_dev(x), to_dev(h2), to_dev(s), family=1, K=K, L=L, counters=cnt,
                    comp_slot=to_dev(slot))
    assert to_host(cnt, np.uint64)[3] == (h2 == 5).sum()


@pytest.mark.parametrize("family", [oracle.E2LSH, oracle.SRP])
@pytest.mark.parametrize("n,d,K,L", [(10000, 1024, 8, 16), (1003, 784, 16, 64), (333, 100, 5, 7)])
def test_dense_bf16_parity(n, d, K, L, family):
    """BF16 dense projection (BF16 points with row scales, BF16 R, FP32
    accumulation on the BF16 matrix cores) against the FP64 oracle over the
    same BF16 values: projections within the dense band (d-term FP32 sums),
    codes equal outside the near-edge band."""
    dev()
    import torch
    m = K * L
    x = synth.gaussian_clusters(n, d, 20, 0.1, 440 + d)
    q, sc = synth.quantise_rows(x, "bf16")
    x64 = oracle.decode(q, sc)
    R = synth.gaussian_matrix(d, m, 441)
    Rb = torch.from_numpy(R).to(torch.bfloat16)
    R16 = Rb.to(torch.float32).numpy()                  # the BF16 values, exactly
    Rt = Rb.T.contiguous().view(torch.int16).to(dev())  # [m][d] bits
    b = synth.shifts(m, 4.0, 442)
    ref = oracle.hash_points(x64, family, K, L, kind="dense", w=4.0, b=b, R=R16)
    out = lsh.lsh_hash_dense_bf16(to_dev(q), to_dev(sc), Rt, family=family, K=K, L=L, w=4.0,
                                  b=to_dev(b) if family == 0 else None, codes=True, proj=True)
    compare_hash(out, ref, x64, K, L, weight_max=float(np.abs(R16).max()),
                 what=f"dense bf16 n={n} d={d}")


@pytest.mark.parametrize("family", [oracle.E2LSH, oracle.SRP])
@pytest.mark.parametrize("n,d,K,L", [
    (37, 32768, 16, 64),   # longest row the recheck takes: 128 KB of row hash entries, one wave
    (50, 64, 32, 256),     # m = 8192: one wave; too many keys to stage, stored directly
])
def test_hash_at_the_lds_limits(n, d, K, L, family):
    """Shapes at the edge of what one CU's LDS holds run with one wave per
    workgroup and still match the FP64 oracle exactly (recheck on)."""
    dev()
    m = K * L
    x = synth.gaussian_clusters(n, d, 5, 0.1, 3 + d)
    h, s = synth.cs_state(d, m, 4 + d)
    b = synth.shifts(m, 4.0, 4 + d)
    x64 = x.astype(np.float64)
    ref = oracle.hash_points(x64, family, K, L, kind="cs", w=4.0, b=b, h=h, s=s)
    out = lsh.lsh_hash_cs(to_dev(x), to_dev(h), to_dev(s), family=family, K=K, L=L, w=4.0,
                          b=to_dev(b), codes=True, proj=True, recheck=True)
    compare_hash(out, ref, x64, K, L, exact=True, what=f"lds limit d={d} m={m}")


def test_hash_beyond_the_lds_limits_is_refused():
    """m = 16384 bins do not fit one wave's LDS share, and the recheck takes
    at most 32768 coordinates: both are refused with EINVAL before any
    launch (the counters passed are left untouched)."""
    import torch
    device = dev()
    n = 8
    for d, K, L, rc, msg in [(64, 64, 256, False, "LDS"), (32769, 16, 4, True, "d <= 32768")]:
        m = K * L
        x = torch.ones((n, d), dtype=torch.float32, device=device)
        h = torch.zeros(d, dtype=torch.int32, device=device)
        s = torch.ones(d, dtype=torch.int8, device=device)
        b = torch.zeros(m, dtype=torch.float32, device=device)
        cnt = torch.full((4,), 7, dtype=torch.int64, device=device)
        with pytest.raises(lsh.LshError, match=msg):
            lsh.lsh_hash_cs(x, h, s, family=0, K=K, L=L, w=4.0, b=b, recheck=rc, counters=cnt)
        torch.cuda.synchronize()
        assert (cnt == 7).all()


@pytest.mark.parametrize("family", [oracle.E2LSH, oracle.SRP])
@pytest.mark.parametrize("heavy", [2, 256, 257])
def test_recheck_bin_table_every_path(heavy, family):
    """The recheck recomputes flagged components from a table of each bin's
    coordinates in ascending order.  A bin of up to 256 coordinates is ordered
    by one wave, a larger one sends the table to the full sort: both paths
    (heavy = 256 and 257 coordinates in one bin) give codes equal to the FP64
    oracle's, on rows with a wide dynamic range so that many components are
    flagged and recomputed."""
    dev()
    n, d, K, L = 300, 600, 8, 8
    m = K * L
    g = np.random.default_rng(heavy)
    h = np.where(np.arange(d) < heavy, 5, g.integers(0, m - 1, d))
    h = np.where((np.arange(d) >= heavy) & (h >= 5), h + 1, h).astype(np.uint32)  # skip bin 5
    s = np.where(g.random(d) < 0.5, -1, 1).astype(np.int8)
    b = synth.shifts(m, 4.0, 12)
    x = (g.standard_normal((n, d)) * np.exp2(g.integers(-20, 12, (n, d)))).astype(np.float32)
    x64 = x.astype(np.float64)
    ref = oracle.hash_points(x64, family, K, L, kind="cs", w=4.0, b=b, h=h, s=s)
    cnt = to_dev(np.zeros(4, np.uint64))
    out = lsh.lsh_hash_cs(to_dev(x), to_dev(h), to_dev(s), family=family, K=K, L=L, w=4.0,
                          b=to_dev(b), codes=True, recheck=True, counters=cnt)
    compare_hash(out, ref, x64, K, L, exact=True, what=f"bin table heavy={heavy}")
    assert int(to_host(cnt, np.uint64)[0]) > 0


@pytest.mark.parametrize("family", [oracle.E2LSH, oracle.SRP])
def test_recheck_reuses_the_table_in_its_workspace(family):
    """recheck = 2 reuses the table (CSR of h) that a recheck = 1 call built in
    the same workspace: codes, keys and counters equal those of recheck = 1,
    for CS on BF16 rows and for HCS (N = 2) on FP32 rows, over several calls
    on other rows; the codes equal the FP64 oracle's."""
    dev()
    import torch
    K, L = 16, 32
    d = 4096
    x = synth.gaussian_clusters(900, d, 10, 0.1, 41)
    q, sc = synth.quantise_rows(x, "bf16")
    x64 = oracle.decode(q, sc)
    h, s = synth.cs_state(d, K * L, 42)
    b = synth.shifts(K * L, 4.0, 42)
    kw = dict(family=family, K=K, L=L, w=4.0, b=to_dev(b), codes=True)
    ws = torch.empty(lsh.lib().lsh_hash_workspace_bytes(d, K * L, 1), dtype=torch.uint8,
                     device=dev())
    qd, sd_ = to_dev(q), to_dev(sc)
    for i, (lo, hi) in enumerate(((0, 300), (300, 700), (700, 900))):
        c1, c2 = to_dev(np.zeros(4, np.uint64)), to_dev(np.zeros(4, np.uint64))
        one = lsh.lsh_hash_cs(qd[lo:hi], to_dev(h), to_dev(s), scale=sd_[lo:hi], recheck=1,
                              counters=c1, **kw)
        two = lsh.lsh_hash_cs(qd[lo:hi], to_dev(h), to_dev(s), scale=sd_[lo:hi],
                              recheck=1 if i == 0 else 2, ws=ws, counters=c2, **kw)
        for key in ("keys", "codes"):
            assert torch.equal(one[key], two[key]), (i, key)
        assert (to_host(c1, np.uint64) == to_host(c2, np.uint64)).all()
    ref = oracle.hash_points(x64[700:900], family, K, L, kind="cs", w=4.0, b=b, h=h, s=s)
    assert (to_host(two["codes"]) == ref["codes"]).all()
    # HCS N = 2 (64 x 64 -> 16 x 32), FP32 rows
    dk, mk = (64, 64), (16, 32)
    hk, sk = synth.hcs_state(dk, mk, 43)
    hkd, skd = to_dev(np.concatenate(hk)), to_dev(np.concatenate(sk))
    xd = to_dev(x)
    ws2 = torch.empty(lsh.lib().lsh_hash_workspace_bytes(d, K * L, 1), dtype=torch.uint8,
                      device=dev())
    for i, (lo, hi) in enumerate(((0, 450), (450, 900))):
        one = lsh.lsh_hash_hcs(xd[lo:hi], dk, mk, hkd, skd, recheck=1, **kw)
        two = lsh.lsh_hash_hcs(xd[lo:hi], dk, mk, hkd, skd, recheck=1 if i == 0 else 2, ws=ws2,
                               **kw)
        for key in ("keys", "codes"):
            assert torch.equal(one[key], two[key]), (i, key)
