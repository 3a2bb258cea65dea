"""lsh_hash_cs_noalloc (static scratch, no allocation) against lsh_hash_cs
(caller workspace) through the C ABI: two calls in a row on one GPU, the
second with a smaller input, with the FP64 near-edge recheck on (the path
that uses the scratch).  Codes, projections, keys and counters must be
bit-identical to the workspace entry point's, and the rechecked codes equal
to the FP64 oracle's."""
import numpy as np
import pytest
import torch

import oracle
from paper_2503_06737_amd import lsh, synth
from gpu_util import compare_hash, dev, to_dev

pytestmark = pytest.mark.gpu


def _outputs(n, K, L, device):
    m = K * L
    return {"keys": torch.empty((L, n), dtype=torch.int64, device=device),
            "codes": torch.empty((n, m), dtype=torch.int32, device=device),
            "proj": torch.empty((n, m), dtype=torch.float32, device=device),
            "counters": torch.zeros(4, dtype=torch.int64, device=device)}


@pytest.mark.parametrize("family", [oracle.E2LSH, oracle.SRP])
def test_noalloc_matches_workspace_entry_point(family):
    device = dev()
    K, L, w = 16, 32, 4.0
    m = K * L
    # (n, d, dtype, seed): BF16 rows of 16384 (the largest recheck table of
    # this shape), then fewer, shorter FP32 rows so the second call's CSR is
    # smaller and a stale first table would show
    cases = [(1500, 16384, "bf16", 61), (700, 1000, "f32", 62)]
    for n, d, kind, seed in cases:
        print(f"noalloc family={family} n={n} d={d} {kind}", flush=True)
        x = synth.gaussian_clusters(n, d, 10, 0.1, seed)
        if kind == "f32":
            q, sc = x, None
            x64 = x.astype(np.float64)
        else:
            q, sc = synth.quantise_rows(x, kind)
            x64 = oracle.decode(q, sc)
        h, s = synth.cs_state(d, m, seed + 1)
        b = synth.shifts(m, w, seed + 2)
        qd, hd, sd, bd = to_dev(q), to_dev(h), to_dev(s), to_dev(b)
        scd = None if sc is None else to_dev(sc)
        kw = dict(family=family, K=K, L=L, w=w, b=bd, scale=scd, recheck=True)
        ref_cnt = to_dev(np.zeros(4, np.uint64))
        want = lsh.lsh_hash_cs(qd, hd, sd, codes=True, proj=True, counters=ref_cnt, **kw)
        got = _outputs(n, K, L, device)
        lsh.lsh_hash_cs_noalloc(qd, hd, sd, got, **kw)
        torch.cuda.synchronize()
        for name in ("keys", "codes", "proj"):
            assert torch.equal(got[name], want[name]), f"{name} differ (n={n} d={d})"
        assert torch.equal(got["counters"], ref_cnt), (got["counters"], ref_cnt)
        ref = oracle.hash_points(x64, family, K, L, kind="cs", w=w, b=b, h=h, s=s)
        compare_hash(got, ref, x64, K, L, exact=True, what=f"noalloc n={n} d={d}")


def test_noalloc_rejects_beyond_the_scratch():
    """d above the static scratch's 32768 coordinates is refused with recheck."""
    device = dev()
    n, d, K, L = 4, 32769, 4, 4
    x = torch.zeros((n, d), dtype=torch.float32, device=device)
    h = torch.zeros(d, dtype=torch.int32, device=device)
    s = torch.ones(d, dtype=torch.int8, device=device)
    b = torch.zeros(K * L, dtype=torch.float32, device=device)
    with pytest.raises(lsh.LshError, match="no-allocation recheck"):
        lsh.lsh_hash_cs_noalloc(x, h, s, _outputs(n, K, L, device), family=0, K=K, L=L, w=4.0,
                                b=b, recheck=True)
