"""Continuous-batching server: every query of a mixed query/insert stream
against the oracle (one index over every point that arrived before it, the
query's watermark), the same query run alone, segment merges, and the HBM
budget."""
import numpy as np
import pytest

import oracle
from paper_2503_06737_amd import lsh, serve, synth
from gpu_util import dev, to_dev, to_host

pytestmark = pytest.mark.gpu


def _setup(n0, d, K, L, w, family, seed):
    x0 = synth.gaussian_clusters(n0, d, 8, 0.1, seed)
    h, s = synth.cs_state(d, K * L, seed + 1)
    b = synth.shifts(K * L, w, seed + 1)
    qsrc = iter(synth.gaussian_clusters(4000, d, 8, 0.1, seed, stream=1))
    isrc = iter(synth.gaussian_clusters(4000, d, 8, 0.1, seed, stream=2))
    take = lambda it: (lambda m: np.stack([next(it) for _ in range(m)]))
    return x0, h, s, b, take(qsrc), take(isrc)


def _serve(n0=3000, d=64, K=8, L=8, w=8.0, family=lsh.E2LSH, n_req=60, max_points=40,
           budget=60_000, seed=71, inflight=2, realtime=False, storage="f32", query_streams=2,
           query_frac=0.7):
    dev()
    x0, h, s, b, qsrc, isrc = _setup(n0, d, K, L, w, family, seed)
    reqs = serve.poisson_stream(n_req, 1e4, query_frac, max_points, d, qsrc, isrc, seed)
    srv = serve.Server(to_dev(x0), to_dev(h), to_dev(s), to_dev(b), K=K, L=L, w=w,
                       capacity=n0 + sum(r.points.shape[0] for r in reqs), budget_bytes=budget,
                       k=10, metric=family, max_inflight=inflight, recheck=True, storage=storage,
                       query_streams=query_streams)
    stats = srv.serve(reqs, realtime=realtime)
    return srv, reqs, stats, (x0, h, s, b, K, L, w, family, storage)


def _oracle_points(srv, reqs, params):
    """Every point in id order as the FP64 oracle sees it: FP32 values, or the
    oracle's own BF16 / FP8 quantisation decoded (the GPU's stored codes must
    equal the oracle's bit for bit)."""
    x0, storage = params[0], params[8]
    allx = np.concatenate([x0] + [r.points for r in reqs if r.kind == "insert"])
    if storage == "f32":
        return allx.astype(np.float64)
    q, sc = oracle.quantise_rows(allx, storage)
    n = allx.shape[0]
    qg = to_host(srv.base[:n], np.uint16 if storage == "bf16" else np.uint8)
    assert (qg == q).all(), "stored codes differ from the oracle's quantisation"
    assert (to_host(srv.scale[:n]) == sc).all()
    return oracle.decode(q, sc)


def _check_oracle(srv, reqs, params):
    x0, h, s, b, K, L, w, family, storage = params
    allx = _oracle_points(srv, reqs, params)
    okw = dict(kind="cs", w=w, b=b, h=h, s=s)
    ref_idx = oracle.build_index(oracle.hash_points(allx, family, K, L, **okw)["keys"])
    for r in reqs:
        if r.kind != "query":
            continue
        q64 = r.points.astype(np.float64)
        qk = oracle.hash_points(q64, family, K, L, **okw)["keys"]
        rids, rsc, rnc = oracle.query([ref_idx], allx, q64, qk, 10, r.watermark, family)
        assert (to_host(r.ncand) == rnc).all(), f"request at {r.arrival}: ncand"
        np.testing.assert_allclose(to_host(r.score), rsc, rtol=1e-5, atol=1e-5)
        ids = to_host(r.ids)
        for i in range(ids.shape[0]):
            fin = np.isfinite(rsc[i])
            kth = rsc[i][fin][-1] if fin.any() else np.inf
            strict = rsc[i] < kth * (1 - 1e-5) - 1e-5
            assert set(ids[i][strict]) == set(rids[i][strict])


@pytest.mark.parametrize("storage", ["f32", "bf16", "fp8"])
def test_serve_matches_oracle_and_alone(storage):
    srv, reqs, stats, params = _serve(storage=storage)
    assert stats.batches > 3 and stats.builds_checked >= 2
    _check_oracle(srv, reqs, params)
    # the same query alone (its own call, same watermark) gives the same bits
    segs = [sg.index for sg in srv.segments]
    for r in reqs:
        if r.kind != "query":
            continue
        Q = to_dev(r.points)
        qk = srv._hash(Q)
        ids, sc, nc = lsh.lsh_query(segs, srv.base[:srv.n], Q, qk, k=10,
                                    watermark=r.watermark, metric=srv.metric,
                                    base_scale=None if srv.scale is None else srv.scale[:srv.n])
        assert (to_host(ids) == to_host(r.ids)).all()
        assert (to_host(sc).view(np.uint32) == to_host(r.score).view(np.uint32)).all()
        assert (to_host(nc) == to_host(r.ncand)).all()


def test_serve_merges_segments_and_runs_oversized_requests_alone():
    # a budget below every request: each request runs alone, with nothing
    # else in flight, so inserts create more than 16 segments and force merges
    srv, reqs, stats, params = _serve(n_req=90, budget=1, family=lsh.SRP, w=1.0, seed=73,
                                      inflight=4)
    assert stats.batches == len(reqs)
    assert stats.max_inflight_seen == 1
    assert stats.merges >= 1 and len(srv.segments) <= serve.MAX_SEGMENTS
    _check_oracle(srv, reqs, params)


@pytest.mark.parametrize("storage", ["f32", "fp8"])
def test_serve_budget_bounds_bytes_in_flight(storage):
    """With every request within the budget, the transient bytes of the
    batches in flight never exceed it, while several batches are in flight
    at once (their work overlaps on the device)."""
    dev()
    d, K, L, w, seed = 64, 8, 8, 8.0, 75
    x0, h, s, b, qsrc, isrc = _setup(3000, d, K, L, w, lsh.E2LSH, seed)
    reqs = serve.poisson_stream(120, 1e4, 0.7, 40, d, qsrc, isrc, seed)
    probe = serve.Server(to_dev(x0), to_dev(h), to_dev(s), to_dev(b), K=K, L=L, w=w,
                         capacity=4000, budget_bytes=1, storage=storage)
    largest = max(probe._request_bytes(r) for r in reqs)
    budget = 3 * largest
    srv = serve.Server(to_dev(x0), to_dev(h), to_dev(s), to_dev(b), K=K, L=L, w=w,
                       capacity=3000 + sum(r.points.shape[0] for r in reqs), budget_bytes=budget,
                       k=10, max_inflight=4, recheck=True, storage=storage)
    stats = srv.serve(reqs, realtime=False)
    assert 0 < stats.peak_bytes <= budget
    assert stats.max_inflight_seen >= 2
    _check_oracle(srv, reqs, (x0, h, s, b, K, L, w, lsh.E2LSH, storage))


def test_serve_realtime_latency_fields():
    srv, reqs, stats, _ = _serve(n_req=40, realtime=True)
    summary = serve.summarize(reqs, stats, max(r.done for r in reqs))
    assert summary["queries"] + summary["inserts"] == 40
    assert all(np.isfinite(r.done) and r.done >= 0 for r in reqs)


def _draw_serve(i):
    g = np.random.default_rng([0x5E7E, i])
    return dict(n_req=int(g.integers(20, 121)), max_points=int(g.choice([1, 16, 64, 300])),
                budget=int(g.choice([1, 30_000, 200_000, 10**9])), inflight=int(g.integers(1, 6)),
                storage=str(g.choice(["f32", "bf16", "fp8"])), family=int(g.integers(0, 2)),
                query_streams=int(g.integers(1, 4)), query_frac=float(g.choice([0.3, 0.7, 0.95])),
                seed=200 + i)


@pytest.mark.parametrize("i", range(8))
def test_serve_random_configurations(i):
    """Random server configurations (budget from one byte to unlimited, 1-5
    batches in flight, 1-3 query streams, request sizes up to 300 points, any
    storage and family): every query answer equals the oracle's over exactly
    the points inserted before it arrived, and the bytes in flight stay within
    the budget whenever no single request exceeds it."""
    c = _draw_serve(i)
    print(f"random serving configuration {i}: {c}", flush=True)
    fam = c.pop("family")
    srv, reqs, stats, params = _serve(family=fam, w=8.0 if fam == lsh.E2LSH else 1.0, **c)
    assert stats.batches >= 1 and stats.max_inflight_seen <= c["inflight"]
    largest = max(srv._request_bytes(r) for r in reqs)
    if largest <= c["budget"]:
        assert stats.peak_bytes <= c["budget"]
    assert len(srv.segments) <= serve.MAX_SEGMENTS
    _check_oracle(srv, reqs, params)
