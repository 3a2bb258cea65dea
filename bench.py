"""Benchmark: points hashed + indexed per second, CS-E2LSH vs dense E2LSH.

Workload (image-like rows): n = 1,000,000 points, d = 784, FP32 with ~80%
exact zeros (x = Bernoulli(0.2) * U(0,1)), K = 16 components per table,
L = 64 tables (m = 1024), w = 4.  One step = CS-E2LSH hashing of every point
(bucket keys only) + the index build (per table, the (key, id) pairs put in
key order and the bucket offsets), from points resident in HBM to finished
tables.

Printed as one JSON line.  Beside the headline value the same run measures
the dense E2LSH baseline (Y = X R on FP32 matrix cores, same index build),
CS-SRP and dense SRP, query latency (p50/p99 of hash + probe + re-rank of
query batches against the built index), the serving loop under sustained and
overloaded request streams with an FP32 base and sustained streams with a
BF16 / FP8 base, CS against HCS at 500k x 4096, BF16/FP8 hashing with and
without the FP64 recheck, per-kernel timings with HIP events on the stream
the kernels run on, and the oracle leg: the FP64 CPU oracle on the same
workload (all rows hashed and one index built on the host cores, all
threads and one thread), then the low-precision servers' first answers
checked against the oracle.

  python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu] [--quick]
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0        # MI355X HBM3E, GB/s
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "hash_kernel_c2_traffic.json")
HASH_SRC = os.path.join(ROOT, "paper_2503_06737_amd", "csrc", "hash.hip")
FP32_MFMA_PEAK_TF = 157.3    # MI355X dense FP32 matrix, TFLOP/s
BF16_MFMA_PEAK_TF = 2500.0   # MI355X dense BF16 matrix, TFLOP/s


def _events(torch):
    return torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)


def timed(torch, fn, reps):
    """Median and all times (ms) of fn() over reps runs, HIP events on the current stream."""
    ts = []
    for _ in range(reps):
        a, b = _events(torch)
        a.record()
        fn()
        b.record()
        b.synchronize()
        ts.append(a.elapsed_time(b))
    return float(np.median(ts)), ts


def hash_traffic():
    """HBM bytes per hash launch from the committed rocprofv3 counter summary
    (FETCH_SIZE + WRITE_SIZE, each scaled by the copy-kernel calibration), or
    None when the kernel source changed since the counters were taken."""
    import hashlib
    try:
        with open(TRAFFIC_FILE) as f:
            t = json.load(f)
        with open(HASH_SRC, "rb") as f:
            sha = hashlib.sha256(f.read()).hexdigest()
    except OSError:
        return None
    if t.get("source_sha256") != sha:
        return None
    return t.get("traffic_bytes_per_launch")


def copy_ceiling(torch, dev, nbytes=1 << 30, reps=5):
    """Streaming ceiling of this GPU: a plain elementwise copy (read nbytes,
    write nbytes) timed with HIP events.  Under rocprofv3 --pmc the same
    launches calibrate FETCH_SIZE / WRITE_SIZE against known sizes."""
    src = torch.ones(nbytes // 4, dtype=torch.float32, device=dev)
    dst = torch.empty_like(src)
    for _ in range(2):
        torch.neg(src, out=dst)
    med, _ = timed(torch, lambda: torch.neg(src, out=dst), reps)
    del src, dst
    return {"kernel": "torch.neg(out=) elementwise, 1 GiB read + 1 GiB written",
            "bytes_per_launch": 2 * nbytes, "ms": round(med, 4),
            "gbs": round(2 * nbytes / (med * 1e-3) / 1e9, 1)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--quick", action="store_true", help="skip every extra")
    ap.add_argument("--extras", default="steps,query,hcs,precision",
                    help="comma-separated extras: steps (dense E2LSH, CS-SRP, dense SRP), "
                         "query (latency and serving), hcs, precision")
    ap.add_argument("--n", type=int, default=None, help="override n (testing only)")
    ap.add_argument("--no-copy", action="store_true", help="skip the streaming-copy ceiling")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU; --gpus must be 1 "
                          "(the multi-GPU design shards points and is not built)"}))
        sys.exit(2)

    # One hardware queue per stream this run keeps busy at once: the null
    # stream, the build's side stream, and serving's insert and two query
    # streams.  With HIP's default of four, a stream used before serving
    # starts leaves two of serving's streams on one in-order queue, where one
    # waits behind the other's kernels: the overload stream lost 30% of its
    # throughput.  Read when HIP initialises, so it is set before torch is
    # imported.
    if int(os.environ.get("GPU_MAX_HW_QUEUES", "4")) < 8:
        os.environ["GPU_MAX_HW_QUEUES"] = "8"

    import torch
    from paper_2503_06737_amd import lsh, synth

    wl = synth.C2
    n = args.n or wl.n
    copy = None if args.no_copy else copy_ceiling(torch, torch.device("cuda:0"))
    if copy:
        print(f"[bench] copy ceiling {copy['gbs']} GB/s", file=sys.stderr, flush=True)
    d, K, L, m, w = wl.d, wl.K, wl.L, wl.m, wl.w
    dev = torch.device("cuda:0")
    t0 = time.time()
    x_host = wl.points(n)
    h, s = wl.cs()
    b = wl.b()
    R = wl.R()
    print(f"[bench] generated {n}x{d} points in {time.time() - t0:.1f}s", file=sys.stderr, flush=True)

    X = torch.from_numpy(x_host).to(dev)
    hd, sd = torch.from_numpy(h.view(np.int32)).to(dev), torch.from_numpy(s).to(dev)
    bd, Rd = torch.from_numpy(b).to(dev), torch.from_numpy(R).to(dev)
    keys = torch.empty((L, n), dtype=torch.int64, device=dev)
    mem = torch.empty(lsh.lib().lsh_index_bytes(n, L), dtype=torch.uint8, device=dev)
    ws = torch.empty(lsh.lib().lsh_build_workspace_bytes(n, L), dtype=torch.uint8, device=dev)

    import ctypes as C
    L_ = lsh.lib()

    def hash_into(family, dense=False):
        pts = lsh.points(X)
        disc = lsh.Disc(family, m, K, L, w, bd.data_ptr() if family == 0 else None, 0)
        out = lsh.Out(keys.data_ptr(), n, None, None, None)
        st = C.c_void_p(torch.cuda.current_stream().cuda_stream)
        if dense:
            rc = L_.lsh_hash_dense(C.byref(pts), C.c_void_p(Rd.data_ptr()), C.byref(disc),
                                   C.byref(out), st)
        else:
            rc = L_.lsh_hash_cs(C.byref(pts), C.c_void_p(hd.data_ptr()), C.c_void_p(sd.data_ptr()),
                                C.byref(disc), C.byref(out), None, 0, st)
        lsh._check(rc)

    index_holder = {}
    # the build's heavy-bucket kernels run on a second stream, concurrently
    # with its segment sorts (the call joins it back to the current stream)
    side = torch.cuda.Stream(dev)

    def build():
        idx = lsh.lsh_build_index(keys, mem=mem, ws=ws, side_stream=side)
        index_holder["idx"] = idx

    def step(family=0, dense=False):
        hash_into(family, dense)
        build()

    # ---------------------------------------------------------------- headline
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    ev = [_events(torch) for _ in range(args.steps)]
    hash_ev = [_events(torch) for _ in range(args.steps)]
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    for i in range(args.steps):
        ev[i][0].record()
        hash_ev[i][0].record()
        hash_into(0)
        hash_ev[i][1].record()
        build()
        ev[i][1].record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t_start
    ms_step = wall * 1e3 / args.steps
    step_ms = [a.elapsed_time(b) for a, b in ev]
    hash_ms = [a.elapsed_time(b) for a, b in hash_ev]
    value = n * args.steps / wall

    hash_med = float(np.median(hash_ms))
    bytes_per_point = d * 4 + 8 * L          # read the row, write L keys
    hash_gbs = n * bytes_per_point / (hash_med * 1e-3) / 1e9
    build_med = float(np.median([sm - hm for sm, hm in zip(step_ms, hash_ms)]))

    res = {
        "metric": "points hashed+indexed/s (CS-E2LSH, one index build)",
        "value": round(value, 1),
        "unit": "points/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic (seeded; image-like sparse rows, Bernoulli(0.2) x U(0,1))",
        "config": {"workload": wl.name, "n": n, "d": d, "K": K, "L": L, "m": m, "w": w,
                   "family": "CS-E2LSH", "index": "per table: MSD split on the top varying bits, LDS sorts of the segments, parallel pivot split of heavy buckets"},
        "roofline": {"bound": "hbm", "achieved": round(hash_gbs, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(hash_gbs / HBM_PEAK_GBS, 4), "traffic": hash_traffic(),
                     "kernel": "hash_kernel (CS-E2LSH sketch + discretise + keys)",
                     "bytes_per_launch": n * bytes_per_point,
                     "avg_launch_ms": round(hash_med, 4)},
        "breakdown_ms": {"hash": round(hash_med, 4), "index_build": round(build_med, 4)},
    }
    if copy:
        res["roofline"]["copy_ceiling_gbs"] = copy["gbs"]
        res["roofline"]["frac_of_copy_ceiling"] = round(hash_gbs / copy["gbs"], 4)
    print(f"[bench] CS-E2LSH step {np.median(step_ms):.3f} ms (hash {hash_med:.3f})",
          file=sys.stderr, flush=True)

    ex = set() if args.quick else {e for e in args.extras.split(",") if e}
    if ex:
        extra = {}
        other_steps = (("dense_e2lsh", 0, True), ("cs_srp", 1, False), ("dense_srp", 1, True))
        for name, fam, dense in (other_steps if "steps" in ex else ()):
            for _ in range(2):
                step(fam, dense)
            torch.cuda.synchronize()
            st_ms, _ = timed(torch, lambda: step(fam, dense), max(3, args.steps // 2))
            hs_ms, _ = timed(torch, lambda: hash_into(fam, dense), max(3, args.steps // 2))
            e = {"ms_per_step": round(st_ms, 4), "points_per_s": round(n / (st_ms * 1e-3), 1),
                 "hash_ms": round(hs_ms, 4)}
            if dense:
                tf = 2.0 * n * d * m / (hs_ms * 1e-3) / 1e12
                e["hash_tflops"] = round(tf, 2)
                e["mfma_frac"] = round(tf / FP32_MFMA_PEAK_TF, 4)
            else:
                e["hash_gbs"] = round(n * bytes_per_point / (hs_ms * 1e-3) / 1e9, 1)
            extra[name] = e
            print(f"[bench] {name}: {e}", file=sys.stderr, flush=True)
        if "steps" in ex:
            extra["speedup_cs_vs_dense_e2lsh"] = {
                "hash_only": round(extra["dense_e2lsh"]["hash_ms"] / hash_med, 2),
                "hash_plus_index": round(extra["dense_e2lsh"]["ms_per_step"] /
                                         float(np.median(step_ms)), 2)}
            extra["dense_e2lsh_bf16"] = dense_bf16_step(torch, lsh, X, keys, build, n, d, K, L,
                                                        m, w, R, bd, args.steps)
            extra["speedup_cs_vs_dense_e2lsh"]["hash_only_vs_bf16_dense"] = round(
                extra["dense_e2lsh_bf16"]["hash_ms"] / hash_med, 2)
            extra["space"] = state_space(torch, lsh, synth, d, m, K, L, hd, sd, Rd)
            extra["per_table_sketches"] = tables_throughput(torch, lsh, synth, X, bd, hash_med)

        # query latency: hash + probe + exact re-rank of query batches against a
        # CS-E2LSH index of the serving-shaped workload (2M x 960 Gaussian
        # clusters, K=16, L=32).  The image-like workload above is a
        # throughput case: its mostly-empty bins put most points in a few huge
        # buckets, so it is not used for queries.
        del X, keys, mem, ws
        index_holder.clear()
        torch.cuda.empty_cache()
        if "query" in ex:
            extra["query_latency"], extra["serving"] = query_latency(torch, lsh, synth, dev)
            torch.cuda.empty_cache()
        if "hcs" in ex:
            extra["hcs_vs_cs"] = hcs_throughput(torch, lsh, dev)
            torch.cuda.empty_cache()
        if "precision" in ex:
            extra["precision"] = precision_path(torch, lsh, dev)
            torch.cuda.empty_cache()
        res["extras"] = extra

    # ---------------------------------------------------------------- CPU oracle
    if not args.no_cpu:
        res["cpu_baseline"] = cpu_baseline(x_host, h, s, b, K, L, w)
        serving_x = res.get("extras", {}).get("serving")
        for smp in SERVED_SAMPLES:
            serving_x[smp["run"]]["oracle_agreement"] = oracle_agreement(smp)
            print(f"[bench] {smp['run']} oracle agreement "
                  f"{serving_x[smp['run']]['oracle_agreement']}", file=sys.stderr, flush=True)
    SERVED_SAMPLES.clear()
    print(json.dumps(res), flush=True)


def dense_bf16_step(torch, lsh, X, keys, build, n, d, K, L, m, w, R, bd, steps):
    """Dense E2LSH with BF16 operands on the BF16 matrix cores (the points
    stored as BF16 with row scales, R rounded to BF16), the same index
    build: how fast a dense projection gets when its precision is given up.
    The BF16 copy of the points is made on the device before timing."""
    q, sc = lsh.lsh_quantize_rows(X, "bf16")
    Rt = torch.from_numpy(R).to(X.device).to(torch.bfloat16).T.contiguous().view(torch.int16)

    def hash_once():
        keys.copy_(lsh.lsh_hash_dense_bf16(q, sc, Rt, family=0, K=K, L=L, w=w, b=bd)["keys"])

    def hash_only():
        return lsh.lsh_hash_dense_bf16(q, sc, Rt, family=0, K=K, L=L, w=w, b=bd)

    def step():
        hash_once()
        build()

    for _ in range(2):
        step()
    torch.cuda.synchronize()
    st_ms, _ = timed(torch, step, max(3, steps // 2))
    hs_ms, _ = timed(torch, hash_only, max(3, steps // 2))
    tf = 2.0 * n * d * m / (hs_ms * 1e-3) / 1e12
    e = {"ms_per_step": round(st_ms, 4), "points_per_s": round(n / (st_ms * 1e-3), 1),
         "hash_ms": round(hs_ms, 4), "hash_tflops": round(tf, 2),
         "mfma_frac": round(tf / BF16_MFMA_PEAK_TF, 4), "dtype": "bf16 operands, f32 accumulate",
         "note": "step time includes a key copy; hash_ms is the projection+discretise+key kernel"}
    print(f"[bench] dense_e2lsh_bf16: {e}", file=sys.stderr, flush=True)
    del q, sc, Rt
    return e


def tables_throughput(torch, lsh, synth, X, bd, shared_ms):
    """Independent per-table sketches (the protocol of Section 6: L sketches
    of K components, O(L d) additions per point) against the shared sketch
    (one sketch of K L components, O(d)): on the image-like 1M x 784 points
    at K = 16, L = 64, and on 10k x 1024 cluster points at the recall
    protocol's K = 8, L = 16."""
    res = {}
    n, d = X.shape
    K, L = 16, 64
    ht, st = synth.cs_tables_state(d, K, L, 11)
    htd = torch.from_numpy(ht.view(np.int32)).to(X.device)
    std_ = torch.from_numpy(st).to(X.device)
    fn = lambda: lsh.lsh_hash_cs_tables(X, htd, std_, family=0, K=K, L=L, w=4.0, b=bd)
    for _ in range(2):
        fn()
    torch.cuda.synchronize()
    ms, _ = timed(torch, fn, 5)
    res["image_like_1M_784_K16_L64"] = {
        "per_table_ms": round(ms, 3), "shared_ms": round(shared_ms, 4),
        "per_table_points_per_s": round(n / (ms * 1e-3), 1),
        "ratio": round(ms / shared_ms, 1), "additions_ratio": L}
    wl = synth.C1
    Xc = torch.from_numpy(wl.points()).to(X.device)
    K, L = 8, 16
    ht, st = synth.cs_tables_state(wl.d, K, L, 12)
    hs, ss = synth.cs_state(wl.d, K * L, 12)
    b = torch.from_numpy(synth.shifts(K * L, 4.0, 12)).to(X.device)
    t = lambda a: torch.from_numpy(a.view(np.int32) if a.dtype == np.uint32 else a).to(X.device)
    htd, std_, hsd, ssd = t(ht), t(st), t(hs), t(ss)
    ftab = lambda: lsh.lsh_hash_cs_tables(Xc, htd, std_, family=0, K=K, L=L, w=4.0, b=b)
    fsh = lambda: lsh.lsh_hash_cs(Xc, hsd, ssd, family=0, K=K, L=L, w=4.0, b=b)
    for f in (ftab, fsh):
        for _ in range(2):
            f()
    torch.cuda.synchronize()
    mt, _ = timed(torch, ftab, 10)
    msh, _ = timed(torch, fsh, 10)
    res["clusters_10k_1024_K8_L16"] = {
        "per_table_ms": round(mt, 4), "shared_ms": round(msh, 4),
        "ratio": round(mt / msh, 2), "additions_ratio": L}
    print(f"[bench] per-table sketches {res}", file=sys.stderr, flush=True)
    return res


def state_space(torch, lsh, synth, d, m, K, L, hd, sd, Rd):
    """Bytes of each family's projection state as allocated on the device
    (the space comparison of Section 6): dense R (FP32 and BF16), the count
    sketch's h and s, the higher-order sketch's per-mode tables for the
    500k x 4096 workload's N = 2 and 3, and L independent per-table count
    sketches (h and s per table)."""
    res = {"d": d, "m": m,
           "dense_f32": Rd.numel() * Rd.element_size(),
           "dense_bf16": Rd.numel() * 2,
           "cs": hd.numel() * hd.element_size() + sd.numel() * sd.element_size()}
    wl3 = synth.C3
    for i, name in enumerate(("hcs_n2", "hcs_n3")):
        hk, sk = wl3.hcs_state(i)
        hkd = torch.from_numpy(np.concatenate(hk).view(np.int32)).to(hd.device)
        skd = torch.from_numpy(np.concatenate(sk)).to(hd.device)
        res[name] = {"d": wl3.d, "dk": list(wl3.hcs[i][0]), "mk": list(wl3.hcs[i][1]),
                     "bytes": hkd.numel() * 4 + skd.numel(), "cs_same_d_bytes": 5 * wl3.d}
    ht, st = synth.cs_tables_state(d, K, L, 3)
    htd, std_ = torch.from_numpy(ht.view(np.int32)).to(hd.device), torch.from_numpy(st).to(hd.device)
    res["cs_per_table"] = htd.numel() * 4 + std_.numel()
    print(f"[bench] space {res}", file=sys.stderr, flush=True)
    return res


def query_latency(torch, lsh, synth, dev):
    wl = synth.C5
    t0 = time.time()
    xh = wl.points()
    Qh = wl.queries(1024)
    h, s = wl.cs()
    b = wl.b()
    print(f"[bench] serving-shaped data {xh.shape} in {time.time() - t0:.1f}s", file=sys.stderr,
          flush=True)
    X = torch.from_numpy(xh).to(dev)
    Q = torch.from_numpy(Qh).to(dev)
    hd = torch.from_numpy(h.view(np.int32)).to(dev)
    sd = torch.from_numpy(s).to(dev)
    bd = torch.from_numpy(b).to(dev)
    kw = dict(family=0, K=wl.K, L=wl.L, w=wl.w, b=bd)
    keys = lsh.lsh_hash_cs(X, hd, sd, **kw)["keys"]
    idx = lsh.lsh_build_index(keys)
    torch.cuda.synchronize()
    out = []
    for bs in (1, 64, 1024):
        def q_batch(bs=bs):
            qk = lsh.lsh_hash_cs(Q[:bs], hd, sd, **kw)["keys"]
            return lsh.lsh_query([idx], X, Q[:bs], qk, k=10, metric=0)
        for _ in range(3):
            q_batch()
        med, ts = timed(torch, q_batch, 50 if bs < 1024 else 20)
        _, _, nc = q_batch()
        out.append({"batch": bs, "p50_ms": round(float(np.percentile(ts, 50)), 4),
                    "p99_ms": round(float(np.percentile(ts, 99)), 4),
                    "queries_per_s": round(bs / (med * 1e-3), 1),
                    "mean_candidates": round(float(nc.float().mean().item()), 1)})
        print(f"[bench] query {out[-1]}", file=sys.stderr, flush=True)
    lat = {"workload": wl.name, "k": 10, "batches": out}
    del idx, keys
    torch.cuda.empty_cache()
    return lat, serving(torch, synth, dev, wl, X, xh, hd, sd, bd)


# served answers kept for the oracle leg (agreement of the low-precision path)
SERVED_SAMPLES = []


def serving(torch, synth, dev, wl, X, xh, hd, sd, bd):
    """Continuously batched query/insert stream against the same index: a
    sustainable Poisson rate and the planned 50,000 req/s (overload) with an
    FP32 base, then the sustainable rate with the base stored as BF16 and as
    FP8-E4M3FN (per-row scales, FP64 near-edge recheck).  The answers of the
    low-precision runs' first queries are kept for the oracle leg, which
    compares them with the FP64 oracle on the same stored values."""
    from paper_2503_06737_amd import serve
    qpool = wl.points(400_000, stream=1)
    ipool = wl.points(100_000, stream=2)
    cur = {"q": 0, "i": 0}

    def src(pool, key):
        def take(m):
            lo = cur[key] % (pool.shape[0] - m)
            cur[key] = lo + m
            return pool[lo:lo + m]
        return take

    def server(reqs, storage="f32"):
        cap = X.shape[0] + sum(r.points.shape[0] for r in reqs if r.kind == "insert")
        return serve.Server(X, hd, sd, bd, K=wl.K, L=wl.L, w=wl.w, capacity=cap,
                            budget_bytes=2 << 30, k=10, max_inflight=4, storage=storage,
                            recheck=storage != "f32")

    out = {"budget_bytes": 2 << 30, "max_inflight": 4, "query_streams": 2}
    runs = (("sustained", 600.0, 1200, "f32"), ("planned_overload", 50_000.0, 20_000, "f32"),
            ("sustained_bf16", 600.0, 1200, "bf16"), ("sustained_fp8", 600.0, 1200, "fp8"))
    for name, rate, n_req, storage in runs:
        # warm-up, not measured: a server of the same configuration serves a
        # short stream of its own (device and pinned-memory allocator caches,
        # kernel set-up); the measured server then starts from that state
        wreqs = serve.poisson_stream(min(n_req // 4, 600), rate, 0.9, 4096, wl.d,
                                     src(qpool, "q"), src(ipool, "i"), wl.seed + 4)
        wsrv = server(wreqs, storage)
        wsrv.serve(wreqs, realtime=True)
        del wsrv
        reqs = serve.poisson_stream(n_req, rate, 0.9, 4096, wl.d, src(qpool, "q"),
                                    src(ipool, "i"), wl.seed + 3)
        srv = server(reqs, storage)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        st = srv.serve(reqs, realtime=True)
        wall = time.perf_counter() - t0
        summ = serve.summarize(reqs, st, wall)
        summ.update({"offered_req_per_s": rate, "query_frac": 0.9, "max_points": 4096,
                     "storage": storage, "recheck": storage != "f32",
                     "resident_base_bytes": srv.base.numel() * srv.base.element_size()})
        out[name] = summ
        print(f"[bench] serving {name}: {summ}", file=sys.stderr, flush=True)
        if storage != "f32":
            # the first 64 query requests, with every insert before the last of them
            qs = [r for r in reqs if r.kind == "query"][:64]
            last = qs[-1].watermark
            ins = [r.points for r in reqs if r.kind == "insert" and r.first_id < last]
            SERVED_SAMPLES.append({
                "run": name, "storage": storage, "base": xh, "inserts": ins,
                "h": hd.cpu().numpy().view(np.uint32), "s": sd.cpu().numpy(),
                "b": bd.cpu().numpy(), "K": wl.K, "L": wl.L, "w": wl.w,
                "queries": [(r.points, r.watermark, r.ids.cpu().numpy(), r.score.cpu().numpy(),
                             r.ncand.cpu().numpy()) for r in qs]})
        del srv, reqs
        torch.cuda.empty_cache()
    out["workload"] = wl.name + " base, fresh query (stream 1) and insert (stream 2) draws"
    return out


def _device_clusters(torch, n, d, n_centres, sigma, seed, dev):
    """Gaussian clusters drawn on the device (seeded): the recipe of the
    cluster workloads, without a multi-GB host transfer."""
    g = torch.Generator(device=dev).manual_seed(seed)
    mu = torch.randn((n_centres, d), generator=g, device=dev)
    c = torch.randint(0, n_centres, (n,), generator=g, device=dev)
    x = torch.empty((n, d), device=dev)
    step = 65536
    for lo in range(0, n, step):
        hi = min(n, lo + step)
        x[lo:hi] = mu[c[lo:hi]] + sigma * torch.randn((hi - lo, d), generator=g, device=dev)
    return x


def table_stats(torch, idx, n):
    """Bucket statistics of a built index: tables whose every point shares one
    key (constant tables), distinct keys per table, the largest bucket."""
    _, _, offs, nuniq = idx.arrays()
    nu = nuniq.long()
    ar = torch.arange(offs.shape[1] - 1, device=offs.device)
    sizes = (offs[:, 1:].long() - offs[:, :-1].long()) * (ar[None, :] < nu[:, None])
    big = sizes.max(dim=1).values.float() / max(n, 1)
    return {"constant_tables": int((nu == 1).sum().item()),
            "distinct_keys_median": int(nu.median().item()), "distinct_keys_min": int(nu.min().item()),
            "largest_bucket_frac_max": round(float(big.max().item()), 4),
            "largest_bucket_frac_median": round(float(big.median().item()), 4)}


def hcs_throughput(torch, lsh, dev):
    """HCS (N = 2 and 3) vs CS at m = 1024 on 500k x 4096 clusters: hashing
    alone (keys only) and hash + index build.  HCS assigns its sketch
    components to tables by the workload's seeded permutation; the bucket
    statistics are reported with and without it (contiguous tables sit inside
    one mode slice, and an empty mode bin makes such a table constant)."""
    from paper_2503_06737_amd import synth
    wl = synth.C3
    n, d, K, L, w = wl.n, wl.d, wl.K, wl.L, wl.w
    X = _device_clusters(torch, n, d, wl.n_centres, wl.sigma, wl.seed, dev)
    h, s = wl.cs()
    b = torch.from_numpy(wl.b()).to(dev)
    slot = torch.from_numpy(wl.slots().view(np.int32)).to(dev)
    hd, sd = torch.from_numpy(h.view(np.int32)).to(dev), torch.from_numpy(s).to(dev)
    bytes_pp = d * 4 + 8 * L
    keys = torch.empty((L, n), dtype=torch.int64, device=dev)
    mem = torch.empty(lsh.lib().lsh_index_bytes(n, L), dtype=torch.uint8, device=dev)
    ws = torch.empty(lsh.lib().lsh_build_workspace_bytes(n, L), dtype=torch.uint8, device=dev)
    res = {"workload": wl.name, "n": n, "d": d, "m": K * L, "K": K, "L": L}

    def bench_fn(hash_fn):
        def step():
            keys.copy_(hash_fn()["keys"])
            return lsh.lsh_build_index(keys, mem=mem, ws=ws)
        for _ in range(2):
            hash_fn()
            step()
        torch.cuda.synchronize()
        med, _ = timed(torch, hash_fn, 5)
        smed, _ = timed(torch, step, 5)
        idx = step()
        e = {"hash_ms": round(med, 4), "gbs": round(n * bytes_pp / (med * 1e-3) / 1e9, 1),
             "hash_copy_index_ms": round(smed, 4), **table_stats(torch, idx, n)}
        assert idx.check() == (0, 0)
        return e

    res["cs"] = bench_fn(lambda: lsh.lsh_hash_cs(X, hd, sd, family=0, K=K, L=L, w=w, b=b))
    for i, name in enumerate(("hcs_n2", "hcs_n3")):
        dk, mk = wl.hcs[i]
        hk, sk = wl.hcs_state(i)
        hkd = torch.from_numpy(np.concatenate(hk).view(np.int32)).to(dev)
        skd = torch.from_numpy(np.concatenate(sk)).to(dev)
        res[name] = bench_fn(lambda: lsh.lsh_hash_hcs(X, dk, mk, hkd, skd, family=0, K=K, L=L,
                                                      w=w, b=b, comp_slot=slot))
        res[name]["dk"], res[name]["mk"] = list(dk), list(mk)
        keys.copy_(lsh.lsh_hash_hcs(X, dk, mk, hkd, skd, family=0, K=K, L=L, w=w, b=b)["keys"])
        res[name]["contiguous_tables"] = table_stats(torch, lsh.lsh_build_index(keys, mem=mem,
                                                                                ws=ws), n)
    print(f"[bench] hcs_vs_cs {res}", file=sys.stderr, flush=True)
    del X, keys, mem, ws
    return res


def precision_path(torch, lsh, dev):
    """BF16 / FP8-E4M3FN points with a per-row scale (200k x 16384 clusters,
    K=16, L=32, m=512): hashing with and without the FP64 near-edge recheck.
    recomputed = components re-evaluated in FP64; changed = those whose FP32
    code differed (the fast path's disagreement with the FP64 evaluation)."""
    from paper_2503_06737_amd import synth
    n, d, K, L, w = 200_000, 16_384, 16, 32, 4.0
    X = _device_clusters(torch, n, d, 50, 0.1, 250306737 + 4000, dev)
    amax = X.abs().amax(dim=1).clamp_min(1e-30)
    h, s = synth.cs_state(d, K * L, 9)
    hd, sd = torch.from_numpy(h.view(np.int32)).to(dev), torch.from_numpy(s).to(dev)
    b = torch.from_numpy(synth.shifts(K * L, w, 9)).to(dev)
    res = {"n": n, "d": d, "K": K, "L": L, "m": K * L}
    for name, dt, qmax, esz in (("bf16", torch.bfloat16, 1.0, 2), ("fp8_e4m3fn",
                                                                    torch.float8_e4m3fn, 448.0, 1)):
        scale = (amax / qmax).float()
        q = (X / scale[:, None]).clamp(-qmax, qmax).to(dt)
        bytes_pp = d * esz + 4 + 8 * L
        e = {}
        # recheck 2: the workspace already holds the recheck's table of h (a
        # server's calls after its first)
        ws = torch.empty(lsh.lib().lsh_hash_workspace_bytes(d, K * L, 1), dtype=torch.uint8,
                         device=dev)
        lsh.lsh_hash_cs(q[:1], hd, sd, family=0, K=K, L=L, w=w, b=b, scale=scale[:1], recheck=1,
                        ws=ws)
        for rc, key in ((0, "fast"), (1, "recheck"), (2, "recheck_table_kept")):
            fn = lambda c=None: lsh.lsh_hash_cs(q, hd, sd, family=0, K=K, L=L, w=w, b=b,
                                                scale=scale, recheck=rc, counters=c,
                                                ws=ws if rc == 2 else None)
            for _ in range(2):
                fn()
            torch.cuda.synchronize()
            med, _ = timed(torch, fn, 5)
            c = torch.zeros(4, dtype=torch.int64, device=dev)
            fn(c)
            cnt = c.cpu().numpy()
            e[key] = {
                "ms": round(med, 4), "gbs": round(n * bytes_pp / (med * 1e-3) / 1e9, 1),
                **({"recomputed": int(cnt[0]), "changed": int(cnt[1]),
                    "changed_per_million_codes": round(cnt[1] / (n * K * L) * 1e6, 3)} if rc
                   else {"uncertain": int(cnt[0])})}
        res[name] = e
        print(f"[bench] precision {name}: {e}", file=sys.stderr, flush=True)
        del q
    del X
    return res


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(x_host, h, s, b, K, L, w):
    """Oracle leg, part 1: the FP64 oracle (C, OpenMP) on this host over the
    same workload, every row hashed (decode, CS sketch, discretise, keys; in
    row chunks to bound memory) and one index over all keys (per-table sort).
    Median of 3 after one warm-up, with all OpenMP threads; then once more
    with one thread on the first 100,000 rows (scaled to points/s)."""
    import oracle
    oracle.lib()
    threads = oracle.max_threads()

    def run(x):
        n = x.shape[0]
        keys = np.empty((L, n), np.uint64)
        chunk = 50000
        t0 = time.perf_counter()
        for lo in range(0, n, chunk):
            x64 = oracle.decode(x[lo:lo + chunk])
            out = oracle.hash_points(x64, oracle.E2LSH, K, L, kind="cs", w=w, b=b, h=h, s=s)
            keys[:, lo:lo + chunk] = out["keys"]
        t_hash = time.perf_counter() - t0
        oracle.build_index(keys)
        return t_hash, time.perf_counter() - t0

    n = x_host.shape[0]
    run(x_host[:100_000])                         # warm-up
    times = sorted((run(x_host) for _ in range(3)), key=lambda t: t[1])
    t_hash, spent = times[1]
    oracle.set_threads(1)
    n1 = min(n, 100_000)
    t1_hash, t1 = run(x_host[:n1])
    oracle.set_threads(threads)
    return {"value": round(n / spent, 1), "unit": "points/s", "cores": threads, "kind": "oracle",
            "sample": f"the whole workload ({n} rows), median of 3: FP64 hashing {t_hash:.2f}s + "
                      f"one index build over all keys {spent - t_hash:.2f}s",
            "cpu_model": _cpu_model(), "host_cpus": os.cpu_count(),
            "single_thread": {"value": round(n1 / t1, 1), "unit": "points/s", "cores": 1,
                              "sample": f"first {n1} rows: hashing {t1_hash:.2f}s + index "
                                        f"{t1 - t1_hash:.2f}s"}}


def oracle_agreement(smp):
    """Oracle leg, part 2: the answers a low-precision server gave, against
    the FP64 oracle over the same stored values.  The oracle quantises the
    base and the inserts itself (its codes equal the device's bit for bit, as
    the tests check), decodes them to FP64, hashes and indexes them, and
    answers every sampled query at its watermark.  candidates_equal: the
    query's candidate count equals the oracle's (the union of its buckets);
    topk_equal: the top-k ids equal the oracle's outside near-ties of score."""
    import oracle
    t0 = time.perf_counter()
    allx = np.concatenate([smp["base"]] + smp["inserts"]) if smp["inserts"] else smp["base"]
    q, sc = oracle.quantise_rows(allx, smp["storage"])
    del allx
    n = q.shape[0]
    K, L, w = smp["K"], smp["L"], smp["w"]
    okw = dict(kind="cs", w=w, b=smp["b"], h=smp["h"], s=smp["s"])
    x64 = np.empty((n, q.shape[1]), np.float64)
    keys = np.empty((L, n), np.uint64)
    chunk = 100_000
    for lo in range(0, n, chunk):
        x64[lo:lo + chunk] = oracle.decode(q[lo:lo + chunk], sc[lo:lo + chunk])
        keys[:, lo:lo + chunk] = oracle.hash_points(x64[lo:lo + chunk], oracle.E2LSH, K, L,
                                                    **okw)["keys"]
    del q
    idx = oracle.build_index(keys)
    del keys
    npts = cand_eq = topk_eq = 0
    for pts, wm, ids, score, ncand in smp["queries"]:
        q64 = pts.astype(np.float64)
        qk = oracle.hash_points(q64, oracle.E2LSH, K, L, **okw)["keys"]
        rids, rsc, rnc = oracle.query([idx], x64, q64, qk, 10, wm, oracle.E2LSH)
        npts += q64.shape[0]
        cand_eq += int((ncand == rnc).sum())
        for i in range(q64.shape[0]):
            fin = np.isfinite(rsc[i])
            kth = rsc[i][fin][-1] if fin.any() else np.inf
            strict = rsc[i] < kth * (1 - 1e-5) - 1e-5
            topk_eq += int(set(ids[i][strict]) == set(rids[i][strict]))
    return {"query_requests": len(smp["queries"]), "query_points": npts,
            "candidates_equal_frac": round(cand_eq / max(npts, 1), 6),
            "topk_equal_frac": round(topk_eq / max(npts, 1), 6),
            "oracle_points": n, "oracle_s": round(time.perf_counter() - t0, 1)}


if __name__ == "__main__":
    main()
