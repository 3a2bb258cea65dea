"""Continuously batched serving of the LSH index on one GPU.

The paper defines the index (Section 3.1) and the query by the union of a
point's buckets (Section 3.1) re-ranked by exact distance (Section 6); it
says nothing about serving.  This module runs that path as a service: query
and insert requests arrive over time, and every kernel is a library call
(`lsh_hash_cs`, `lsh_build_index`, `lsh_query`).

* Requests are admitted first in, first out, into a batch whose projected
  device bytes stay within an HBM budget.  A single request larger than the
  budget runs alone.
* A batch first commits its inserts: the points are appended to the
  resident base, hashed, and indexed as a new segment whose ids continue
  from the last segment.  Then it answers its queries against all segments.
* A query sees exactly the inserts that arrived before it (its watermark).
  Queries of one batch are grouped by watermark, one `lsh_query` call per
  group, so a result never depends on how requests were batched.
* At most 16 segments are live.  When an insert would make a 17th, the
  insert segments are merged by re-indexing their stored keys as one
  segment.
* Up to `max_inflight` batches are enqueued on the stream at once, so the
  host prepares batch i+1 while the GPU runs batch i.  A request's latency
  runs from its arrival to the moment the host observes its batch's
  completion event.

Host copies of request points are part of the measured latency (the points
arrive in host memory).
"""
from __future__ import annotations

import math
import time
from collections import deque
from dataclasses import dataclass, field

import numpy as np
import torch

from . import lsh

MAX_SEGMENTS = 16


@dataclass
class Request:
    arrival: float          # seconds from the start of the stream
    kind: str               # "query" | "insert"
    points: np.ndarray      # [m, d] float32 (host)
    # filled in by the server
    watermark: int = -1     # queries: ids visible to this query
    first_id: int = -1      # inserts: id of the first inserted point
    batch: int = -1
    done: float = math.nan  # completion observed on the host (seconds)
    ids: torch.Tensor | None = None
    score: torch.Tensor | None = None
    ncand: torch.Tensor | None = None


@dataclass
class Segment:
    id_base: int
    n: int
    keys: torch.Tensor      # [L][n] int64 on the device (kept for merges)
    index: lsh.Index


@dataclass
class Stats:
    batches: int = 0
    merges: int = 0
    peak_bytes: int = 0
    points_hashed: int = 0
    busy_s: float = 0.0
    batch_sizes: list = field(default_factory=list)


def poisson_stream(n_req: int, rate: float, query_frac: float, max_points: int, d: int,
                   query_source, insert_source, seed: int) -> list[Request]:
    """A seeded request stream: exponential inter-arrival times (rate per
    second), query with probability query_frac, sizes floor(exp(U[0, ln
    (max_points + 1)))) clipped to [1, max_points].  query_source(m) and
    insert_source(m) return the next m points of their streams."""
    g = np.random.Generator(np.random.PCG64(np.random.SeedSequence([seed, 0x5E2F])))
    t = 0.0
    out = []
    for _ in range(n_req):
        t += g.exponential(1.0 / rate)
        kind = "query" if g.random() < query_frac else "insert"
        m = int(np.exp(g.random() * np.log(max_points + 1)))
        m = min(max(m, 1), max_points)
        src = query_source if kind == "query" else insert_source
        out.append(Request(arrival=t, kind=kind, points=np.ascontiguousarray(src(m), np.float32)))
    return out


class Server:
    def __init__(self, base: torch.Tensor, h, s, b, *, K: int, L: int, w: float, capacity: int,
                 budget_bytes: int, k: int = 10, metric: int = lsh.E2LSH, max_inflight: int = 2,
                 recheck: bool = False):
        dev = base.device
        self.recheck = recheck
        self.d = base.shape[1]
        self.K, self.L, self.w, self.k, self.metric = K, L, w, k, metric
        self.h, self.s, self.b = h, s, b
        self.budget = int(budget_bytes)
        self.max_inflight = max_inflight
        self.base = torch.empty((capacity, self.d), dtype=torch.float32, device=dev)
        n0 = base.shape[0]
        self.base[:n0] = base
        self.n = n0
        keys = self._hash(self.base[:n0])
        self.segments: list[Segment] = [Segment(0, n0, keys, lsh.lsh_build_index(keys))]
        self.stats = Stats()
        self.arrived_inserts = n0   # ids of everything that arrived so far (watermarks)

    # ------------------------------------------------------------- kernels
    def _hash(self, x: torch.Tensor) -> torch.Tensor:
        return lsh.lsh_hash_cs(x, self.h, self.s, family=self.metric, K=self.K, L=self.L,
                               w=self.w, b=self.b if self.metric == lsh.E2LSH else None,
                               recheck=self.recheck)["keys"]

    def _request_bytes(self, r: Request) -> int:
        m = r.points.shape[0]
        if r.kind == "query":
            return m * (4 * self.d + 8 * self.L + 12 * self.k + 4)
        return (m * 8 * self.L + lsh.lib().lsh_index_bytes(m, self.L)
                + lsh.lib().lsh_build_workspace_bytes(m, self.L))

    def _insert(self, pts: torch.Tensor) -> None:
        m = pts.shape[0]
        if self.n + m > self.base.shape[0]:
            raise RuntimeError("base capacity exhausted")
        self.base[self.n:self.n + m] = pts
        keys = self._hash(self.base[self.n:self.n + m])
        if len(self.segments) >= MAX_SEGMENTS:
            # merge every insert segment (ids are contiguous) and this one
            ins = self.segments[1:]
            keys = torch.cat([sg.keys for sg in ins] + [keys], dim=1)
            first = ins[0].id_base
            self.segments = self.segments[:1]
            self.stats.merges += 1
        else:
            first = self.n
        self.segments.append(Segment(first, keys.shape[1], keys,
                                     lsh.lsh_build_index(keys, id_base=first)))
        self.n += m

    def _run_batch(self, batch: list[Request], pinned) -> None:
        ins = [r for r in batch if r.kind == "insert"]
        qs = [r for r in batch if r.kind == "query"]
        if ins:
            pts = pinned([r.points for r in ins])
            self._insert(pts)
            self.stats.points_hashed += pts.shape[0]
        if qs:
            Q = pinned([r.points for r in qs])
            qk = self._hash(Q)
            self.stats.points_hashed += Q.shape[0]
            lo = 0
            while lo < len(qs):     # one call per watermark group
                hi = lo
                while hi < len(qs) and qs[hi].watermark == qs[lo].watermark:
                    hi += 1
                a = sum(r.points.shape[0] for r in qs[:lo])
                z = a + sum(r.points.shape[0] for r in qs[lo:hi])
                segs = [sg.index for sg in self.segments if sg.id_base < qs[lo].watermark]
                ids, sc, nc = lsh.lsh_query(segs, self.base[:self.n], Q[a:z], qk[:, a:z],
                                            k=self.k, watermark=qs[lo].watermark,
                                            metric=self.metric)
                off = 0
                for r in qs[lo:hi]:
                    m = r.points.shape[0]
                    r.ids, r.score, r.ncand = ids[off:off + m], sc[off:off + m], nc[off:off + m]
                    off += m
                lo = hi

    # --------------------------------------------------------------- serve
    def serve(self, requests: list[Request], realtime: bool = True) -> Stats:
        """Serve the stream.  realtime=False admits every request at once in
        arrival order (the same batches as an infinitely fast arrival)."""
        dev = self.base.device
        # watermarks follow arrival order (inserts before a query are visible)
        seen = self.arrived_inserts
        for r in requests:
            if r.kind == "insert":
                r.first_id = seen
                seen += r.points.shape[0]
            else:
                r.watermark = seen
        self.arrived_inserts = seen

        def pinned(arrs: list) -> torch.Tensor:
            # the requests' points copied once, into one pinned buffer (the
            # host allocator keeps it until the copy to the device is done)
            m = sum(a.shape[0] for a in arrs)
            host = torch.empty((m, self.d), dtype=torch.float32, pin_memory=True)
            off = 0
            for a in arrs:
                host[off:off + a.shape[0]].copy_(torch.from_numpy(a))
                off += a.shape[0]
            return host.to(dev, non_blocking=True)

        inflight: deque = deque()
        live = 0      # bytes of the batches in flight
        i = 0
        t0 = time.perf_counter()
        clock = (lambda: time.perf_counter() - t0) if realtime else (lambda: math.inf)
        stamp = lambda: time.perf_counter() - t0
        while i < len(requests) or inflight:
            while inflight and inflight[0][1].query():
                ev0, ev1, reqs, nbytes = inflight.popleft()
                now = stamp()
                for r in reqs:
                    r.done = now
                live -= nbytes
                self.stats.busy_s += ev0.elapsed_time(ev1) * 1e-3
            now = clock()
            if (i < len(requests) and len(inflight) < self.max_inflight
                    and requests[i].arrival <= now):
                batch, nbytes = [], 0
                while i < len(requests) and requests[i].arrival <= now:
                    rb = self._request_bytes(requests[i])
                    if batch and nbytes + rb > self.budget:
                        break
                    batch.append(requests[i])
                    nbytes += rb
                    i += 1
                for r in batch:
                    r.batch = self.stats.batches
                self.stats.batches += 1
                self.stats.batch_sizes.append(sum(r.points.shape[0] for r in batch))
                ev0 = torch.cuda.Event(enable_timing=True)
                ev1 = torch.cuda.Event(enable_timing=True)
                ev0.record()
                self._run_batch(batch, pinned)
                ev1.record()
                live += nbytes
                self.stats.peak_bytes = max(self.stats.peak_bytes, live)
                inflight.append((ev0, ev1, batch, nbytes))
                continue
            if inflight:
                inflight[0][1].synchronize() if not realtime else time.sleep(20e-6)
            elif i < len(requests):
                wait = requests[i].arrival - clock()
                if wait > 0:
                    time.sleep(min(wait, 1e-3))
        torch.cuda.synchronize()
        return self.stats


def summarize(requests: list[Request], stats: Stats, wall_s: float) -> dict:
    q = [r for r in requests if r.kind == "query"]
    ins = [r for r in requests if r.kind == "insert"]

    def pct(xs, p):
        return round(float(np.percentile(xs, p)) * 1e3, 3) if xs else None

    lq = [r.done - r.arrival for r in q]
    li = [r.done - r.arrival for r in ins]
    qpts = sum(r.points.shape[0] for r in q)
    ipts = sum(r.points.shape[0] for r in ins)
    return {
        "requests": len(requests), "queries": len(q), "inserts": len(ins),
        "query_points": qpts, "insert_points": ipts,
        "query_latency_ms": {"p50": pct(lq, 50), "p99": pct(lq, 99)},
        "insert_latency_ms": {"p50": pct(li, 50), "p99": pct(li, 99)},
        "query_points_per_s": round(qpts / wall_s, 1),
        "points_per_s": round((qpts + ipts) / wall_s, 1),
        "batches": stats.batches, "mean_batch_points": round(float(np.mean(stats.batch_sizes)), 1),
        "segment_merges": stats.merges, "peak_budget_bytes": stats.peak_bytes,
        "gpu_busy_frac": round(stats.busy_s / wall_s, 3),   # batch time / wall time
    }
