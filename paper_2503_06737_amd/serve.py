"""Continuously batched serving of the LSH index on one GPU.

The paper defines the index (Section 3.1) and the query by the union of a
point's buckets (Section 3.1) re-ranked by exact distance (Section 6); it
says nothing about serving.  This module runs that path as a service: query
and insert requests arrive over time, and every kernel is a library call
(`lsh_quantize_rows`, `lsh_hash_cs`, `lsh_build_index`, `lsh_query`).

* Storage.  The resident base holds FP32 rows, or BF16 / FP8-E4M3FN codes
  with one FP32 scale per row (quantised on the device as points arrive).
  Hashing reads the stored form, so the index describes exactly the points
  the re-rank scores; with ``recheck`` the hashcodes equal those of an FP64
  evaluation over the stored (dequantised) values.
* Admission.  Requests are admitted first in, first out, into a batch while
  the transient device bytes of every batch in flight plus this one stay
  within ``budget_bytes``, and the batch within its share of the budget
  (``budget_bytes / max_inflight``), so that several batches are in flight
  at once.  A request larger than the budget runs alone, once nothing else is
  in flight.  Resident bytes (the base and the segments'
  keys and indexes) are counted separately.
* Streams.  Inserts run on one stream, in id order (the streams are shared
  by the servers of a device, so cached device memory carries over): the points are appended
  to the base, hashed, and indexed as a new segment whose ids continue from
  the last one.  Queries run on a pool of query streams; a batch's queries
  wait on an event recorded after the latest insert, so they see every point
  that arrived before them.  Batches on different streams overlap on the
  device: one batch's re-rank runs beside the next batch's hashing and
  index build.  They overlap only on hardware queues of their own: a process
  gets GPU_MAX_HW_QUEUES of them (HIP's default is 4), bound to streams as
  they are first used, so a process that also keeps other streams busy
  should raise it (bench.py sets 8).
* A query sees exactly the inserts that arrived before it (its watermark).
  Queries of one batch are grouped by watermark, one `lsh_query` call per
  group, so a result never depends on how requests were batched.
* At most 16 segments are live.  When an insert would make a 17th, the
  insert segments are merged by re-indexing their stored keys as one
  segment.
* Each index build's consistency counters (`lsh_build_check_async`) are
  copied to pinned memory beside the batch's completion event; a nonzero
  count stops the server with `IndexBuildError`.
* A request's latency runs from its arrival to the moment the host observes
  its batch's completion event, and includes the host-to-device copy of its
  points (they arrive in host memory and pass through a fixed ring of pinned
  chunks, allocated once per device).
"""
from __future__ import annotations

import gc
import math
import time
from dataclasses import dataclass, field

import numpy as np
import torch

from . import lsh

MAX_SEGMENTS = 16
STORAGE = ("f32", "bf16", "fp8")


class IndexBuildError(RuntimeError):
    """An index build reported a nonzero consistency counter."""


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

    @property
    def nbytes(self) -> int:
        return self.keys.numel() * 8 + self.index.mem.numel()


@dataclass
class Stats:
    batches: int = 0
    merges: int = 0
    peak_bytes: int = 0           # transient bytes of the batches in flight
    peak_resident_bytes: int = 0  # base + segments
    points_hashed: int = 0
    busy_s: float = 0.0           # union of the batches' device intervals
    batch_time_s: float = 0.0     # sum of the batches' device intervals
    max_inflight_seen: int = 0
    builds_checked: int = 0
    batch_sizes: list = field(default_factory=list)
    # batches whose host-side enqueue took over 2 ms:
    # (batch, points, insert points, merged, enqueue ms, of which staging copies ms)
    slow_enqueues: list = field(default_factory=list)
    gc_pauses_ms: list = field(default_factory=list)  # the collector's passes while serving
    staging_wait_s: float = 0.0   # host waits for a pinned staging chunk to come free


@dataclass
class _Inflight:
    reqs: list
    nbytes: int
    ev_start: torch.cuda.Event
    ev_end: torch.cuda.Event
    held: list                    # segments the batch's queries read
    checks: list                  # pinned int32 [2] build counters


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


# Streams shared by every server on a device.  torch's caching allocator
# keeps freed device blocks per stream, so a server that reuses the streams
# of an earlier one (a warm-up run, a restarted service) reuses its cached
# blocks instead of calling the runtime's allocator, which can synchronize
# the device, in the middle of a stream.
_STREAM_POOL: dict = {}


def _streams(dev, nq: int):
    key = (str(dev), nq)
    if key not in _STREAM_POOL:
        _STREAM_POOL[key] = (torch.cuda.Stream(dev), [torch.cuda.Stream(dev) for _ in range(nq)])
    return _STREAM_POOL[key]


class _PinnedRing:
    """Fixed pinned host chunks that stage request points on their way to the
    device.  A chunk is reused once the copy that read it has run (the event
    recorded after that copy), so serving never allocates pinned memory: the
    runtime's pinned allocation of a new, larger buffer took tens of
    milliseconds on the request path.  Shared by the servers of a device."""

    def __init__(self, nchunks: int, chunk_bytes: int):
        self.bufs = [torch.empty(chunk_bytes, dtype=torch.uint8, pin_memory=True)
                     for _ in range(nchunks)]
        self.evs: list = [None] * nchunks
        self.chunk_bytes = chunk_bytes
        self.i = 0
        self.wait_s = 0.0   # host time spent waiting for a chunk's copy to finish

    def to_device(self, arrs: list, d: int, dev) -> torch.Tensor:
        """The rows of arrs ([m_i][d] float32 host arrays), in order, as one
        [sum m_i][d] device tensor written on the current stream."""
        m = sum(a.shape[0] for a in arrs)
        out = torch.empty((m, d), dtype=torch.float32, device=dev)
        rows = self.chunk_bytes // (4 * d)
        stream = torch.cuda.current_stream(dev)
        o, ai, ar = 0, 0, 0
        while o < m:
            j = self.i
            self.i = (j + 1) % len(self.bufs)
            if self.evs[j] is not None:
                t = time.perf_counter()
                self.evs[j].synchronize()
                self.wait_s += time.perf_counter() - t
            host = self.bufs[j][:rows * d * 4].view(torch.float32).view(rows, d)
            hn = host.numpy()
            f = 0
            while f < rows and ai < len(arrs):
                t = min(rows - f, arrs[ai].shape[0] - ar)
                hn[f:f + t] = arrs[ai][ar:ar + t]
                f, ar = f + t, ar + t
                if ar == arrs[ai].shape[0]:
                    ai, ar = ai + 1, 0
            out[o:o + f].copy_(host[:f], non_blocking=True)
            ev = torch.cuda.Event()
            ev.record(stream)
            self.evs[j] = ev
            o += f
        return out


_RING_POOL: dict = {}
RING_CHUNKS, RING_CHUNK_BYTES = 64, 4 << 20


def _ring(dev, d: int) -> _PinnedRing:
    key = str(dev)
    r = _RING_POOL.get(key)
    if r is None or r.chunk_bytes < 4 * d:
        r = _RING_POOL[key] = _PinnedRing(RING_CHUNKS, max(RING_CHUNK_BYTES, 4 * d))
    return r


class Server:
    def __init__(self, base: torch.Tensor, h, s, b, *, K: int, L: int, w: float, capacity: int,
                 budget_bytes: int, k: int = 10, metric: int = lsh.E2LSH, max_inflight: int = 4,
                 recheck: bool = False, storage: str = "f32", query_streams: int = 2):
        """base: [n0][d] FP32 device tensor of the initial points (quantised
        on the device when storage is "bf16" or "fp8")."""
        if storage not in STORAGE:
            raise ValueError(f"storage must be one of {STORAGE}")
        dev = base.device
        self.device = dev
        self.recheck = recheck
        self._hash_ws = {}  # stream -> recheck workspace holding the table of h
        self.storage = storage
        self.d = base.shape[1]
        self.K, self.L, self.w, self.k, self.metric = K, L, w, k, metric
        self.h, self.s, self.b = h, s, b
        self.budget = int(budget_bytes)
        self.max_inflight = max(1, int(max_inflight))
        elt = {"f32": torch.float32, "bf16": torch.int16, "fp8": torch.uint8}[storage]
        self.base = torch.empty((capacity, self.d), dtype=elt, device=dev)
        self.scale = (None if storage == "f32"
                      else torch.empty(capacity, dtype=torch.float32, device=dev))
        self.s_ins, self.s_q = _streams(dev, max(1, query_streams))
        self.ring = _ring(dev, self.d)
        self._rr = 0
        self._ins_done: torch.cuda.Event | None = None
        n0 = base.shape[0]
        self.n = 0
        self.segments: list[Segment] = []
        self.stats = Stats()
        self.s_ins.wait_stream(torch.cuda.current_stream(dev))   # base was written there
        checks: list = []
        with torch.cuda.stream(self.s_ins):
            self._append(base, checks)
        torch.cuda.synchronize(dev)
        self._verify(checks)
        self.arrived_inserts = n0   # ids of everything that arrived so far (watermarks)

    # ------------------------------------------------------------- kernels
    def _stored(self, lo: int, hi: int):
        """(points, row scales) of base rows lo..hi in their stored form."""
        return self.base[lo:hi], None if self.scale is None else self.scale[lo:hi]

    def _hash(self, x: torch.Tensor, scale=None) -> torch.Tensor:
        # With the recheck, each stream keeps its workspace: the first call on
        # it builds the recheck's table of h there, later calls reuse it
        # (calls on one stream run in order).
        ws, mode = None, 0
        if self.recheck:
            st = torch.cuda.current_stream().cuda_stream
            ws = self._hash_ws.get(st)
            mode = 2 if ws is not None else 1
            if ws is None:
                nb = lsh.lib().lsh_hash_workspace_bytes(x.shape[1], self.K * self.L, 1)
                ws = self._hash_ws[st] = torch.empty(max(nb, 1), dtype=torch.uint8,
                                                     device=x.device)
        return lsh.lsh_hash_cs(x, self.h, self.s, family=self.metric, K=self.K, L=self.L,
                               w=self.w, b=self.b if self.metric == lsh.E2LSH else None,
                               scale=scale, recheck=mode, ws=ws)["keys"]

    def _build(self, keys: torch.Tensor, id_base: int, checks: list) -> lsh.Index:
        idx = lsh.lsh_build_index(keys, id_base=id_base)
        chk = torch.zeros(2, dtype=torch.int32).pin_memory()
        idx.check_async(chk)
        checks.append(chk)
        idx.ws = None   # the workspace is free once the copy is enqueued (same stream)
        return idx

    def _append(self, pts: torch.Tensor, checks: list) -> None:
        """Store FP32 device rows at the end of the base, hash them from their
        stored form and index them as a new segment (on the current stream)."""
        m = pts.shape[0]
        lo = self.n
        if lo + m > self.base.shape[0]:
            raise RuntimeError("base capacity exhausted")
        if self.storage == "f32":
            self.base[lo:lo + m] = pts
        else:
            lsh.lsh_quantize_rows(pts, self.storage, q=self.base[lo:lo + m],
                                  scale=self.scale[lo:lo + m])
        keys = self._hash(*self._stored(lo, lo + m))
        if len(self.segments) >= MAX_SEGMENTS:
            # merge every insert segment (ids are contiguous) and this one
            ins = self.segments[1:]
            keys = torch.cat([sg.keys for sg in ins] + [keys], dim=1)
            first = ins[0].id_base
            self.segments = self.segments[:1]
            self.stats.merges += 1
        else:
            first = lo
        self.segments.append(Segment(first, keys.shape[1], keys,
                                     self._build(keys, first, checks)))
        self.n += m

    # ---------------------------------------------------------- accounting
    def _request_bytes(self, r: Request) -> int:
        """Transient device bytes of one request: the points copied in, the
        hash outputs and query results or the index-build workspace."""
        m = r.points.shape[0]
        L = self.L
        if r.kind == "query":
            return m * (4 * self.d + 8 * L + 12 * self.k + 4)
        return m * 4 * self.d + lsh.lib().lsh_build_workspace_bytes(m, L)

    def _merge_bytes(self, m_ins: int) -> int:
        """Transient bytes of the merge an insert of m_ins points triggers (0 if none)."""
        if m_ins == 0 or len(self.segments) < MAX_SEGMENTS:
            return 0
        nm = sum(sg.n for sg in self.segments[1:]) + m_ins
        return nm * 8 * self.L + lsh.lib().lsh_build_workspace_bytes(nm, self.L)

    def resident_bytes(self) -> int:
        b = self.base.numel() * self.base.element_size()
        if self.scale is not None:
            b += self.scale.numel() * 4
        return b + sum(sg.nbytes for sg in self.segments)

    def _verify(self, checks: list) -> None:
        for c in checks:
            self.stats.builds_checked += 1
            if int(c[0]) or int(c[1]):
                raise IndexBuildError(f"index build counters {c.tolist()}: big-sort parts not "
                                      "queued / run-head waits given up; the segment is wrong")

    # --------------------------------------------------------------- batch
    def _pinned(self, arrs: list) -> torch.Tensor:
        """The requests' points staged through the pinned ring and copied to
        the device on the current stream."""
        return self.ring.to_device(arrs, self.d, self.device)

    def _run_batch(self, batch: list[Request], nbytes: int) -> _Inflight:
        ins = [r for r in batch if r.kind == "insert"]
        qs = [r for r in batch if r.kind == "query"]
        ev0 = torch.cuda.Event(enable_timing=True)
        ev1 = torch.cuda.Event(enable_timing=True)
        checks: list = []
        held: list = []
        tp = 0.0  # host time spent copying request points into pinned memory
        if ins:
            with torch.cuda.stream(self.s_ins):
                ev0.record()
                t0 = time.perf_counter()
                pts = self._pinned([r.points for r in ins])
                tp += time.perf_counter() - t0
                self._append(pts, checks)
                done = torch.cuda.Event()
                done.record()
                self._ins_done = done
            self.stats.points_hashed += pts.shape[0]
        if qs:
            sq = self.s_q[self._rr]
            self._rr = (self._rr + 1) % len(self.s_q)
            with torch.cuda.stream(sq):
                if not ins:
                    ev0.record()
                t0 = time.perf_counter()
                Q = self._pinned([r.points for r in qs])
                tp += time.perf_counter() - t0
                qk = self._hash(Q)
                self.stats.points_hashed += Q.shape[0]
                # the bucket lookup sees every insert that arrived before
                # (hashing the queries does not depend on them)
                if self._ins_done is not None:
                    sq.wait_event(self._ins_done)
                bq, bs = self.base[:self.n], None if self.scale is None else self.scale[:self.n]
                lo = 0
                while lo < len(qs):     # one call per watermark group
                    hi = lo
                    while hi < len(qs) and qs[hi].watermark == qs[lo].watermark:
                        hi += 1
                    a = sum(r.points.shape[0] for r in qs[:lo])
                    z = a + sum(r.points.shape[0] for r in qs[lo:hi])
                    segs = [sg for sg in self.segments if sg.id_base < qs[lo].watermark]
                    held.extend(segs)
                    ids, sc, nc = lsh.lsh_query([sg.index for sg in segs], bq, Q[a:z],
                                                qk[:, a:z], k=self.k,
                                                watermark=qs[lo].watermark, metric=self.metric,
                                                base_scale=bs)
                    off = 0
                    for r in qs[lo:hi]:
                        m = r.points.shape[0]
                        r.ids, r.score, r.ncand = ids[off:off + m], sc[off:off + m], nc[off:off + m]
                        off += m
                    lo = hi
                ev1.record()
        else:
            with torch.cuda.stream(self.s_ins):
                ev1.record()
        self._last_pin_ms = tp * 1e3
        return _Inflight(batch, nbytes, ev0, ev1, held, checks)

    # --------------------------------------------------------------- serve
    def serve(self, requests: list[Request], realtime: bool = True) -> Stats:
        """Serve the stream.  realtime=False admits every request at once in
        arrival order (the same batches as an infinitely fast arrival)."""
        # watermarks follow arrival order (inserts before a query are visible)
        seen = self.arrived_inserts
        for r in requests:
            if r.kind == "insert":
                r.first_id = seen
                seen += r.points.shape[0]
            else:
                r.watermark = seen
        self.arrived_inserts = seen

        # The objects alive now (the request stream, the resident state) are
        # moved out of the collector's reach: its full passes would otherwise
        # walk them all and stall the request loop for tens of milliseconds.
        gc.collect()
        gc.freeze()
        gc_t = {}

        def gc_cb(phase, info):
            if phase == "start":
                gc_t["t"] = time.perf_counter()
            elif "t" in gc_t:
                self.stats.gc_pauses_ms.append(round((time.perf_counter() - gc_t.pop("t")) * 1e3, 3))

        gc.callbacks.append(gc_cb)
        try:
            return self._serve(requests, realtime)
        finally:
            gc.callbacks.remove(gc_cb)
            gc.unfreeze()

    def _serve(self, requests: list[Request], realtime: bool) -> Stats:
        inflight: list[_Inflight] = []
        finished: list[_Inflight] = []
        # a batch grows to at most its share of the budget, so that several
        # batches can be in flight at once (a single larger request still
        # runs, once the bytes in flight leave room for it)
        slot = max(1, self.budget // self.max_inflight)
        wait0 = self.ring.wait_s
        live = 0      # transient bytes of the batches in flight
        i = 0
        t_ref = torch.cuda.Event(enable_timing=True)
        t_ref.record(torch.cuda.default_stream(self.device))
        t0 = time.perf_counter()
        clock = (lambda: time.perf_counter() - t0) if realtime else (lambda: math.inf)
        stamp = lambda: time.perf_counter() - t0
        self.stats.peak_resident_bytes = max(self.stats.peak_resident_bytes,
                                             self.resident_bytes())
        while i < len(requests) or inflight:
            for rec in [b for b in inflight if b.ev_end.query()]:
                now = stamp()
                for r in rec.reqs:
                    r.done = now
                live -= rec.nbytes
                self._verify(rec.checks)
                rec.held = []
                inflight.remove(rec)
                finished.append(rec)
            now = clock()
            admitted = False
            if (i < len(requests) and len(inflight) < self.max_inflight
                    and requests[i].arrival <= now):
                batch, nbytes, m_ins = [], 0, 0
                while i < len(requests) and requests[i].arrival <= now:
                    r = requests[i]
                    rb = self._request_bytes(r)
                    mi = m_ins + (r.points.shape[0] if r.kind == "insert" else 0)
                    tot = nbytes + rb + self._merge_bytes(mi) - self._merge_bytes(m_ins)
                    if batch and (tot > slot or live + tot > self.budget):
                        break
                    if not batch and inflight and live + tot > self.budget:
                        break
                    batch.append(r)
                    nbytes, m_ins = tot, mi
                    i += 1
                if batch:
                    for r in batch:
                        r.batch = self.stats.batches
                    self.stats.batches += 1
                    self.stats.batch_sizes.append(sum(r.points.shape[0] for r in batch))
                    te = time.perf_counter()
                    merges = self.stats.merges
                    inflight.append(self._run_batch(batch, nbytes))
                    te = (time.perf_counter() - te) * 1e3
                    if te > 2.0:
                        self.stats.slow_enqueues.append(
                            (self.stats.batches - 1, self.stats.batch_sizes[-1], m_ins,
                             self.stats.merges > merges, round(te, 2),
                             round(self._last_pin_ms, 2)))
                    live += nbytes
                    self.stats.peak_bytes = max(self.stats.peak_bytes, live)
                    self.stats.max_inflight_seen = max(self.stats.max_inflight_seen,
                                                       len(inflight))
                    self.stats.peak_resident_bytes = max(self.stats.peak_resident_bytes,
                                                         self.resident_bytes())
                    admitted = True
            if admitted:
                continue
            if inflight:
                if realtime:
                    time.sleep(20e-6)
                else:
                    inflight[0].ev_end.synchronize()
            elif i < len(requests):
                wait = requests[i].arrival - clock()
                if wait > 0:
                    time.sleep(min(wait, 1e-3))
        torch.cuda.synchronize(self.device)
        self.stats.staging_wait_s += self.ring.wait_s - wait0
        # device time: union and sum of the batches' [start, end] intervals
        iv = sorted((t_ref.elapsed_time(b.ev_start) * 1e-3, t_ref.elapsed_time(b.ev_end) * 1e-3)
                    for b in finished)
        union, cur_lo, cur_hi = 0.0, None, None
        for lo, hi in iv:
            self.stats.batch_time_s += hi - lo
            if cur_hi is None or lo > cur_hi:
                if cur_hi is not None:
                    union += cur_hi - cur_lo
                cur_lo, cur_hi = lo, hi
            else:
                cur_hi = max(cur_hi, hi)
        if cur_hi is not None:
            union += cur_hi - cur_lo
        self.stats.busy_s += union
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
        "peak_resident_bytes": stats.peak_resident_bytes,
        "max_batches_in_flight": stats.max_inflight_seen,
        "gpu_busy_frac": round(stats.busy_s / wall_s, 3),   # device-busy union / wall time
        # summed batch device time over the busy union: above 1 when batches overlap
        "device_overlap": round(stats.batch_time_s / stats.busy_s, 3) if stats.busy_s else None,
        "builds_checked": stats.builds_checked,
        "slow_enqueues": len(stats.slow_enqueues),
        "gc_passes": len(stats.gc_pauses_ms),
        "gc_pause_max_ms": max(stats.gc_pauses_ms) if stats.gc_pauses_ms else 0.0,
        "staging_wait_ms": round(stats.staging_wait_s * 1e3, 3),
        "slowest_enqueues": sorted(stats.slow_enqueues, key=lambda e: -e[4])[:5],
    }
