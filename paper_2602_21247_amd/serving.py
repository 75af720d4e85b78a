"""Serving: continuous batching of insertions and k-NN queries over an index
resident in HBM.

The host scheduler only batches and orders; every step of a request runs in
the library (pipnn_insert, pipnn_search). Two host threads drive two HIP
streams, so query batches and insert batches overlap on the device:

- the query thread admits arrived queries (in arrival order, up to a batch
  limit and a scratch-memory budget), searches them as one batch against the
  most recently published graph, and records each request's epoch (the
  number of insert batches committed before it) and completion time;
- the insert thread admits arrived insertion requests (while the reserved
  capacity and the batch limit allow), appends their points to X, inserts
  them as one pipnn_insert call with one group per request (so each request
  links only to the index and to its own points), and publishes the updated
  graph into the spare of two graph copies that queries read.

Admission by memory: a query batch is limited by the free HBM its visited
bitmaps need; an insertion that does not fit the reserved capacity grows it
(new X, reservoirs, graph copies and the index's per-point buffers, by
pipnn_reserve with the new X) when the free HBM (hipMemGetInfo, plus what
torch holds cached) covers the growth, with query batches paused while the
buffers are swapped; otherwise the insertion is deferred and retried as
memory frees, and rejected after a timeout.

A request arriving while a batch is on the GPU is admitted by the next batch
of its kind as soon as the thread is free: continuous batching, not a
queue drained between batches. Each query's result depends only on its
epoch's graph, and each insertion's effect only on its own points (HashPrune
does not depend on the order of its records), so results are the same alone
and in the mix.

The threading contract of the library that this relies on: pipnn_search and
pipnn_insert may run at the same time on one index from two threads and two
streams; nothing else overlaps.
"""
from __future__ import annotations

import threading
import time
from dataclasses import dataclass, field

import numpy as np


@dataclass
class Request:
    rid: int
    kind: str            # "insert" or "query"
    arrival: float       # seconds after the start of the run
    data: np.ndarray     # points (insert) or queries (query), rows x d
    k: int = 10


@dataclass
class Result:
    rid: int
    kind: str
    arrival: float
    admitted: float = 0.0
    done: float = 0.0
    epoch: int = -1      # insert batches committed before it ran (queries)
    batch: int = -1      # sequence number of the batch that served it
    ids: np.ndarray | None = None
    dist: np.ndarray | None = None
    first_id: int = -1   # first point id given to an insertion
    status: str = "ok"   # "ok", or "rejected" (no memory for the growth it needed)

    @property
    def latency(self) -> float:
        return self.done - self.arrival


@dataclass
class ServerConfig:
    L: int = 64                    # beam width of the queries
    max_query_batch: int = 4096    # queries per search launch
    max_insert_batch: int = 65536  # points per insert launch
    query_scratch_bytes: int = 1 << 30  # at most this much of visited bitmaps per batch
    hbm_keep_bytes: int = 2 << 30  # free HBM that admission leaves untouched
    grow_factor: float = 1.25      # capacity after a growth: at least this times the old
    defer_timeout_s: float = 5.0   # an insertion waiting this long for memory is rejected


def free_hbm_bytes(torch) -> int:
    """Free device memory: what the driver reports (hipMemGetInfo) plus what
    torch's caching allocator holds unused."""
    free, _ = torch.cuda.mem_get_info()
    return int(free) + int(torch.cuda.memory_reserved() - torch.cuda.memory_allocated())


class Server:
    """Continuous batching over an index built by the caller.

    X_cap: device tensor with room for the capacity (the index was created
    on its first n rows and reserved to X_cap.shape[0]); res / graph /
    degree: device buffers of the same capacity, holding the build."""

    def __init__(self, idx, X_cap, res, graph, degree, start: int, cfg: ServerConfig):
        import torch
        self.torch = torch
        self.idx, self.X, self.res, self.g, self.deg = idx, X_cap, res, graph, degree
        self.start = int(start)
        self.cfg = cfg
        self.cap = X_cap.shape[0]
        self.n = idx.n
        # two published copies of the graph; queries read pub[cur]
        self.pub = [graph.clone(), graph.clone()]
        self.cur = 0
        self.pub_n = self.n
        self.epoch = 0
        self.readers = [0, 0]             # query batches in flight on each copy
        self.growing = False              # buffers are being swapped: no query starts
        self.growths = []                 # (new capacity, seconds) of each growth
        self.rejected = 0
        self.s_q = torch.cuda.Stream()
        self.s_i = torch.cuda.Stream()
        self.lock = threading.Condition()
        self.error: BaseException | None = None

    # ---- admission
    def _query_batch(self, pending, now):
        """Arrived queries in arrival order while the batch limit and the
        memory for their visited bitmaps (n bits per query) allow."""
        per_q = ((self.pub_n + 31) // 32) * 4
        budget = min(self.cfg.query_scratch_bytes,
                     max(0, free_hbm_bytes(self.torch) - self.cfg.hbm_keep_bytes))
        limit = min(self.cfg.max_query_batch, max(1, budget // per_q))
        out, tot = [], 0
        while pending and pending[0].arrival <= now and tot + len(pending[0].data) <= limit:
            r = pending.pop(0)
            out.append(r)
            tot += len(r.data)
        if not out and pending and pending[0].arrival <= now:
            out.append(pending.pop(0))   # a single request over the limit runs alone
        return out

    def _insert_batch(self, pending, now):
        out, tot = [], 0
        while pending and pending[0].arrival <= now:
            m = len(pending[0].data)
            if self.n + tot + m > self.cap or (out and tot + m > self.cfg.max_insert_batch):
                break
            out.append(pending.pop(0))
            tot += m
        return out

    def _growth_bytes(self, new_cap: int) -> int:
        """Device memory a growth to new_cap takes while the old buffers still
        exist: X, reservoirs, the graph and its two published copies, degrees,
        and the index's own per-point buffers (pipnn_workspace_bytes' bound)."""
        row = (self.X.shape[1] * self.X.element_size() + self.res.shape[1] * 8
               + 3 * self.g.shape[1] * 4 + 4)
        idx_b = self.idx.workspace_bytes(new_cap)
        return new_cap * row + idx_b

    def _grow(self, need: int) -> bool:
        """Grow the capacity to hold `need` points if the free HBM allows;
        query batches are paused while the buffers are swapped."""
        torch = self.torch
        new_cap = max(need, int(self.cap * self.cfg.grow_factor))
        if self._growth_bytes(new_cap) + self.cfg.hbm_keep_bytes > free_hbm_bytes(torch):
            return False
        t0 = time.perf_counter()
        with self.lock:
            self.growing = True
            while self.readers[0] or self.readers[1]:
                self.lock.wait()
        try:
            torch.cuda.synchronize()
            n = self.n
            X = torch.empty((new_cap, self.X.shape[1]), dtype=self.X.dtype, device="cuda")
            X[:n].copy_(self.X[:n])
            res = torch.empty((new_cap, self.res.shape[1]), dtype=self.res.dtype, device="cuda")
            res[:n].copy_(self.res[:n])
            g = torch.full((new_cap, self.g.shape[1]), -1, dtype=self.g.dtype, device="cuda")
            g[:n].copy_(self.g[:n])
            deg = torch.zeros(new_cap, dtype=self.deg.dtype, device="cuda")
            deg[:n].copy_(self.deg[:n])
            self.idx.reserve(new_cap, X=X)
            self.X, self.res, self.g, self.deg = X, res, g, deg
            self.pub = [g.clone(), g.clone()]
            self.cap = new_cap
            torch.cuda.synchronize()
        finally:
            with self.lock:
                self.growing = False
                self.lock.notify_all()
        self.growths.append((new_cap, time.perf_counter() - t0))
        return True

    # ---- the two workers
    def _run_queries(self, pending, results, t0, seq):
        torch = self.torch
        while pending:
            now = time.perf_counter() - t0
            if pending[0].arrival > now:
                time.sleep(min(1e-4, pending[0].arrival - now))
                continue
            with self.lock:
                while self.growing:
                    self.lock.wait()
            batch = self._query_batch(pending, now)
            adm = time.perf_counter() - t0
            with self.lock:
                while self.growing:
                    self.lock.wait()
                cur, epoch = self.cur, self.epoch
                self.readers[cur] += 1
            Q = np.concatenate([r.data for r in batch]).astype(np.float32, copy=False)
            k = max(r.k for r in batch)
            with torch.cuda.stream(self.s_q):
                Qd = torch.from_numpy(Q).to("cuda", non_blocking=False)
                ids, dist, _ = self.idx.search(self.pub[cur], Qd, k, max(k, self.cfg.L),
                                               self.start)
                ev = torch.cuda.Event()
                ev.record(self.s_q)
            ev.synchronize()
            done = time.perf_counter() - t0
            with self.lock:
                self.readers[cur] -= 1
                self.lock.notify_all()
            ids_h, dist_h = ids.cpu().numpy().view(np.uint32), dist.cpu().numpy()
            o = 0
            b = seq[0]
            seq[0] += 1
            for r in batch:
                m = len(r.data)
                results[r.rid] = Result(r.rid, "query", r.arrival, adm, done, epoch, b,
                                        ids_h[o:o + m, :r.k].copy(), dist_h[o:o + m, :r.k].copy())
                o += m

    def _run_inserts(self, pending, results, t0, seq):
        torch = self.torch
        while pending:
            now = time.perf_counter() - t0
            if pending[0].arrival > now:
                time.sleep(min(1e-4, pending[0].arrival - now))
                continue
            batch = self._insert_batch(pending, now)
            if not batch:
                # the first arrived request does not fit: grow, or defer it
                # until memory frees, or reject it after the timeout
                r = pending[0]
                if not self._grow(self.n + len(r.data)):
                    if now - r.arrival > self.cfg.defer_timeout_s:
                        pending.pop(0)
                        self.rejected += 1
                        results[r.rid] = Result(r.rid, "insert", r.arrival, now, now,
                                                status="rejected")
                    else:
                        time.sleep(1e-3)
                continue
            adm = time.perf_counter() - t0
            P = np.concatenate([r.data for r in batch])
            groups = np.concatenate([np.full(len(r.data), i, dtype=np.int32)
                                     for i, r in enumerate(batch)])
            n0, m = self.n, len(P)
            with torch.cuda.stream(self.s_i):
                self.X[n0:n0 + m].copy_(torch.from_numpy(P).to(self.X.dtype))
                gd = torch.from_numpy(groups).cuda()
                # the snapshot this batch publishes is the next epoch
                self.idx.insert(m, self.res, self.g, self.deg, gd, epoch=self.epoch + 1)
                self.n = n0 + m
                # publish into the spare copy once no query batch reads it
                with self.lock:
                    spare = 1 - self.cur
                    while self.readers[spare] > 0:
                        self.lock.wait()
                self.pub[spare].copy_(self.g)
                ev = torch.cuda.Event()
                ev.record(self.s_i)
            ev.synchronize()
            done = time.perf_counter() - t0
            with self.lock:
                self.cur = spare
                self.pub_n = self.n
                self.epoch += 1
            b = seq[0]
            seq[0] += 1
            o = n0
            for r in batch:
                results[r.rid] = Result(r.rid, "insert", r.arrival, adm, done, -1, b,
                                        first_id=o)
                o += len(r.data)

    def run(self, requests: list[Request]) -> dict[int, Result]:
        """Serve the requests at their arrival times; returns results by id."""
        reqs = sorted(requests, key=lambda r: (r.arrival, r.rid))
        qs = [r for r in reqs if r.kind == "query"]
        ins = [r for r in reqs if r.kind == "insert"]
        results: dict[int, Result] = {}
        t0 = time.perf_counter()
        qseq, iseq = [0], [0]

        def guard(fn, *a):
            try:
                fn(*a)
            except BaseException as e:  # surfaced after the join
                self.error = e

        ti = threading.Thread(target=guard, args=(self._run_inserts, ins, results, t0, iseq))
        ti.start()
        guard(self._run_queries, qs, results, t0, qseq)
        ti.join()
        if self.error is not None:
            raise self.error
        return results


def summarize(results: dict[int, Result], wall_s: float) -> dict:
    """p50/p99 latency per request class, inserts/s and QPS."""
    out = {}
    for kind in ("query", "insert"):
        lat = np.array([r.latency for r in results.values()
                        if r.kind == kind and r.status == "ok"])
        if len(lat):
            out[kind] = {"count": int(len(lat)), "p50_ms": float(np.percentile(lat, 50) * 1e3),
                         "p99_ms": float(np.percentile(lat, 99) * 1e3),
                         "mean_ms": float(lat.mean() * 1e3)}
    return out
