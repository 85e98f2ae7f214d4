"""Serving loop for viewport aggregation queries (continuous batching).

Interactive exploration zooms in and out (Sec. 1, level-of-detail
exploration) and wants answers at the resolution of the screen: a query is a
square viewport, a distance bound eps (one pixel), a polygon set and COUNT or
SUM.  The server keeps the point table resident in HBM (reordered into a
bucket grid so a viewport is one contiguous range per bucket row), and for
every query

1. admits the query's approximation build once its memory estimate fits the
   budget (queries wait, they do not fail, unless a single query can never
   fit),
2. builds the approximation of the polygon set clipped to the viewport on a
   build stream (builds overlap with running probes on the device),
3. joins the ready queries into one batch: one persistent launch of
   ``sba_aggregate_batch`` over all their point ranges, on the probe stream,
   while later arrivals keep being admitted and built,
4. on completion copies the per-polygon results to the host, releases the
   approximation and its memory, and resolves the query's future.

The control plane is Python; every step on the data runs in libsba's kernels.
"""
from __future__ import annotations

import collections
import concurrent.futures as cf
import dataclasses
import threading
import time

import numpy as np

from . import Approx, Task, aggregate_batch, bucket_points


@dataclasses.dataclass
class Query:
    vx: int
    vy: int
    vw: int
    eps: int
    set_id: int
    agg: str = "count"          # "count" or "sum"


@dataclasses.dataclass
class Result:
    counts: np.ndarray
    sums: np.ndarray | None
    latency_ms: float
    build_ms: float
    points_scanned: int


class Rejected(RuntimeError):
    pass


class _Job:
    __slots__ = ("q", "fut", "t_arrival", "est", "approx", "ranges", "counts", "sums", "t_built",
                 "build_ms", "npts")

    def __init__(self, q, fut, t):
        self.q, self.fut, self.t_arrival = q, fut, t
        self.est = 0
        self.approx = None
        self.ranges = []
        self.counts = self.sums = None
        self.t_built = 0.0
        self.build_ms = 0.0
        self.npts = 0


class Server:
    """Viewport query server over one resident point table.

    xy (int32 [2n]) and values (int64 [n]) are GPU tensors; polygon_sets is
    a list of objects with ring_off / vert_off / xy arrays.  box = (x0, y0,
    side) is the extent the bucket grid covers (G x G buckets).
    """

    def __init__(self, xy, values, polygon_sets, box, G: int = 256, mem_budget: int | None = None,
                 max_batch: int = 256, kind: str = "grid", builders: int = 4,
                 max_inflight: int = 1, budget_fraction: float = 0.5):
        import torch
        self.torch = torch
        self.dev = xy.device
        x0, y0, side = box
        self.box = box
        self.G = G
        self.cell = max(1, -(-int(side) // G))
        self.probe_stream = torch.cuda.Stream(device=self.dev)
        self.build_streams = [torch.cuda.Stream(device=self.dev) for _ in range(max(1, builders))]
        t0 = time.perf_counter()
        with torch.cuda.stream(self.probe_stream):
            self.xy, self.values, off = bucket_points(xy, values, x0, y0, self.cell, G,
                                                      stream=self.probe_stream)
        self.probe_stream.synchronize()
        self.bucket_off = off.cpu().numpy()
        self.prep_ms = 1000.0 * (time.perf_counter() - t0)
        self.sets = []
        for ps in polygon_sets:
            self.sets.append((torch.from_numpy(np.ascontiguousarray(ps.ring_off)).to(self.dev),
                              torch.from_numpy(np.ascontiguousarray(ps.vert_off)).to(self.dev),
                              torch.from_numpy(np.ascontiguousarray(ps.xy)).to(self.dev),
                              int(ps.n_polys), int(ps.xy.shape[0] // 2)))
        self.kind = kind
        # admission budget: the given bytes, or a fraction of the device
        # memory free once the point table and its bucketed copy are resident
        # (hipMemGetInfo through torch)
        if mem_budget is None:
            free, _ = torch.cuda.mem_get_info(self.dev)
            mem_budget = int(budget_fraction * free)
        self.budget = int(mem_budget)
        self.reserved = 0
        self.peak_reserved = 0
        self.max_batch = max_batch
        self._lock = threading.Condition()
        self._pending = collections.deque()
        self._ready = collections.deque()
        self._stop = False
        self.batches = []             # (n_queries, n_tasks) per launch
        self.max_inflight = max(1, max_inflight)
        self._paused = False
        self._inflight_jobs = []
        self._builders = [threading.Thread(target=self._build_loop, args=(st,), daemon=True)
                          for st in self.build_streams]
        self._batcher = threading.Thread(target=self._batch_loop, daemon=True)
        for t in self._builders:
            t.start()
        self._batcher.start()

    # ------------------------------------------------------------ helpers
    def estimate_bytes(self, q: Query) -> int:
        """Device bytes a query's build and probe may hold at once, an upper
        estimate: 8 B per viewport cell (a cell side of eps / 1.5 undercuts
        the real one), 192 B per vertex of the polygon set (the build's edge,
        event and sort arrays cover every vertex before the window cuts
        them), 64 B per polygon and 4 MB.  A GPU test holds it against the
        peak a build really takes over the serving query mix (at most two
        thirds of the estimate there)."""
        s = max(1, int(q.eps / 1.5))
        cells = (q.vw // s + 3) ** 2
        nv = self.sets[q.set_id][4]
        np_ = self.sets[q.set_id][3]
        return int(8 * cells + 192 * nv + 64 * np_ + (4 << 20))

    def ranges_of(self, q: Query):
        """Point index ranges whose buckets meet the viewport (one per bucket row)."""
        x0, y0, _ = self.box
        G, c = self.G, self.cell
        bx0 = min(G - 1, max(0, (q.vx - x0) // c))
        bx1 = min(G - 1, max(0, (q.vx + q.vw - 1 - x0) // c))
        by0 = min(G - 1, max(0, (q.vy - y0) // c))
        by1 = min(G - 1, max(0, (q.vy + q.vw - 1 - y0) // c))
        off = self.bucket_off
        out = []
        for by in range(by0, by1 + 1):
            a, b = int(off[by * G + bx0]), int(off[by * G + bx1 + 1])
            if b > a:
                if out and out[-1][1] == a:
                    out[-1] = (out[-1][0], b)
                else:
                    out.append((a, b))
        return out

    # ------------------------------------------------------------ public
    def submit(self, q: Query) -> cf.Future:
        fut = cf.Future()
        job = _Job(q, fut, time.perf_counter())
        job.est = self.estimate_bytes(q)
        if job.est > self.budget:
            fut.set_exception(Rejected(f"query needs ~{job.est} B, budget is {self.budget} B"))
            return fut
        with self._lock:
            self._pending.append(job)
            self._lock.notify_all()
        return fut

    def pause(self):
        """Stop launching batches (admission and builds go on)."""
        with self._lock:
            self._paused = True

    def resume(self):
        with self._lock:
            self._paused = False
            self._lock.notify_all()

    def n_ready(self) -> int:
        with self._lock:
            return len(self._ready)

    def _builders_alive(self):
        return any(t.is_alive() for t in self._builders)

    def close(self):
        self.resume()
        with self._lock:
            self._stop = True
            self._lock.notify_all()
        for t in self._builders:
            t.join()
        self._batcher.join()

    # ------------------------------------------------------------ threads
    def _build_loop(self, stream):
        torch = self.torch
        while True:
            with self._lock:
                while ((self._pending and self.reserved + self._pending[0].est > self.budget)
                       or (not self._pending and not self._stop)):
                    if self._pending and self._pending[0].fut.cancelled():
                        self._pending.popleft()
                        continue
                    self._lock.wait(0.05)
                if self._stop and not self._pending:
                    return
                if not self._pending:
                    continue
                job = self._pending.popleft()
                if job.fut.cancelled() or not job.fut.set_running_or_notify_cancel():
                    continue
                self.reserved += job.est
                self.peak_reserved = max(self.peak_reserved, self.reserved)
            try:
                q = job.q
                ro, vo, pxy, np_, _ = self.sets[q.set_id]
                win = (q.vx, q.vy, q.vx + q.vw, q.vy + q.vw)
                t0 = time.perf_counter()
                with torch.cuda.stream(stream):
                    job.approx = Approx(ro, vo, pxy, q.eps, kind=self.kind, window=win,
                                        stream=stream)
                job.build_ms = 1000.0 * (time.perf_counter() - t0)
                job.ranges = self.ranges_of(q)
                job.npts = sum(b - a for a, b in job.ranges)
                job.t_built = time.perf_counter()
            except Exception as e:  # noqa: BLE001 - reported through the future
                self._release(job)
                job.fut.set_exception(e)
                continue
            with self._lock:
                self._ready.append(job)
                self._lock.notify_all()

    def _release(self, job):
        with self._lock:
            self.reserved -= job.est
            self._lock.notify_all()

    def _ready_nonempty(self):
        with self._lock:
            return bool(self._ready)

    def _batch_loop(self):
        try:
            self._batch_loop_body()
        except BaseException as e:  # noqa: BLE001 - fail every waiting query, never hang
            self._fail_all(e)
            raise

    def _fail_all(self, exc):
        with self._lock:
            self._stop = True
            jobs = list(self._pending) + list(self._ready)
            self._pending.clear()
            self._ready.clear()
            self._lock.notify_all()
        for job in jobs + list(self._inflight_jobs):
            if not job.fut.done():
                job.fut.set_exception(RuntimeError(f"server failed: {exc!r}"))

    def _batch_loop_body(self):
        torch = self.torch
        inflight = collections.deque()   # (event, jobs), in launch order
        self._inflight_jobs = []
        while True:
            # complete finished launches, in order
            while inflight and inflight[0][0].query():
                self._finish(*inflight.popleft())
                self._inflight_jobs = [j for _, b in inflight for j in b]
            with self._lock:
                can_launch = (self._ready and not self._paused
                              and (len(inflight) < self.max_inflight
                                   or len(self._ready) >= self.max_batch))
                if not can_launch:
                    if (self._stop and not inflight and not self._ready and not self._pending
                            and not self._builders_alive()):
                        return
                    self._lock.wait(0.0002 if inflight else 0.002)
                    continue
                batch = []
                while self._ready and len(batch) < self.max_batch:
                    batch.append(self._ready.popleft())
            tasks = []
            for job in batch:
                np_ = max(job.approx.n_polys, 1)
                job.counts = torch.empty(np_, dtype=torch.int64, device=self.dev)
                job.sums = (torch.empty(np_, dtype=torch.int64, device=self.dev)
                            if job.q.agg == "sum" else None)
                vals = self.values if job.q.agg == "sum" else None
                view = (job.q.vx, job.q.vy, job.q.vw, job.q.vw)
                for a, b in (job.ranges or [(0, 0)]):
                    tasks.append(Task(job.approx, self.xy, vals, a, b, view, job.counts,
                                      job.sums))
            with torch.cuda.stream(self.probe_stream):
                aggregate_batch(tasks, stream=self.probe_stream)
                ev = torch.cuda.Event()
                ev.record(self.probe_stream)
            self.batches.append((len(batch), len(tasks)))
            inflight.append((ev, batch))
            self._inflight_jobs = [j for _, b in inflight for j in b]

    def _finish(self, ev, jobs):
        ev.synchronize()
        for job in jobs:
            c = job.counts.cpu().numpy()[:job.approx.n_polys]
            s = job.sums.cpu().numpy()[:job.approx.n_polys] if job.sums is not None else None
            lat = 1000.0 * (time.perf_counter() - job.t_arrival)
            n = job.npts
            job.approx.close(sync=False)   # its batch has completed
            job.approx = None
            self._release(job)
            job.fut.set_result(Result(c, s, lat, job.build_ms, n))


def latency_summary(results) -> dict:
    lat = np.array([r.latency_ms for r in results])
    return {"n": int(lat.size), "p50_ms": float(np.percentile(lat, 50)),
            "p99_ms": float(np.percentile(lat, 99)), "mean_ms": float(lat.mean()),
            "max_ms": float(lat.max())}
