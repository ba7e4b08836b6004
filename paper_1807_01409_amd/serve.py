"""Continuous-batching query server over a graph resident in HBM.

Requests arrive on a clock (open loop).  A dispatcher admits waiting
requests in arrival order while the estimated device bytes of everything in
flight stay under a budget (tid_plan_estimate), and hands each admitted group
to a free worker.  Every worker owns a library context and its own HIP
stream, so the batches of different workers run on the device at the same
time; a request that arrives while others are running joins the next group
as soon as a worker and budget free up.  Each group runs as one
tid_query_batch call, whose results are exactly those of tid_query alone.
"""
from __future__ import annotations

import collections
import queue
import threading
import time
from dataclasses import dataclass, field
from typing import Callable, List, Optional, Sequence

import numpy as np

from .tid import Context, Graph, TidError


@dataclass
class Request:
    rid: int
    plan: object
    arrival: float          # seconds from the start of the run
    est_bytes: int = 0
    admitted: float = -1.0
    done: float = -1.0
    rows: int = -1
    result: Optional[np.ndarray] = None
    error: str = ""             # set when the request failed (it is not retried again)


@dataclass
class ServeStats:
    completed: int
    wall_s: float
    qps: float
    p50_ms: float
    p99_ms: float
    mean_batch: float
    max_inflight_bytes: int
    max_queue: int
    latencies_ms: List[float] = field(default_factory=list)
    failed: int = 0             # requests that failed alone after their group failed


class Server:
    """Workers share one resident graph (read only) loaded by the first context.
    layout: also build the graph's predicate-partitioned columns, so that the
    patterns with a constant predicate read only their predicates' slices."""

    def __init__(self, triples, workers: int = 4, budget_bytes: int = 64 << 30,
                 max_batch: int = 256, allocator: str = "pool", device: int = 0,
                 layout: bool = True):
        self.ctxs = [Context(device, allocator=allocator) for _ in range(workers)]
        self.graph: Graph = self.ctxs[0].load(triples)
        if layout:
            self.graph.partition(True)
        self.budget = int(budget_bytes)
        self.max_batch = int(max_batch)
        self._jobs: "queue.Queue" = queue.Queue()
        self._done: "queue.Queue" = queue.Queue()
        self._threads = []
        self._keep = False
        self._t0 = 0.0
        for w in range(workers):
            th = threading.Thread(target=self._worker, args=(w,), daemon=True)
            th.start()
            self._threads.append(th)

    # -- workers ------------------------------------------------------------
    def _worker(self, w: int):
        ctx = self.ctxs[w]
        while True:
            batch = self._jobs.get()
            if batch is None:
                return
            try:
                tabs = ctx.query_batch(self.graph, [r.plan for r in batch])
                for r, t in zip(batch, tabs):
                    if self._keep is True or (self._keep and r.rid in self._keep):
                        r.result = t.to_numpy()
                        r.rows = r.result.shape[0]
                    else:
                        r.rows = t.nrows
                    t.free()
                err = None
            except TidError as e:
                # A group that ran out of device memory (or hit another library
                # error) is retried one request at a time, so that one large
                # request fails alone and the others are still served.
                err = None
                for r in batch:
                    try:
                        t = ctx.query(self.graph, r.plan)
                        if self._keep is True or (self._keep and r.rid in self._keep):
                            r.result = t.to_numpy()
                            r.rows = r.result.shape[0]
                        else:
                            r.rows = t.nrows
                        t.free()
                    except TidError as e1:
                        r.error = str(e1)
                        r.rows = -1
            except Exception as e:  # noqa: BLE001 - reported to the dispatcher
                err = e
            now = time.perf_counter() - self._t0
            for r in batch:
                r.done = now
            self._done.put((w, batch, err))

    def close(self):
        for _ in self._threads:
            self._jobs.put(None)
        for th in self._threads:
            th.join()
        self.graph.free()
        for c in self.ctxs:
            c.close()

    # -- dispatcher ----------------------------------------------------------
    def run(self, requests: Sequence[Request], keep_results=False,
            warmup_s: float = 0.0) -> ServeStats:
        """Serve `requests` (sorted by arrival) in real time; returns latency
        and throughput over the requests arriving after `warmup_s`.
        keep_results: True keeps every result on the host (Request.result), a
        set of request ids keeps those only, False keeps row counts alone."""
        ctx0 = self.ctxs[0]
        for r in requests:
            r.est_bytes = ctx0.plan_estimate(self.graph, r.plan)
        self._keep = keep_results
        reqs = sorted(requests, key=lambda r: r.arrival)
        waiting: "collections.deque[Request]" = collections.deque()
        free = len(self.ctxs)
        inflight = 0
        nxt = 0
        finished = 0
        batches = []
        max_inflight = 0
        max_queue = 0
        self._t0 = time.perf_counter()
        while finished < len(reqs):
            now = time.perf_counter() - self._t0
            while nxt < len(reqs) and reqs[nxt].arrival <= now:
                waiting.append(reqs[nxt])
                nxt += 1
            max_queue = max(max_queue, len(waiting))
            # admit in arrival order while a worker and budget are free; a
            # request larger than the budget runs alone when nothing else does
            while free and waiting:
                group = []
                while waiting and len(group) < self.max_batch:
                    r = waiting[0]
                    if inflight + r.est_bytes > self.budget and (group or inflight):
                        break
                    group.append(waiting.popleft())
                    inflight += r.est_bytes
                if not group:
                    break
                t_adm = time.perf_counter() - self._t0
                for r in group:
                    r.admitted = t_adm
                self._jobs.put(group)
                batches.append(len(group))
                free -= 1
            max_inflight = max(max_inflight, inflight)
            # wait for a completion or the next arrival
            timeout = 0.05
            if nxt < len(reqs):
                timeout = max(0.0, min(timeout, reqs[nxt].arrival - now))
            try:
                w, batch, err = self._done.get(timeout=timeout if timeout > 0 else 1e-4)
            except queue.Empty:
                continue
            if err is not None:
                raise err
            free += 1
            for r in batch:
                inflight -= r.est_bytes
            finished += len(batch)
        wall = time.perf_counter() - self._t0
        meas = [r for r in reqs if r.arrival >= warmup_s]
        lat = np.array([(r.done - r.arrival) * 1e3 for r in meas]) if meas else np.zeros(1)
        span = (max(r.done for r in meas) - warmup_s) if meas else wall
        return ServeStats(completed=len(meas), wall_s=wall,
                          qps=len(meas) / span if span > 0 else 0.0,
                          p50_ms=float(np.percentile(lat, 50)),
                          p99_ms=float(np.percentile(lat, 99)),
                          mean_batch=float(np.mean(batches)) if batches else 0.0,
                          max_inflight_bytes=int(max_inflight), max_queue=int(max_queue),
                          latencies_ms=lat.tolist(), failed=sum(1 for r in reqs if r.error))



class CircularServer:
    """Serving with the library's circular chunked shared scan (tid_serve_*).

    The resident graph is cut into `chunks` contiguous chunks scanned one per
    step, round and round, for every admitted query; a query is admitted at a
    chunk boundary into one of `slots` slots (while the estimated bytes of the
    queries in flight stay under the budget) and finishes one revolution
    later, its joins and other ops run with those of the queries finishing at
    the same step.  Results equal tid_query's."""

    def __init__(self, triples, chunks: int = 16, slots: int = 512,
                 budget_bytes: int = 64 << 30, device: int = 0):
        import ctypes

        from . import _lib as L
        from .tid import _check
        self._ct = ctypes
        self._L = L
        self._check = _check
        self.ctx = Context(device)
        self.graph: Graph = self.ctx.load(triples)
        self.budget = int(budget_bytes)
        self.slots = int(slots)
        out = ctypes.c_void_p()
        _check(self.ctx.ptr, self.ctx._lib.tid_serve_open(self.ctx.ptr, self.graph._p, int(chunks),
                                                          self.slots, ctypes.byref(out)))
        self._s = out
        self.chunks = int(chunks)

    def close(self):
        if self._s:
            self.ctx._lib.tid_serve_close(self._s)
            self._s = None
        self.graph.free()
        self.ctx.close()

    def _submit(self, plan) -> int:
        from .tid import _plan
        keep: list = []
        cp = _plan(plan, keep)
        t = self._ct.c_uint64()
        self._check(self.ctx.ptr, self.ctx._lib.tid_serve_submit(self._s, self._ct.byref(cp),
                                                                 self._ct.byref(t)))
        return int(t.value)

    def _step(self) -> List[int]:
        buf = (self._ct.c_uint64 * self.slots)()
        n = self._ct.c_int32()
        self._check(self.ctx.ptr, self.ctx._lib.tid_serve_step(self._s, buf, self.slots,
                                                               self._ct.byref(n)))
        return [int(buf[i]) for i in range(n.value)]

    def _result(self, ticket: int):
        from .tid import Table, TidError
        out = self._ct.c_void_p()
        st = self.ctx._lib.tid_serve_result(self._s, ticket, self._ct.byref(out))
        if st != 0:
            raise TidError(st, self.ctx._lib.tid_last_error(self.ctx.ptr).decode())
        return Table(self.ctx, out)

    def run(self, requests: Sequence[Request], keep_results=False,
            warmup_s: float = 0.0) -> ServeStats:
        from .tid import TidError
        for r in requests:
            r.est_bytes = self.ctx.plan_estimate(self.graph, r.plan)
        reqs = sorted(requests, key=lambda r: r.arrival)
        waiting: "collections.deque[Request]" = collections.deque()
        inflight: dict = {}
        inflight_bytes = 0
        nxt = finished = 0
        steps = max_queue = max_inflight = 0
        t0 = time.perf_counter()
        while finished < len(reqs):
            now = time.perf_counter() - t0
            while nxt < len(reqs) and reqs[nxt].arrival <= now:
                waiting.append(reqs[nxt])
                nxt += 1
            max_queue = max(max_queue, len(waiting))
            # admit in arrival order while slots and budget allow; a request
            # larger than the budget runs alone when nothing else does
            while waiting and len(inflight) < self.slots:
                r = waiting[0]
                if inflight_bytes + r.est_bytes > self.budget and inflight:
                    break
                waiting.popleft()
                r.admitted = time.perf_counter() - t0
                inflight[self._submit(r.plan)] = r
                inflight_bytes += r.est_bytes
            max_inflight = max(max_inflight, inflight_bytes)
            if not inflight:
                if nxt < len(reqs):
                    time.sleep(max(0.0, min(0.001, reqs[nxt].arrival - now)))
                continue
            done = self._step()
            steps += 1
            tnow = time.perf_counter() - t0
            for tk in done:
                r = inflight.pop(tk)
                inflight_bytes -= r.est_bytes
                try:
                    t = self._result(tk)
                    if keep_results is True or (keep_results and r.rid in keep_results):
                        r.result = t.to_numpy()
                        r.rows = r.result.shape[0]
                    else:
                        r.rows = t.nrows
                    t.free()
                except TidError as e:
                    r.error = str(e)
                r.done = tnow
                finished += 1
        wall = time.perf_counter() - t0
        meas = [r for r in reqs if r.arrival >= warmup_s]
        lat = np.array([(r.done - r.arrival) * 1e3 for r in meas]) if meas else np.zeros(1)
        span = (max(r.done for r in meas) - warmup_s) if meas else wall
        return ServeStats(completed=len(meas), wall_s=wall,
                          qps=len(meas) / span if span > 0 else 0.0,
                          p50_ms=float(np.percentile(lat, 50)),
                          p99_ms=float(np.percentile(lat, 99)),
                          mean_batch=float(len(reqs)) / max(steps, 1) * self.chunks,
                          max_inflight_bytes=int(max_inflight), max_queue=int(max_queue),
                          latencies_ms=lat.tolist(), failed=sum(1 for r in reqs if r.error))
