"""Request loop for matching queries against one resident data graph.

The library implements this loop natively (``cstm_server_*``, bound as
``cstm.Server``); ``replay_native`` drives it with a request stream.  The
``Server`` class below is the same policy over a pluggable backend, used to
test the policy on the host and to run it over custom backends.

Requests (query graphs) arrive one at a time.  The loop

* admits them in arrival order while their CSTs fit a device-memory budget
  (each request is charged an upper bound on its CST build from the label
  index, ``Graph.estimate_bytes``, doubled for the block cache's power-of-two
  rounding; a request larger than the whole budget is refused),
* builds each admitted request's CST as soon as it is admitted, on one of
  several builder threads with a stream each, while earlier requests are
  being enumerated,
* hands every built CST to the next free enumeration lane: a lane takes all
  CSTs built so far (up to ``max_batch``) and counts them in one persistent
  launch on its own stream (``batch_count``); with two or more lanes a new
  batch starts while a long one is still running, so requests that arrive
  while others are on the GPU overlap with them instead of queueing behind
  them,
* returns each request's count as soon as its batch ends, frees its CST and
  gives its memory back to admission.

Counts do not depend on which requests share a batch: each CST is counted on
its own, the batch only shares the launch.  ``run_sequential`` is the plain
form for comparison: one request at a time, build then count, in arrival order.

The device work goes through a backend object (``CstmBackend`` for the HIP
library); tests substitute a host-only backend to check the loop's logic.
"""

from __future__ import annotations

import collections
import math
import threading
import time

import numpy as np


class Request:
    __slots__ = ("rid", "query", "t_arrival", "t_admit", "t_built", "t_launch", "t_done", "count", "error",
                 "charge", "handle", "batch_size", "lane", "_event")

    def __init__(self, rid, query, t_arrival):
        self.rid = rid
        self.query = query
        self.t_arrival = t_arrival
        self.t_admit = self.t_built = self.t_launch = self.t_done = None
        self.count = None
        self.error = None
        self.charge = 0
        self.handle = None
        self.batch_size = 0
        self.lane = -1
        self._event = threading.Event()

    def wait(self, timeout=None) -> bool:
        return self._event.wait(timeout)

    @property
    def done(self) -> bool:
        return self._event.is_set()

    @property
    def latency(self) -> float | None:
        return None if self.t_done is None else self.t_done - self.t_arrival


class CstmBackend:
    """Device work of the loop through the HIP library."""

    def __init__(self, ctx, graph):
        import torch

        from . import cstm

        self._torch = torch
        self._cstm = cstm
        self.ctx = ctx
        self.graph = graph

    def new_stream(self):
        return self._torch.cuda.Stream(device=self.ctx.device)  # default priority

    def estimate(self, q) -> int:
        return 2 * self.graph.estimate_bytes(q.qlabel, q.qedges)

    def build(self, q, stream):
        return self._cstm.CST(self.ctx, self.graph, q.qlabel, q.qedges, stream=stream)

    def count_batch(self, handles, stream, limits=None):
        return self._cstm.batch_count(self.ctx, handles, stream=stream, limits=limits)

    def release(self, handle):
        handle.close()


class Server:
    """Continuous-batching loop (see the module docstring)."""

    def __init__(self, backend, *, mem_budget: int = 64 << 30, lanes: int = 2, builders: int = 4,
                 max_batch: int = 256, clock=time.perf_counter):
        if lanes < 1 or builders < 1:
            raise ValueError("lanes and builders must be at least 1")
        self.backend = backend
        self.mem_budget = int(mem_budget)
        self.max_batch = int(max_batch)
        self.clock = clock
        self._cv = threading.Condition()
        self._pending = collections.deque()  # arrived, not admitted
        self._ready = collections.deque()  # built, not launched
        self._in_use = 0  # bytes charged to admitted requests
        self._peak = 0
        self._busy_lanes = 0
        self._max_overlap = 0
        self._closing = False
        self._next_id = 0
        self.requests = []
        self.batches = []  # (lane, size, seconds)
        self._build_streams = [backend.new_stream() for _ in range(builders)]
        self._lane_streams = [backend.new_stream() for _ in range(lanes)]
        self._threads = [threading.Thread(target=self._build_loop, args=(st,), name=f"cstm-build{i}", daemon=True)
                         for i, st in enumerate(self._build_streams)]
        for i in range(lanes):
            self._threads.append(threading.Thread(target=self._lane_loop, args=(i,), name=f"cstm-lane{i}",
                                                  daemon=True))
        for t in self._threads:
            t.start()

    # ------------------------------------------------------------ client side

    def submit(self, query, t_arrival: float | None = None) -> Request:
        with self._cv:
            if self._closing:
                raise RuntimeError("server is closed")
            r = Request(self._next_id, query, self.clock() if t_arrival is None else t_arrival)
            self._next_id += 1
            self.requests.append(r)
            self._pending.append(r)
            self._cv.notify_all()
        return r

    def close(self, timeout: float | None = None):
        """Finish every submitted request, then stop the threads."""
        with self._cv:
            self._closing = True
            self._cv.notify_all()
        for t in self._threads:
            t.join(timeout)

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    @property
    def peak_bytes(self) -> int:
        """Largest total charge of admitted requests seen at one time."""
        return self._peak

    @property
    def max_overlap(self) -> int:
        """Most enumeration lanes that were running launches at one time."""
        return self._max_overlap

    # ------------------------------------------------------------ workers

    def _finish(self, r: Request, count=None, error=None):
        r.count = count
        r.error = error
        r.t_done = self.clock()
        if r.handle is not None:
            try:
                self.backend.release(r.handle)
            finally:
                r.handle = None
        with self._cv:
            self._in_use -= r.charge
            r.charge = 0
            self._cv.notify_all()
        r._event.set()

    def _build_loop(self, stream):
        while True:
            refuse = None
            with self._cv:
                while True:
                    while not self._pending and not self._closing:
                        self._cv.wait()
                    if not self._pending:
                        self._cv.notify_all()  # let the lanes see that no more work comes
                        return
                    r = self._pending[0]
                    if r.charge == 0:
                        try:
                            r.charge = max(1, int(self.backend.estimate(r.query)))
                        except Exception as e:  # malformed query
                            refuse = f"rejected: {e}"
                    if refuse is None and r.charge > self.mem_budget:
                        refuse = f"rejected: CST bound {r.charge} B exceeds the {self.mem_budget} B budget"
                    if refuse is not None:
                        self._pending.popleft()
                        r.charge = 0
                        break
                    # admission in arrival order: the head request waits until it fits
                    if self._in_use + r.charge <= self.mem_budget:
                        self._pending.popleft()
                        self._in_use += r.charge
                        self._peak = max(self._peak, self._in_use)
                        r.t_admit = self.clock()
                        break
                    self._cv.wait()
            if refuse is not None:
                self._finish(r, error=refuse)
                continue
            try:
                r.handle = self.backend.build(r.query, stream)
            except Exception as e:
                self._finish(r, error=f"build failed: {e}")
                continue
            r.t_built = self.clock()
            with self._cv:
                self._ready.append(r)
                self._cv.notify_all()

    def _lane_loop(self, lane: int):
        stream = self._lane_streams[lane]
        while True:
            with self._cv:
                while not self._ready and not (self._closing and self._drained()):
                    self._cv.wait()
                if not self._ready:
                    self._cv.notify_all()
                    return
                batch = []
                while self._ready and len(batch) < self.max_batch:
                    batch.append(self._ready.popleft())
                self._busy_lanes += 1
                self._max_overlap = max(self._max_overlap, self._busy_lanes)
            t0 = self.clock()
            for r in batch:
                r.t_launch = t0
                r.batch_size = len(batch)
                r.lane = lane
            try:
                counts = self.backend.count_batch([r.handle for r in batch], stream)
                err = None
            except Exception as e:
                counts, err = [None] * len(batch), f"enumeration failed: {e}"
            with self._cv:
                self._busy_lanes -= 1
            self.batches.append((lane, len(batch), self.clock() - t0))
            for r, c in zip(batch, counts):
                self._finish(r, count=None if err else int(c), error=err)

    def _drained(self) -> bool:
        # called with the lock held: nothing waits for admission and the builder is idle
        return not self._pending and all(r.t_built is not None or r.done for r in self.requests)


def run_sequential(backend, arrivals, queries, *, limit: int = 0, clock=time.perf_counter):
    """Plain form: one request at a time in arrival order, build then count on one stream.

    ``arrivals`` are offsets in seconds from the start; ``limit`` > 0 asks for
    min(total, limit); returns the requests."""
    stream = backend.new_stream()
    start = clock()
    out = []
    for rid, (t, q) in enumerate(zip(arrivals, queries)):
        now = clock() - start
        if now < t:
            time.sleep(t - now)
        r = Request(rid, q, start + t)
        r.t_admit = clock()
        h = backend.build(q, stream)
        r.t_built = r.t_launch = clock()
        try:
            r.count = int(backend.count_batch([h], stream, [limit] if limit else None)[0])
        except Exception as e:
            r.error = f"enumeration failed: {e}"
        finally:
            backend.release(h)
        r.t_done = clock()
        r.batch_size = 1
        r._event.set()
        out.append(r)
    return out


def replay(server: Server, arrivals, queries, *, clock=time.perf_counter):
    """Submit ``queries[i]`` at ``arrivals[i]`` seconds after the start; wait for all."""
    start = clock()
    reqs = []
    for t, q in zip(arrivals, queries):
        now = clock() - start
        if now < t:
            time.sleep(t - now)
        reqs.append(server.submit(q, t_arrival=start + t))
    for r in reqs:
        r.wait()
    return reqs


def replay_native(server, arrivals, queries, *, limit: int = 0, clock=time.perf_counter):
    """Submit ``queries[i]`` to a ``cstm.Server`` at ``arrivals[i]`` seconds after
    the start (each with the result limit ``limit``, 0 = all), wait for every
    result, and return them as ``Request`` records timed on the server's own
    clock (submission to result)."""
    start = clock()
    tickets = []
    for t, q in zip(arrivals, queries):
        now = clock() - start
        if now < t:
            time.sleep(t - now)
        tickets.append((server.submit(q.qlabel, q.qedges, limit), q))
    out = []
    for rid, (tk, q) in enumerate(tickets):
        res = server.wait(tk)
        r = Request(rid, q, res["submit_s"])
        r.t_admit = res["admit_s"]
        r.t_built = res["built_s"]
        r.t_launch = res["launch_s"]
        r.t_done = res["done_s"]
        r.batch_size = res["batch_size"]
        r.lane = res["lane"]
        if res["status"] == 0:
            r.count = int(res["count"])
        else:
            r.error = f"status {res['status']}"
        r._event.set()
        out.append(r)
    return out


def poisson_arrivals(n: int, qps: float, seed: int) -> np.ndarray:
    """Arrival offsets (seconds) of a Poisson process of rate ``qps``, seeded."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return np.cumsum(rng.exponential(1.0 / qps, size=n))


def nearest_rank(values, p: float) -> float:
    """The p-th percentile by the nearest-rank rule (p in (0, 100])."""
    v = sorted(values)
    if not v:
        return float("nan")
    return v[max(0, math.ceil(p / 100.0 * len(v)) - 1)]


def summarize(reqs) -> dict:
    ok = [r for r in reqs if r.error is None]
    lat = [r.latency for r in ok]
    span = (max(r.t_done for r in reqs) - min(r.t_arrival for r in reqs)) if reqs else 0.0
    total = sum(r.count for r in ok)
    def mean_ms(a, b):
        xs = [getattr(r, b) - getattr(r, a) for r in ok if getattr(r, a) is not None and getattr(r, b) is not None]
        return 1e3 * float(np.mean(xs)) if xs else None

    return {
        "requests": len(reqs),
        "completed": len(ok),
        "errors": len(reqs) - len(ok),
        "p50_ms": 1e3 * nearest_rank(lat, 50),
        "p99_ms": 1e3 * nearest_rank(lat, 99),
        # mean time per stage: waiting for admission, building, waiting for a lane, enumerating
        "mean_ms": {"admit_wait": mean_ms("t_arrival", "t_admit"), "build": mean_ms("t_admit", "t_built"),
                    "launch_wait": mean_ms("t_built", "t_launch"), "enumerate": mean_ms("t_launch", "t_done")},
        "mean_batch": float(np.mean([r.batch_size for r in ok])) if ok else 0.0,
        "embeddings": total,
        "seconds": span,
        "embeddings_per_s": total / span if span > 0 else 0.0,
    }
