"""Driving the library's request server and its one-at-a-time baseline.

The serving loop itself is native (``cstm_server_*``, bound as
``cstm.Server``): it admits requests in arrival order while their CSTs fit a
device-memory budget, builds admitted CSTs on builder threads (a stream
each), and hands built CSTs to enumeration lanes that count everything built
so far in one persistent launch each, several lanes at once.  This module
replays a request stream against it (``replay_native``), runs the plain form
for comparison (``run_sequential``: one request at a time, build then count,
in arrival order, through a backend object), and summarizes latencies
(arrival to result, nearest-rank p50/p99) and throughput.
"""

from __future__ import annotations

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
    """Device work of the one-at-a-time form through the HIP library."""

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


def _limit_of(limit, i: int) -> int:
    """Result limit of request i: ``limit`` is one int for all, or one per request."""
    return int(limit) if isinstance(limit, (int, np.integer)) else int(limit[i])


def run_sequential(backend, arrivals, queries, *, limit=0, clock=time.perf_counter, progress=None):
    """Plain form: one request at a time in arrival order, build then count on one stream.

    ``arrivals`` are offsets in seconds from the start; ``limit`` > 0 asks for
    min(total, limit) (one int, or one per request); ``progress`` (optional)
    is called with a line every 100 requests; returns the requests."""
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
            lim = _limit_of(limit, rid)
            r.count = int(backend.count_batch([h], stream, [lim] if lim else None)[0])
        except Exception as e:
            r.error = f"enumeration failed: {e}"
        finally:
            backend.release(h)
        r.t_done = clock()
        r.batch_size = 1
        r._event.set()
        out.append(r)
        if progress and (rid + 1) % 100 == 0:
            progress(f"plain form: {rid + 1} of {len(queries)} requests done")
    return out


def replay_native(server, arrivals, queries, *, limit=0, clock=time.perf_counter):
    """Submit ``queries[i]`` to a ``cstm.Server`` at ``arrivals[i]`` seconds after
    the start (each with the result limit ``limit``, one int or one per
    request, 0 = all), wait for every result, and return them as ``Request``
    records timed on the server's own clock (submission to result)."""
    start = clock()
    tickets = []
    for i, (t, q) in enumerate(zip(arrivals, queries)):
        now = clock() - start
        if now < t:
            time.sleep(t - now)
        tickets.append((server.submit(q.qlabel, q.qedges, _limit_of(limit, i)), q))
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
