"""Host-side checks of the serving helpers with a stand-in backend (no GPU):
the one-at-a-time form, nearest-rank percentiles and the seeded Poisson
arrivals.  The server itself is native and is tested on the GPU.

The stand-in "builds" a request by returning its query and "counts" a batch
by sleeping for the longest query's duration and returning each query's known
count.
"""

from __future__ import annotations

import threading
import time

import numpy as np

from paper_2102_10768_amd import serve


class FakeQuery:
    def __init__(self, i, count, seconds, nbytes):
        self.i = i
        self.count = count
        self.seconds = seconds
        self.nbytes = nbytes


class FakeBackend:
    def __init__(self):
        self.lock = threading.Lock()
        self.live = 0
        self.live_peak = 0
        self.launch_sizes = []

    def new_stream(self):
        return object()

    def estimate(self, q):
        if q.nbytes < 0:
            raise ValueError("malformed")
        return q.nbytes

    def build(self, q, stream):
        with self.lock:
            self.live += q.nbytes
            self.live_peak = max(self.live_peak, self.live)
        time.sleep(0.0005)
        return q

    def count_batch(self, handles, stream, limits=None):
        self.launch_sizes.append(len(handles))
        time.sleep(max(h.seconds for h in handles))
        if any(h.count < 0 for h in handles):
            raise RuntimeError("device error")
        if limits is not None:
            return [min(h.count, lim) if lim else h.count for h, lim in zip(handles, limits)]
        return [h.count for h in handles]

    def release(self, h):
        with self.lock:
            self.live -= h.nbytes


def _queries(n, seed):
    rng = np.random.default_rng(seed)
    out = []
    for i in range(n):
        sec = float(rng.uniform(0.0005, 0.003))
        out.append(FakeQuery(i, int(rng.integers(0, 10**9)), sec, int(rng.integers(1, 100))))
    return out


def test_sequential_form_and_percentiles():
    be = FakeBackend()
    qs = _queries(30, 6)
    arr = serve.poisson_arrivals(len(qs), 500.0, 9)
    reqs = serve.run_sequential(be, arr, qs)
    assert [r.count for r in reqs] == [q.count for q in qs]
    dones = [r.t_done for r in reqs]
    assert dones == sorted(dones)
    s = serve.summarize(reqs)
    assert s["completed"] == 30 and s["p50_ms"] <= s["p99_ms"]
    assert serve.nearest_rank([5, 1, 4, 2, 3], 50) == 3
    assert serve.nearest_rank(list(range(1, 101)), 99) == 99
    assert serve.nearest_rank([7], 99) == 7


def test_poisson_arrivals_rate_and_seed():
    a = serve.poisson_arrivals(20000, 200.0, 201)
    b = serve.poisson_arrivals(20000, 200.0, 201)
    assert np.array_equal(a, b)
    assert np.all(np.diff(a) > 0)
    assert abs(len(a) / a[-1] - 200.0) < 6.0


def test_sequential_form_takes_one_limit_or_one_per_request():
    be = FakeBackend()
    qs = _queries(12, 7)
    arr = serve.poisson_arrivals(len(qs), 2000.0, 10)
    lim = [0, 5, 10**10] * 4
    reqs = serve.run_sequential(be, arr, qs, limit=lim)
    assert [r.count for r in reqs] == [q.count if not m else min(q.count, m) for q, m in zip(qs, lim)]
    reqs = serve.run_sequential(be, arr, qs, limit=3)
    assert [r.count for r in reqs] == [min(q.count, 3) for q in qs]
