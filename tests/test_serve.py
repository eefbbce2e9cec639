"""Host-side checks of the request loop's logic with a stand-in backend (no GPU).

The stand-in "builds" a request by returning its query and "counts" a batch
by sleeping for the longest query's duration and returning each query's known
count; it records how much memory is charged at every moment, so admission,
overlap, ordering and completion can be checked without a device.
"""

from __future__ import annotations

import threading
import time

import numpy as np
import pytest

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


def test_every_request_gets_its_own_count_under_load():
    be = FakeBackend()
    qs = _queries(300, 1)
    arr = serve.poisson_arrivals(len(qs), 2000.0, 7)
    with serve.Server(be, mem_budget=10_000, lanes=2, max_batch=64) as srv:
        reqs = serve.replay(srv, arr, qs)
    assert [r.count for r in reqs] == [q.count for q in qs]
    assert all(r.error is None and r.latency >= 0 for r in reqs)
    assert max(be.launch_sizes) > 1  # requests that queue up share launches
    assert be.live == 0


def test_admission_keeps_charged_bytes_within_budget_in_arrival_order():
    be = FakeBackend()
    qs = _queries(200, 2)
    budget = 400
    with serve.Server(be, mem_budget=budget, lanes=2, max_batch=16) as srv:
        reqs = [srv.submit(q) for q in qs]
        for r in reqs:
            assert r.wait(30)
    assert srv.peak_bytes <= budget
    assert be.live_peak <= budget
    admits = [r.t_admit for r in reqs]
    assert admits == sorted(admits)
    assert [r.count for r in reqs] == [q.count for q in qs]


def test_oversized_and_malformed_requests_are_refused_and_others_proceed():
    be = FakeBackend()
    qs = _queries(20, 3)
    qs[5] = FakeQuery(5, 1, 0.001, 10_000)
    qs[9] = FakeQuery(9, 1, 0.001, -1)
    with serve.Server(be, mem_budget=1000, lanes=1) as srv:
        reqs = [srv.submit(q) for q in qs]
    assert "exceeds" in reqs[5].error and reqs[5].count is None
    assert "rejected" in reqs[9].error
    for i, r in enumerate(reqs):
        if i not in (5, 9):
            assert r.error is None and r.count == qs[i].count


def test_a_long_launch_does_not_block_a_second_lane():
    be = FakeBackend()
    qs = _queries(40, 4)
    qs[0] = FakeQuery(0, 7, 0.3, 10)
    arr = np.linspace(0.0, 0.1, len(qs))
    with serve.Server(be, mem_budget=10_000, lanes=2, max_batch=8) as srv:
        reqs = serve.replay(srv, arr, qs)
    assert srv.max_overlap == 2
    small = [r for r, q in zip(reqs, qs) if q.seconds < 0.1 and r.t_arrival > reqs[0].t_arrival + 0.01]
    # the short requests finish while the first, long launch (0.3 s) is still running
    assert all(r.t_done < reqs[0].t_done for r in small)
    assert [r.count for r in reqs] == [q.count for q in qs]


def test_enumeration_failure_is_reported_per_request():
    be = FakeBackend()
    qs = _queries(10, 5)
    qs[3] = FakeQuery(3, -1, 0.001, 10)
    with serve.Server(be, mem_budget=10_000, lanes=1, max_batch=1) as srv:
        reqs = [srv.submit(q) for q in qs]
    assert reqs[3].error and "failed" in reqs[3].error
    assert all(r.error is None for i, r in enumerate(reqs) if i != 3)
    assert be.live == 0


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


def test_closed_server_refuses_new_requests():
    srv = serve.Server(FakeBackend(), lanes=1)
    srv.close()
    with pytest.raises(RuntimeError):
        srv.submit(FakeQuery(0, 1, 0.001, 1))
