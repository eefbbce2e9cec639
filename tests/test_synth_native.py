"""The native R-MAT and Chung-Lu generators build simple, symmetric, sorted CSRs, independent of the thread count."""

from __future__ import annotations

import numpy as np

from synth import make_graph, native


def test_native_rmat_is_a_simple_sorted_symmetric_csr():
    rp, col = native.rmat_csr(14, 16, 0.57, 0.19, 0.19, 15, threads=4)
    n = 1 << 14
    assert rp.shape == (n + 1,) and rp[0] == 0 and rp[-1] == col.shape[0]
    deg = np.diff(rp)
    src = np.repeat(np.arange(n, dtype=np.int64), deg)
    assert np.all((col >= 0) & (col < n))
    assert not np.any(src == col)
    key = src * n + col
    assert np.all(np.diff(key) > 0)  # rows ascending, no duplicates
    assert np.array_equal(np.sort(col.astype(np.int64) * n + src), key)  # both directions
    assert col.shape[0] // 2 <= 16 * n
    assert deg.max() > 20 * deg.mean()  # R-MAT skew


def test_native_rmat_does_not_depend_on_threads_and_follows_the_seed():
    a = native.rmat_csr(12, 8, 0.57, 0.19, 0.19, 7, threads=1)
    b = native.rmat_csr(12, 8, 0.57, 0.19, 0.19, 7, threads=5)
    c = native.rmat_csr(12, 8, 0.57, 0.19, 0.19, 8, threads=5)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])
    assert not np.array_equal(a[1], c[1])


def test_make_graph_native_kind():
    g = make_graph({"kind": "rmat_native", "scale": 10, "edge_factor": 8, "seed": 3,
                    "labels": {"kind": "uniform", "L": 16}})
    assert g.n == 1024 and g.label.shape == (1024,) and g.label.max() < 16


def _check_simple_sorted_symmetric(n, rp, col):
    assert rp.shape == (n + 1,) and rp[0] == 0 and rp[-1] == col.shape[0]
    src = np.repeat(np.arange(n, dtype=np.int64), np.diff(rp))
    assert np.all((col >= 0) & (col < n)) and not np.any(src == col)
    key = src * n + col
    assert np.all(np.diff(key) > 0)
    assert np.array_equal(np.sort(col.astype(np.int64) * n + src), key)


def test_native_chung_lu_keeps_exactly_m_edges_and_the_weight_skew():
    n, m = 50_000, 400_000
    rp, col = native.chung_lu_csr(n, m, 2.2, 3, threads=3)
    _check_simple_sorted_symmetric(n, rp, col)
    assert col.shape[0] == 2 * m
    # the same recipe drawn by numpy (PCG64, inverse transform) has the same kind of hubs
    g = make_graph({"kind": "chung_lu", "n": n, "m": m, "gamma": 2.2, "seed": 3,
                    "labels": {"kind": "uniform", "L": 2}})
    d_native, d_numpy = np.sort(np.diff(rp))[::-1], np.sort(g.degree)[::-1]
    for top in (1, 10, 100, 1000):
        assert 0.8 < d_native[top - 1] / d_numpy[top - 1] < 1.25
    a = native.chung_lu_csr(n, m, 2.2, 3, threads=1)
    assert np.array_equal(a[0], rp) and np.array_equal(a[1], col)
    b = native.chung_lu_csr(n, m, 2.2, 4, threads=3)
    assert not np.array_equal(b[1], col)
