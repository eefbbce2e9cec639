"""Pins for the CPU oracle: brute force, closed forms, matrix identities, invariants.

The oracle is the reference the HIP path is checked against, so it is itself
pinned here to things other than itself.  The last test plants mistakes in the
oracle (its ``mutate`` switch) and shows that these pins catch each one.
"""

from __future__ import annotations

import math

import numpy as np
import pytest

import oracle
import bruteforce
import closed_forms as cf
from synth import Graph, Query, make_graph, query_set


# ---------------------------------------------------------------- helpers

def random_tiny_graph(rng, n=None, L=None, p=None) -> Graph:
    n = int(rng.integers(4, 10)) if n is None else n
    L = int(rng.integers(1, 4)) if L is None else L
    p = float(rng.uniform(0.25, 0.8)) if p is None else p
    edges = [(i, j) for i in range(n) for j in range(i + 1, n) if rng.random() < p]
    labels = rng.integers(0, L, size=n)
    return cf.graph_from_edges(n, edges, labels, "tiny")


def random_connected_query(rng, k=None, L=3, extra=None) -> Query:
    k = int(rng.integers(1, 6)) if k is None else k
    edges = set()
    for v in range(1, k):
        u = int(rng.integers(0, v))
        edges.add((u, v))
    extra = int(rng.integers(0, 4)) if extra is None else extra
    for _ in range(extra):
        a, b = sorted(int(x) for x in rng.choice(k, 2, replace=False)) if k >= 2 else (0, 0)
        if a != b:
            edges.add((a, b))
    perm = rng.permutation(k)
    labels = rng.integers(0, L, size=k)
    e = sorted((int(min(perm[a], perm[b])), int(max(perm[a], perm[b]))) for a, b in edges)
    return cf.query(labels, e)


def rows_of(res) -> list[tuple]:
    return [tuple(int(x) for x in r) for r in res.rows]


# ---------------------------------------------------------------- brute force

@pytest.mark.parametrize("seed", range(60))
def test_matches_bruteforce_on_tiny_graphs(seed):
    rng = np.random.default_rng(1000 + seed)
    g = random_tiny_graph(rng)
    q = random_connected_query(rng, L=int(g.label.max()) + 1)
    want = bruteforce.embeddings(g, q)
    lcol = oracle.label_grouped_col(g)
    for degf in (True, False):
        for threads in (1, 3):
            for lc in (None, lcol):
                r = oracle.match(g, q, list_rows=True, cap=20000, degree_filter=degf, threads=threads, lcol=lc)
                assert r.status == oracle.OK
                assert r.count == len(want)
                assert rows_of(r) == want


def test_listing_cap_reports_overflow_with_exact_count():
    g = cf.complete(6)
    q = cf.path_query(3)
    r = oracle.match(g, q, list_rows=True, cap=10)
    assert r.status == oracle.EOVERFLOW
    assert r.count == math.perm(6, 3)
    assert len(r.rows) == 10
    assert rows_of(r) == bruteforce.embeddings(g, q)[:10]


# ---------------------------------------------------------------- closed forms

@pytest.mark.parametrize("n,k", [(5, 1), (6, 2), (7, 3), (7, 4), (8, 5), (9, 6)])
def test_connected_queries_in_complete_graph(n, k):
    rng = np.random.default_rng(n * 100 + k)
    g = cf.complete(n)
    for _ in range(3):
        q = random_connected_query(rng, k=k, L=1)
        assert oracle.count(g, q) == cf.clique_host_count(n, k)
    assert oracle.count(g, cf.clique_query([0] * k)) == cf.clique_host_count(n, k)


def test_labelled_clique_in_complete_graph():
    labels = [0, 0, 0, 1, 1, 1, 1, 2, 2]
    g = cf.complete(9, labels)
    host = {0: 3, 1: 4, 2: 2}
    for ql in ([0, 1], [0, 0, 1], [1, 1, 1, 2], [0, 1, 2, 2], [2, 2, 2], [0, 0, 0, 1, 1]):
        want = cf.labelled_clique_host_count(host, {l: ql.count(l) for l in set(ql)})
        assert oracle.count(g, cf.clique_query(ql)) == want


@pytest.mark.parametrize("a,b", [(2, 3), (3, 4), (4, 4), (5, 3)])
def test_odd_cycles_absent_and_c4_in_complete_bipartite(a, b):
    g = cf.complete_bipartite(a, b)
    assert oracle.count(g, cf.cycle_query(3)) == 0
    if a + b >= 5:
        assert oracle.count(g, cf.cycle_query(5)) == 0
    assert oracle.count(g, cf.cycle_query(4)) == cf.c4_in_complete_bipartite(a, b)


def test_edges_wedges_stars_on_random_graphs():
    for seed in range(5):
        g = make_graph({"kind": "er", "n": 400, "p": 0.03, "seed": 900 + seed, "labels": {"kind": "uniform", "L": 1}})
        assert oracle.count(g, cf.path_query(2)) == cf.edge_count(g)
        assert oracle.count(g, cf.path_query(3)) == cf.wedge_count(g)
        for s in (3, 4):
            assert oracle.count(g, cf.star_query(s)) == cf.star_count(g, s)


@pytest.mark.parametrize("n", [3, 5, 8, 13])
def test_paths_in_cycles_and_paths(n):
    for k in range(2, n + 1):
        assert oracle.count(cf.cycle(n), cf.path_query(k)) == cf.path_in_cycle(n, k)
        assert oracle.count(cf.path(n), cf.path_query(k)) == cf.path_in_path(n, k)


def test_single_vertex_and_absent_label():
    g = make_graph({"kind": "er", "n": 500, "p": 0.02, "seed": 5, "labels": {"kind": "uniform", "L": 7}})
    for lab in range(7):
        assert oracle.count(g, cf.query([lab], [])) == int((g.label == lab).sum())
    assert oracle.count(g, cf.query([99], [])) == 0
    assert oracle.count(g, cf.query([0, 99, 1], [(0, 1), (1, 2)])) == 0


# ---------------------------------------------------------------- matrix identities at scale

def _c1_graph():
    return make_graph({"kind": "er", "n": 3000, "p": 10 / 2999, "seed": 11, "labels": {"kind": "uniform", "L": 20}})


def test_triangles_trace_identity():
    g = make_graph({"kind": "chung_lu", "n": 20000, "m": 200000, "gamma": 2.3, "seed": 77,
                    "labels": {"kind": "zipf", "L": 4, "s": 1.0}})
    for lab in range(3):
        assert oracle.count(g, cf.cycle_query(3, lab)) == cf.triangle_count_single_label(g, lab)
    for la, lb, lc in [(0, 1, 2), (0, 0, 1), (1, 2, 3), (2, 2, 0)]:
        q = cf.query([la, lb, lc], [(0, 1), (1, 2), (0, 2)])
        assert oracle.count(g, q) == cf.triangle_count_labels(g, la, lb, lc)


def test_distinct_label_trees_equal_tree_dp():
    g = make_graph({"kind": "chung_lu", "n": 30000, "m": 300000, "gamma": 2.3, "seed": 78,
                    "labels": {"kind": "zipf", "L": 16, "s": 1.0}})
    rng = np.random.default_rng(3)
    checked = 0
    for _ in range(12):
        k = int(rng.integers(2, 7))
        labs = rng.choice(16, size=k, replace=False)
        q = random_connected_query(rng, k=k, L=16, extra=0)
        q.qlabel = labs.astype(np.int32)
        want = cf.tree_homomorphism_count(g, q)
        r = oracle.match(g, q, node_budget=3 * 10**8)
        if r.status != oracle.OK:
            continue
        assert r.count == want
        checked += 1
    assert checked >= 8


def test_tree_dp_upper_bounds_every_query():
    g = _c1_graph()
    qs = query_set(g, [4, 5, 6] * 4, 99)
    for q in qs:
        assert oracle.count(g, q) <= cf.tree_homomorphism_count(g, q)


def test_networkx_monomorphisms_on_small_config():
    nx = pytest.importorskip("networkx")
    from networkx.algorithms import isomorphism as iso

    g = _c1_graph()
    G = nx.Graph()
    G.add_nodes_from((v, {"l": int(g.label[v])}) for v in range(g.n))
    for v in range(g.n):
        for w in g.neighbors(v):
            if v < w:
                G.add_edge(v, int(w))
    for q in query_set(g, [4] * 8, 21)[:4]:
        Q = nx.Graph()
        Q.add_nodes_from((u, {"l": int(q.qlabel[u])}) for u in range(q.k))
        Q.add_edges_from((int(a), int(b)) for a, b in q.qedges)
        gm = iso.GraphMatcher(G, Q, node_match=lambda x, y: x["l"] == y["l"])
        want = sum(1 for _ in gm.subgraph_monomorphisms_iter())
        assert oracle.count(g, q) == want


# ---------------------------------------------------------------- invariants

def test_self_match_counts_automorphisms():
    rng = np.random.default_rng(17)
    for _ in range(20):
        q = random_connected_query(rng, k=int(rng.integers(2, 7)), L=2, extra=3)
        aut = cf.automorphism_count(q)
        assert oracle.count(cf.query_as_graph(q), q) == aut


def test_automorphisms_divide_count_and_source_row_listed():
    g = _c1_graph()
    for q in query_set(g, [3, 4, 5, 6] * 3, 23):
        r = oracle.match(g, q, list_rows=True, cap=1 << 20)
        assert r.status == oracle.OK
        assert r.count >= 1
        assert r.count % cf.automorphism_count(q) == 0
        assert tuple(int(x) for x in q.source) in set(rows_of(r))


def test_vertex_permutation_and_query_relabel_invariance():
    rng = np.random.default_rng(5)
    g = random_tiny_graph(rng, n=40, L=3, p=0.15)
    for _ in range(10):
        q = random_connected_query(rng, k=4, L=3, extra=2)
        c = oracle.count(g, q)
        perm = rng.permutation(g.n)
        assert oracle.count(cf.permute_graph(g, perm), q) == c
        assert oracle.count(g, cf.relabel_query(q, rng.permutation(q.k))) == c


def test_disjoint_union_adds_and_extra_edges_never_lower():
    rng = np.random.default_rng(8)
    g1 = random_tiny_graph(rng, n=30, L=2, p=0.2)
    g2 = random_tiny_graph(rng, n=25, L=2, p=0.25)
    u = cf.disjoint_union(g1, g2)
    for _ in range(8):
        q = random_connected_query(rng, k=4, L=2, extra=1)
        assert oracle.count(u, q) == oracle.count(g1, q) + oracle.count(g2, q)
        more = [(v, int(w)) for v in range(g1.n) for w in g1.neighbors(v) if v < w]
        more += [tuple(sorted(int(x) for x in rng.choice(g1.n, 2, replace=False))) for _ in range(30)]
        g1b = cf.graph_from_edges(g1.n, more, g1.label)
        assert oracle.count(g1b, q) >= oracle.count(g1, q)


def test_degree_filter_and_thread_count_do_not_change_results():
    g = _c1_graph()
    for q in query_set(g, [4, 5] * 3, 31):
        a = oracle.match(g, q, degree_filter=True, threads=1, list_rows=True)
        b = oracle.match(g, q, degree_filter=False, threads=0, list_rows=True)
        assert a.count == b.count
        assert rows_of(a) == rows_of(b)


def test_label_grouped_rows_are_regrouped_rows_and_change_no_result():
    g = _c1_graph()
    lcol = oracle.label_grouped_col(g)
    for v in range(0, g.n, 97):
        a, b = g.row_ptr[v], g.row_ptr[v + 1]
        row = lcol[a:b]
        assert sorted(row.tolist()) == g.col[a:b].tolist()
        keys = [(int(g.label[x]), int(x)) for x in row]
        assert keys == sorted(keys)
    for q in query_set(g, [4, 5, 6] * 2, 37):
        a = oracle.match(g, q, list_rows=True)
        b = oracle.match(g, q, list_rows=True, lcol=lcol, threads=2)
        assert a.status == b.status == oracle.OK
        assert a.count == b.count and rows_of(a) == rows_of(b)
        assert b.nodes <= a.nodes


@pytest.mark.parametrize("seed", range(20))
def test_count_limit_is_min_of_total_and_limit(seed):
    rng = np.random.default_rng(7000 + seed)
    g = random_tiny_graph(rng)
    q = random_connected_query(rng, L=int(g.label.max()) + 1)
    total = len(bruteforce.embeddings(g, q))
    for lim in sorted({1, max(1, total // 2), total, total + 1, 10 * total + 3}):
        for threads in (1, 3):
            r = oracle.match(g, q, limit=lim, threads=threads)
            assert r.status == oracle.OK
            assert r.count == min(total, lim)


def test_count_limit_stops_early_on_a_large_count():
    g = cf.complete(60)
    q = cf.clique_query([0] * 4)
    full = oracle.match(g, q)
    assert full.count == cf.clique_host_count(60, 4)
    r = oracle.match(g, q, limit=1000, threads=4)
    assert r.status == oracle.OK and r.count == 1000
    assert r.nodes < full.nodes // 10
    with pytest.raises(ValueError):
        oracle.match(g, q, limit=10, list_rows=True)


def test_node_budget_is_deterministic_and_reports_timeout():
    g = _c1_graph()
    q = query_set(g, [6], 41)[0]
    full = oracle.match(g, q)
    assert full.status == oracle.OK
    again = oracle.match(g, q, node_budget=full.nodes, threads=4)
    assert again.status == oracle.OK and again.nodes == full.nodes
    cut = oracle.match(g, q, node_budget=max(1, full.nodes // 3), threads=4)
    assert cut.status == oracle.ETIMEOUT
    assert cut.count <= full.count


def test_invalid_queries_rejected():
    g = _c1_graph()
    with pytest.raises(ValueError):
        oracle.match(g, cf.query([0, 1, 2], [(0, 1)]))  # disconnected
    with pytest.raises(ValueError):
        oracle.match(g, cf.query([0, 1], [(0, 1), (0, 1)]))  # duplicate edge
    with pytest.raises(ValueError):
        oracle.match(g, cf.query([0, 1], [(0, 0)]))  # self-loop
    with pytest.raises(ValueError):
        oracle.match(g, cf.query([-1], []))


# ---------------------------------------------------------------- planted mistakes

def _pins_pass(mutate: int) -> bool:
    """Run a compact battery of pins against a mutated oracle; False if any pin fails."""
    rng = np.random.default_rng(4242)
    for _ in range(25):
        g = random_tiny_graph(rng)
        q = random_connected_query(rng, L=int(g.label.max()) + 1)
        want = bruteforce.embeddings(g, q)
        r = oracle.match(g, q, list_rows=True, cap=20000, mutate=mutate)
        if r.count != len(want) or rows_of(r) != want:
            return False
    if oracle.match(cf.complete(7), cf.path_query(4), mutate=mutate).count != cf.clique_host_count(7, 4):
        return False
    if oracle.match(cf.complete_bipartite(3, 4), cf.cycle_query(3), mutate=mutate).count != 0:
        return False
    return True


@pytest.mark.parametrize("mutate", [1, 2, 3, 4, 5, 6])
def test_planted_mistakes_are_caught(mutate):
    assert _pins_pass(0)
    assert not _pins_pass(mutate)


def test_maximum_query_size():
    assert oracle.count(cf.cycle(40), cf.path_query(32)) == cf.path_in_cycle(40, 32)
    assert oracle.count(cf.path(40), cf.path_query(32)) == cf.path_in_path(40, 32)
    with pytest.raises(ValueError):
        oracle.match(cf.cycle(40), cf.path_query(33))
