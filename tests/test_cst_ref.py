"""Pins for the CST-level reference (Algorithms 1, 2, 5-8 and the workload estimate).

Checked against the paper's worked examples (on a fixture graph consistent with
them), Definition 2 itself, the soundness theorem (all embeddings lie in the
CST) through brute force and the count oracle, and the partition's promises
(disjoint, complete, within budget).
"""

from __future__ import annotations

import json
import os

import numpy as np
import pytest

import oracle
from oracle import cst_ref
import bruteforce
import closed_forms as cf
from synth import make_graph, query_set
from test_oracle import random_connected_query, random_tiny_graph

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def fig4():
    d = json.load(open(os.path.join(GOLDEN, "fig4_fixture.json")))
    g = cf.graph_from_edges(d["n"], [tuple(e) for e in d["edges"]], d["labels"], "fig4")
    q = cf.query(d["query"]["qlabel"], [tuple(e) for e in d["query"]["qedges"]])
    return g, q, d["facts"]


def test_fig4_tree_shape_and_root():
    g, q, _ = fig4()
    cst = cst_ref.build_cst(g, q.qlabel, q.qedges)
    assert cst.root == 0
    assert cst.parent == [-1, 0, 0, 1]
    assert cst.nontree == [(1, 2), (2, 3)]
    assert sorted(cst.cand[0]) == [1, 2]
    assert sorted(cst.cand[2]) == [6, 7, 8]


def test_fig4_workload_example():
    g, q, facts = fig4()
    cst = cst_ref.build_cst(g, q.qlabel, q.qedges)
    c, W = cst_ref.workload(cst)
    f = facts["example_workload"]
    assert W == f["W"]
    assert {str(v): x for v, x in c[0].items()} == f["c_u0"]
    for u, vs in f["leaf_values_one"].items():
        for v in vs:
            assert c[int(u[1:])][v] == 1


def test_fig4_partition_example():
    g, q, facts = fig4()
    cst = cst_ref.build_cst(g, q.qlabel, q.qedges)
    order = [0, 1, 2, 3]
    parts = cst_ref.partition(cst, order, delta_s=1, force_k=2)
    f = facts["example_partition"]
    roots = [sorted(s[0]) for _, s in parts[: len(f["root_parts"])]]
    # with k = 2 the root split is {v1} | {v2}; further splits only refine below it
    root_sets = []
    for _, s in parts:
        if sorted(s[0]) not in root_sets:
            root_sets.append(sorted(s[0]))
    assert root_sets == f["root_parts"]
    part1 = cst_ref.restricted_sets(cst, order, {0: (0, 1)})
    for u, vs in f["part1"].items():
        assert sorted(part1[int(u[1:])]) == vs
    part2 = cst_ref.restricted_sets(cst, order, {0: (1, 2)})
    all_rows = cst_ref.enumerate_cst(cst, order)
    r1 = cst_ref.enumerate_cst(cst, order, part1)
    r2 = cst_ref.enumerate_cst(cst, order, part2)
    assert not set(r1) & set(r2)
    assert sorted(r1 + r2) == all_rows
    del roots


def test_fig4_round_example():
    g, q, facts = fig4()
    cst = cst_ref.build_cst(g, q.qlabel, q.qedges)
    f = facts["example_round"]
    part1 = cst_ref.restricted_sets(cst, f["order"], {0: (0, 1)})
    P = [tuple(p) for p in f["P"]]
    P_o, T_v, T_n, B_v, B_n, surv, rest = cst_ref.fast_round(cst, f["order"], P, N_o=64, cand_override=part1)
    assert [list(p) for p in P_o] == f["P_o"]
    assert [list(t) for t in T_v] == f["T_v"]
    assert [list(t) for t in T_n] == f["T_n"]
    assert B_v == f["B_v"] and B_n == f["B_n"]
    assert [list(p) for p in surv] == f["survivors"]
    assert rest == []
    # a round that cannot take the next p_i whole leaves it in P
    P_o, *_ , rest = cst_ref.fast_round(cst, f["order"], P, N_o=3, cand_override=part1)
    assert len(P_o) == 2 and rest == [P[1]]


def test_fig4_counts_agree_with_oracle():
    g, q, _ = fig4()
    cst = cst_ref.build_cst(g, q.qlabel, q.qedges)
    rows = cst_ref.enumerate_cst(cst, cst_ref.path_order(cst))
    r = oracle.match(g, q, list_rows=True)
    assert [tuple(int(x) for x in row) for row in r.rows] == rows
    assert len(rows) == 3


def _check_definition2(g, cst):
    """Every list is exactly N_G(v) intersected with the neighbour's candidate set."""
    for (up, u), lists in cst.tree_adj.items():
        cs = set(cst.cand[u])
        for vp in cst.cand[up]:
            want = sorted(int(w) for w in g.neighbors(vp) if int(w) in cs)
            assert sorted(lists.get(vp, [])) == want
    for (u, un), lists in cst.nt_adj.items():
        cs = set(cst.cand[un])
        for v in cst.cand[u]:
            assert sorted(lists[v]) == sorted(int(w) for w in g.neighbors(v) if int(w) in cs)


@pytest.mark.parametrize("seed", range(40))
def test_cst_is_sound_and_complete_on_tiny_graphs(seed):
    rng = np.random.default_rng(5000 + seed)
    g = random_tiny_graph(rng)
    q = random_connected_query(rng, L=int(g.label.max()) + 1)
    cst = cst_ref.build_cst(g, q.qlabel, q.qedges)
    _check_definition2(g, cst)
    want = bruteforce.embeddings(g, q)
    # soundness constraint: every embedding's vertices are candidates
    for row in want:
        for u, v in enumerate(row):
            assert v in cst.cand[u]
    order = cst_ref.path_order(cst)
    assert cst_ref.enumerate_cst(cst, order) == want
    # any connected order with parents first gives the same set
    assert cst_ref.enumerate_cst(cst, cst.bfs) == want


def test_cst_on_small_config_matches_oracle_listing():
    g = make_graph({"kind": "er", "n": 3000, "p": 10 / 2999, "seed": 11, "labels": {"kind": "uniform", "L": 20}})
    for q in query_set(g, [4] * 8, 21) + query_set(g, [5, 6], 77):
        cst = cst_ref.build_cst(g, q.qlabel, q.qedges)
        _check_definition2(g, cst)
        r = oracle.match(g, q, list_rows=True)
        rows = [tuple(int(x) for x in row) for row in r.rows]
        assert cst_ref.enumerate_cst(cst, cst_ref.path_order(cst)) == rows
        _, W = cst_ref.workload(cst)
        assert W >= r.count


def test_workload_is_exact_for_distinct_label_trees():
    g = make_graph({"kind": "er", "n": 2000, "p": 0.004, "seed": 3, "labels": {"kind": "uniform", "L": 6}})
    rng = np.random.default_rng(12)
    for _ in range(10):
        k = int(rng.integers(2, 6))
        q = random_connected_query(rng, k=k, L=6, extra=0)
        q.qlabel = rng.choice(6, size=k, replace=False).astype(np.int32)
        cst = cst_ref.build_cst(g, q.qlabel, q.qedges)
        _, W = cst_ref.workload(cst)
        assert W == oracle.count(g, q) == cf.tree_homomorphism_count(g, q)


@pytest.mark.parametrize("seed", range(12))
def test_partitions_are_disjoint_complete_and_within_budget(seed):
    rng = np.random.default_rng(7000 + seed)
    g = make_graph({"kind": "er", "n": 60, "p": 0.2, "seed": 100 + seed, "labels": {"kind": "uniform", "L": 2}})
    q = random_connected_query(rng, k=int(rng.integers(2, 6)), L=2, extra=int(rng.integers(0, 3)))
    cst = cst_ref.build_cst(g, q.qlabel, q.qedges)
    order = cst_ref.path_order(cst)
    full = cst_ref.enumerate_cst(cst, order)
    budget = cst_ref.image_header_bytes(q.k, len(cst.nontree)) + 200
    parts = cst_ref.partition(cst, order, delta_s=budget)
    seen = []
    for ranges, sets in parts:
        assert cst_ref.image_bytes(cst, order, sets) <= budget or all(len(s) == 1 for s in sets)
        seen += cst_ref.enumerate_cst(cst, order, sets)
    assert len(seen) == len(set(seen))
    assert sorted(seen) == full


def test_share_split_on_the_worked_example():
    """Algorithm 3 on the workload example: c(v1) = 4, c(v2) = 3, one run per
    root candidate.  By the rule: v1 goes to the accelerator (4 < 4*delta never
    holds for delta <= 1), then v2 goes to the host iff 3 < 7*delta."""
    g, q, _ = fig4()
    cst = cst_ref.build_cst(g, q.qlabel, q.qedges)
    c, W = cst_ref.workload(cst)
    weights = [c[cst.root][v] for v in cst.cand[cst.root]]
    assert sorted(weights) == [3, 4] and W == 7
    second = weights[1]  # the first run always goes to the accelerator
    for delta in (0.0, 0.4, 3 / 7, 0.43, 0.5, 4 / 7, 0.58, 1.0):
        host, dev, wc, wf = cst_ref.share_split(weights, delta, 2)
        assert dev[0] == (0, 1)
        # by hand: 0 + second < delta * (0 + first + second) = 7 * delta
        assert (host == [(1, 2)]) == (second < 7 * delta)
        assert wc + wf == 7.0
    if second == 3:
        assert cst_ref.share_split(weights, 0.43, 2)[0] == [(1, 2)]
        assert cst_ref.share_split(weights, 3 / 7, 2)[0] == []
    # one run holding both: never the host's (W < delta*W fails for delta <= 1)
    assert cst_ref.share_split(weights, 1.0, 1) == ([], [(0, 2)], 0.0, 7.0)


@pytest.mark.parametrize("seed", range(5))
def test_share_split_keeps_the_host_share_below_delta(seed):
    rng = np.random.default_rng(900 + seed)
    w = rng.integers(0, 1000, size=int(rng.integers(1, 300))).tolist()
    for delta in (0.0, 0.01, 0.1, 0.5, 0.9, 1.0):
        for runs in (0, 1, 3, 17, 1000):
            host, dev, wc, wf = cst_ref.share_split(w, delta, runs)
            # runs tile the root candidates in order, each exactly once
            tiles = sorted(host + dev)
            assert tiles[0][0] == 0 and tiles[-1][1] == len(w)
            assert all(a[1] == b[0] and a[0] < a[1] for a, b in zip(tiles, tiles[1:]))
            assert len(tiles) == min(len(w), runs if runs > 0 else 1024)
            assert wc + wf == float(sum(w))
            assert wc == sum(sum(w[lo:hi]) for lo, hi in host)
            if delta == 0.0:
                assert host == []
            if host:
                assert wc < delta * (wc + wf)
