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
    """Algorithm 3 on the workload example: c(v1) = 4, c(v2) = 3 (Section V-C),
    one run per root candidate.  The root candidates are ordered by degree
    (both 4) then id, so v1's run comes first; by the rule it goes to the
    accelerator (4 < 4*delta never holds for delta <= 1), then v2 goes to the
    host iff 3 < 7*delta."""
    g, q, _ = fig4()
    cst = cst_ref.build_cst(g, q.qlabel, q.qedges)
    c, W = cst_ref.workload(cst)
    assert cst.cand[cst.root] == [1, 2]
    weights = [c[cst.root][v] for v in cst.cand[cst.root]]
    assert weights == [4, 3] and W == 7
    for delta in (0.0, 0.4, 3 / 7, 0.43, 0.5, 4 / 7, 0.58, 1.0):
        host, dev, wc, wf = cst_ref.share_split(weights, delta, 2)
        assert dev[0] == (0, 1)
        # by hand: 0 + 3 < delta * (0 + 4 + 3) = 7 * delta
        assert (host == [(1, 2)]) == (3 < 7 * delta)
        assert wc + wf == 7
    # the float 3/7 lies just below 3/7, so 7 * delta < 3 and v2 stays
    assert cst_ref.share_split(weights, 0.43, 2) == ([(1, 2)], [(0, 1)], 3, 4)
    assert cst_ref.share_split(weights, 3 / 7, 2) == ([], [(0, 1), (1, 2)], 0, 7)
    # one run holding both: never the host's (W < delta*W fails for delta <= 1)
    assert cst_ref.share_split(weights, 1.0, 1) == ([], [(0, 2)], 0, 7)


def test_share_split_is_exact_beyond_double_precision():
    """Weights above 2^53, where a float sum would round: the split still
    follows the rule with exact integers.  Runs [2^60, 1, 1]: the first goes
    to the accelerator; the second goes to the host iff 1 < delta*(2^60 + 1)."""
    big = 1 << 60
    host, dev, wc, wf = cst_ref.share_split([big, 1, 1], 2.0 ** -60, 3)
    # 1 < 2^-60 * (2^60 + 1) = 1 + 2^-60: host.  Third: 1 + 1 < 2^-60 * (2^60 + 2): no.
    assert host == [(1, 2)] and dev == [(0, 1), (2, 3)] and (wc, wf) == (1, big + 1)
    assert float(big) + 1.0 == float(big)  # the same test in doubles could not see the 1


def test_fig4_candidate_order_and_paths():
    """Hand-derived from the fixture graph (Section V-A construction, Section V-B
    order).  Candidates are ordered by degree descending, then id: C(u1) =
    [v4 (deg 4), v3 (3), v5 (3)], C(u2) = [v6 (5), v8 (4), v7 (3)].  Root-to-leaf
    paths: u0-u1-u3 holds 3 CST paths (v1: v3-v9, v5-v10; v2: v4-v9) and u0-u2
    holds 5 (v1: v6, v8; v2: v6, v7, v8), so the path-based order, fewest paths
    first, is u0, u1, u3, u2."""
    g, q, _ = fig4()
    cst = cst_ref.build_cst(g, q.qlabel, q.qedges)
    assert cst.cand == [[1, 2], [4, 3, 5], [6, 8, 7], [9, 10]]
    assert cst.tree_adj[(0, 1)] == {1: [3, 5], 2: [4]}
    assert cst.tree_adj[(1, 3)] == {4: [9], 3: [9], 5: [10]}
    assert cst_ref.tree_paths(cst) == [[0, 2], [0, 1, 3]]
    assert cst_ref.path_embeddings(cst, [0, 1, 3]) == 3
    assert cst_ref.path_embeddings(cst, [0, 2]) == 5
    assert cst_ref.path_order(cst) == [0, 1, 3, 2]


@pytest.mark.parametrize("n,length", [(7, 1), (7, 3), (12, 4)])
def test_path_embeddings_in_complete_graph(n, length):
    """A path query of length+1 vertices (one label) in K_n: every candidate
    set is all n vertices and every tree list has n - 1 entries, so a
    root-to-leaf path of `length` edges holds n * (n-1)^length CST paths."""
    g = cf.complete(n)
    k = length + 1
    q = cf.query([0] * k, [(i, i + 1) for i in range(length)])
    cst = cst_ref.build_cst(g, q.qlabel, q.qedges)
    for p in cst_ref.tree_paths(cst):
        assert cst_ref.path_embeddings(cst, p) == n * (n - 1) ** (len(p) - 1)
    # the root is an inner vertex (ratio n/2 < n/1), so both paths start there
    if length >= 2:
        assert cst.root == 1


def test_root_order_and_workload_on_complete_bipartite():
    """K_{3,10}: side A = 3 vertices of label 0 (degree 10), side B = 10
    vertices of label 1 (degree 3).  Query u0(1) - u1(0) - u2(1).  Ratios
    #C0(u)/d_q(u): u0 10/1, u1 3/2, u2 10/1, so the root is u1 (the middle
    vertex); both root-to-leaf paths hold 3*10 CST paths, the tie goes to the
    smaller leaf, giving the order u1, u0, u2.  W = 3 * 10 * 10 = 300 and the
    count is 3 * 10 * 9 = 270 (u0 and u2 must differ)."""
    edges = [(a, b) for a in range(3) for b in range(3, 13)]
    g = cf.graph_from_edges(13, edges, [0] * 3 + [1] * 10, "k3_10")
    q = cf.query([1, 0, 1], [(0, 1), (1, 2)])
    cst = cst_ref.build_cst(g, q.qlabel, q.qedges)
    assert cst.root == 1 and cst.parent == [1, -1, 1]
    assert cst_ref.path_order(cst) == [1, 0, 2]
    c, W = cst_ref.workload(cst)
    assert W == 300 and set(c[1].values()) == {100}
    assert oracle.count(g, q) == 270


def test_workload_of_stars_in_complete_graphs_and_saturation():
    """Star K_{1,s} (one label) in K_n: the root is the centre (ratio n/s
    against n/1), c_centre(v) = (n-1)^s and W = n (n-1)^s.  K_{1,6} in K_300
    gives 300 * 299^6 ~ 2.1e17, beyond 2^53 (exact as an integer); K_{1,8} in
    K_400 gives ~2.6e23, beyond 2^64, which the unsigned 64-bit form holds as
    2^64 - 1."""
    for n, s_ in ((300, 6), (40, 8)):
        g = cf.complete(n)
        q = cf.query([0] * (s_ + 1), [(0, i) for i in range(1, s_ + 1)])
        cst = cst_ref.build_cst(g, q.qlabel, q.qedges)
        assert cst.root == 0
        c, W = cst_ref.workload(cst)
        assert W == n * (n - 1) ** s_
        assert set(c[0].values()) == {(n - 1) ** s_}
    assert 300 * 299 ** 6 > 2 ** 53
    assert cst_ref.saturate_u64(400 * 399 ** 8) == 2 ** 64 - 1
    assert cst_ref.saturate_u64(300 * 299 ** 6) == 300 * 299 ** 6


def test_fig4_image_bytes_by_hand():
    """size(CST) of the on-chip image, summed by hand for the fixture
    (header 64 + 32 per position + 16 per non-tree edge = 224 B for k = 4 and
    two non-tree edges; 4 B per candidate; per tree edge 4 B per parent
    candidate + 4 B, and 2 B per entry padded to 4 B; per non-tree edge one
    ceil(#C(b)/32)-word bit row per candidate of its earlier end).

    Order u0, u1, u2, u3: candidates 10 -> 40; tree edges u0u1 12 + 8,
    u0u2 12 + 12, u1u3 16 + 8 -> 68; non-tree u1u2 3 rows, u2u3 3 rows -> 24;
    224 + 40 + 68 + 24 = 356 -> 368.  Path order u0, u1, u3, u2: the u2u3
    rows belong to u3 (2 rows) -> 20; total 352.  Partition {v1} under the
    path order: 7 candidates -> 28; tree 12 + 12 + 16 = 40; rows 8 + 8 = 16;
    308 -> 320.  Partition {v2}: 6 -> 24; tree 12 + 16 + 12 = 40; rows 4 + 4;
    296 -> 304.  D_CST: the full CST's longest list is v2's u2 list (3)."""
    g, q, _ = fig4()
    cst = cst_ref.build_cst(g, q.qlabel, q.qedges)
    assert cst_ref.image_header_bytes(4, 2) == 224
    full = cst_ref.restricted_sets(cst, [0, 1, 2, 3], {})
    assert cst_ref.image_bytes(cst, [0, 1, 2, 3], full) == 368
    po = [0, 1, 3, 2]
    assert cst_ref.image_bytes(cst, po, cst_ref.restricted_sets(cst, po, {})) == 352
    p1 = cst_ref.restricted_sets(cst, po, {0: (0, 1)})
    p2 = cst_ref.restricted_sets(cst, po, {0: (1, 2)})
    assert [sorted(x) for x in p1] == [[1], [3, 5], [6, 8], [9, 10]]
    assert [sorted(x) for x in p2] == [[2], [4], [6, 7, 8], [9]]
    assert cst_ref.image_bytes(cst, po, p1) == 320
    assert cst_ref.image_bytes(cst, po, p2) == 304
    assert cst_ref.max_list_len(cst, full) == 3
    assert cst_ref.max_list_len(cst, p1) == 2


def test_fig4_partition_counts_by_hand():
    """Algorithm 2 under the path order u0, u1, u3, u2 (full image 352 B).
    delta_S = 320: kpart = ceil(352/320) = 2 splits C(u0) into {v1} (320 B) and
    {v2} (304 B), both fit: 2 partitions.  delta_S = 304: {v1} is 320 B, so it
    splits again at the next vertex with more than one candidate, u1 = {v3, v5}
    (kpart = 2): {v1, v3} and {v1, v5} are 288 B each (u3 keeps the one leaf
    each reaches, u2 keeps {v6, v8}); with {v2} at 304 B: 3 partitions.
    delta_D = 2 with no byte limit: the full CST's longest list (3) splits the
    root; {v1} fits; under {v2} the u2 list {v6, v7, v8} is cut at u2 into
    {v6, v8} | {v7}: 3 partitions."""
    g, q, _ = fig4()
    cst = cst_ref.build_cst(g, q.qlabel, q.qedges)
    po = [0, 1, 3, 2]
    parts = cst_ref.partition(cst, po, delta_s=320)
    assert [cst_ref.image_bytes(cst, po, s) for _, s in parts] == [320, 304]
    parts = cst_ref.partition(cst, po, delta_s=304)
    assert [cst_ref.image_bytes(cst, po, s) for _, s in parts] == [288, 288, 304]
    assert [sorted(s[1]) for _, s in parts] == [[3], [5], [4]]
    parts = cst_ref.partition(cst, [0, 1, 2, 3], delta_s=1 << 20, delta_d=2)
    assert [sorted(s[2]) for _, s in parts] == [[6, 8], [6, 8], [7]]
    assert len(parts) == 3
    for _, s in parts:
        assert cst_ref.max_list_len(cst, s) <= 2


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
            assert wc + wf == sum(w)
            assert wc == sum(sum(w[lo:hi]) for lo, hi in host)
            if delta == 0.0:
                assert host == []
            if host:
                assert wc < delta * (wc + wf)
