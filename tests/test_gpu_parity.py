"""GPU parity: the HIP path against the CPU oracle (bit-exact counts and sorted lists).

Every test calls through the C ABI (ctypes binding).  Expected values come from
``oracle`` (and, for CST contents, from ``oracle.cst_ref``) on the same seeded
inputs.
"""

from __future__ import annotations

import json
import os
import sys

import numpy as np
import pytest

import oracle
from oracle import cst_ref
import closed_forms as cf
from synth import make_graph, query_set
from test_oracle import random_connected_query, random_tiny_graph
from gpu_common import MODES, ctx, gpu_count, gpu_graph, gpu_rows

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _oracle_rows(g, q):
    r = oracle.match(g, q, list_rows=True, cap=1 << 22)
    assert r.status == oracle.OK
    return r.count, [tuple(int(x) for x in row) for row in r.rows]


def test_library_loads_and_reports_device():
    from paper_2102_10768_amd import cstm

    lib = cstm.load_library()
    assert b"gfx950" in lib.cstm_version()
    assert ctx().lds_bytes() >= 64 * 1024


def test_fig4_fixture_matches_reference_and_oracle():
    d = json.load(open(os.path.join(GOLDEN, "fig4_fixture.json")))
    g = cf.graph_from_edges(d["n"], [tuple(e) for e in d["edges"]], d["labels"], "fig4")
    q = cf.query(d["query"]["qlabel"], [tuple(e) for e in d["query"]["qedges"]])
    say("fig4: load")
    G = gpu_graph(g)
    from paper_2102_10768_amd import cstm

    say("fig4: build")
    c = cstm.CST(ctx(), G, q.qlabel, q.qedges)
    ref = cst_ref.build_cst(g, q.qlabel, q.qedges)
    info = c.info()
    assert info["root"] == ref.root
    assert info["parent"] == ref.parent
    assert info["order"] == cst_ref.path_order(ref)
    for u in range(q.k):
        assert c.candidates(u).tolist() == ref.cand[u]
    say("fig4: enumerate")
    n, rows = c.list(64)
    want_n, want_rows = _oracle_rows(g, q)
    assert n == want_n == 3
    assert sorted(tuple(int(x) for x in r) for r in rows.cpu().numpy()) == want_rows
    c.close()


def _c1():
    return make_graph({"kind": "er", "n": 3000, "p": 10 / 2999, "seed": 11, "labels": {"kind": "uniform", "L": 20}})


@pytest.mark.parametrize("mode", MODES)
def test_small_config_counts_and_lists(mode):
    g = _c1()
    G = gpu_graph(g, mode)
    for i, q in enumerate(query_set(g, [4] * 8, 21) + query_set(g, [5, 6, 7, 8], 22)):
        say(f"small config query {i} ({mode}): labels {q.qlabel.tolist()} edges {q.qedges.tolist()}")
        want_n, want_rows = _oracle_rows(g, q)
        n, rows = gpu_rows(G, q)
        assert n == want_n
        assert rows == want_rows


def test_candidate_sets_match_reference():
    g = _c1()
    G = gpu_graph(g)
    from paper_2102_10768_amd import cstm

    for q in query_set(g, [4, 5, 6, 7] * 2, 55):
        ref = cst_ref.build_cst(g, q.qlabel, q.qedges)
        c = cstm.CST(ctx(), G, q.qlabel, q.qedges)
        info = c.info()
        assert info["root"] == ref.root and info["parent"] == ref.parent
        assert info["order"] == cst_ref.path_order(ref)
        for u in range(q.k):
            assert c.candidates(u).tolist() == ref.cand[u]
        assert info["tree_entries"] == sum(len(l) for lists in ref.tree_adj.values() for l in lists.values())
        c.close()


@pytest.mark.parametrize("mode", MODES)
@pytest.mark.parametrize("seed", range(30))
def test_random_tiny_graphs(seed, mode):
    rng = np.random.default_rng(1000 + seed)
    g = random_tiny_graph(rng)
    q = random_connected_query(rng, L=int(g.label.max()) + 1)
    say(f"tiny seed {seed} ({mode}): n={g.n} k={q.k} m_q={q.m_q}")
    G = gpu_graph(g, mode)
    want_n, want_rows = _oracle_rows(g, q)
    n, rows = gpu_rows(G, q)
    assert n == want_n
    assert rows == want_rows


def test_partition_budget_does_not_change_results():
    g = make_graph({"kind": "chung_lu", "n": 5000, "m": 40000, "gamma": 2.3, "seed": 31,
                    "labels": {"kind": "zipf", "L": 8, "s": 1.0}})
    G = gpu_graph(g)
    qs = query_set(g, [4, 5, 6], 32)
    for q in qs:
        r = oracle.match(g, q, node_budget=5 * 10**8)
        if r.status != oracle.OK:
            continue
        counts = []
        for budget in (0, 16384, 4096, 1024):
            n, info = gpu_count(G, q, budget)
            say(f"budget {budget}: count {n} parts {info['n_parts']} max {info['max_part_bytes']}")
            counts.append(n)
            if budget:
                assert info["max_part_bytes"] <= budget
        assert counts == [r.count] * len(counts)


def test_partition_count_matches_reference_rule():
    g = make_graph({"kind": "er", "n": 300, "p": 0.05, "seed": 9, "labels": {"kind": "uniform", "L": 3}})
    G = gpu_graph(g)
    for q in query_set(g, [3, 4, 5], 10):
        ref = cst_ref.build_cst(g, q.qlabel, q.qedges)
        order = cst_ref.path_order(ref)
        for budget in (2048, 512):
            parts = cst_ref.partition(ref, order, delta_s=budget)
            n, info = gpu_count(G, q, budget)
            assert info["n_parts"] == len(parts)
            assert n == oracle.count(g, q)


@pytest.mark.parametrize("mode", MODES)
def test_edge_cases_single_vertex_absent_label_and_k2(mode):
    g = _c1()
    G = gpu_graph(g, mode)
    for lab in (0, 7, 19):
        n, _ = gpu_count(G, cf.query([lab], []))
        assert n == int((g.label == lab).sum())
    n, _ = gpu_count(G, cf.query([99], []))
    assert n == 0
    n, _ = gpu_count(G, cf.query([0, 99, 1], [(0, 1), (1, 2)]))
    assert n == 0
    for la, lb in [(0, 1), (3, 3)]:
        q = cf.query([la, lb], [(0, 1)])
        want_n, want_rows = _oracle_rows(g, q)
        n, rows = gpu_rows(G, q)
        assert n == want_n and rows == want_rows


@pytest.mark.parametrize("mode", MODES)
def test_closed_forms_on_gpu(mode):
    from math import perm

    G = gpu_graph(cf.complete(9), mode)
    for k in range(1, 7):
        n, _ = gpu_count(G, cf.clique_query([0] * k), partition=mode == "lds")
        assert n == perm(9, k)
    G = gpu_graph(cf.complete_bipartite(4, 5), mode)
    assert gpu_count(G, cf.cycle_query(3), partition=False)[0] == 0
    assert gpu_count(G, cf.cycle_query(4), partition=False)[0] == cf.c4_in_complete_bipartite(4, 5)


@pytest.mark.parametrize("mode", MODES)
def test_batch_matches_individual_counts(mode):
    g = _c1()
    G = gpu_graph(g, mode)
    from paper_2102_10768_amd import cstm

    qs = query_set(g, [3, 4, 5, 6] * 3, 71)
    csts = [cstm.CST(ctx(mode), G, q.qlabel, q.qedges) for q in qs]
    for i, c in enumerate(csts):
        if mode == "lds" or (mode == "auto" and i % 2):
            c.partition(4096)
    got = cstm.batch_count(ctx(mode), csts)
    want = [oracle.count(g, q) for q in qs]
    assert got == want
    for c in csts:
        c.close()


def test_malformed_inputs_rejected():
    from paper_2102_10768_amd import cstm

    g = cf.graph_from_edges(4, [(0, 1), (1, 2)], [0, 0, 0, 0])
    bad_col = g.col.copy()
    bad_col[0] = 3  # row 0 now points at 3, but 3 does not point back
    with pytest.raises(cstm.CstmError):
        cstm.Graph(ctx(), g.row_ptr, bad_col, g.label)
    G = gpu_graph(g)
    with pytest.raises(cstm.CstmError):
        cstm.CST(ctx(), G, [0, 0, 0], [(0, 1)])  # disconnected
    with pytest.raises(cstm.CstmError):
        cstm.CST(ctx(), G, [0, 0], [(0, 0)])  # self-loop


@pytest.mark.parametrize("mode", MODES)
def test_maximum_query_size_and_edgeless_graphs(mode):
    """k = 32 (the largest query): P_32 has 2n embeddings in C_n and 2(n-31)
    in P_n; on a graph without edges only single-vertex queries match."""
    from paper_2102_10768_amd import cstm

    G = gpu_graph(cf.cycle(40), mode)
    assert gpu_count(G, cf.path_query(32), partition=mode == "lds")[0] == cf.path_in_cycle(40, 32)
    G = gpu_graph(cf.path(40), mode)
    assert gpu_count(G, cf.path_query(32), partition=mode == "lds")[0] == cf.path_in_path(40, 32)
    with pytest.raises(cstm.CstmError):
        gpu_count(G, cf.path_query(33))
    empty = cf.graph_from_edges(50, [], np.arange(50) % 3)
    G = gpu_graph(empty, mode)
    assert gpu_count(G, cf.query([1], []))[0] == int((empty.label == 1).sum())
    assert gpu_count(G, cf.query([0, 0], [(0, 1)]))[0] == 0


def test_workload_estimate_matches_reference_dp():
    """W_CST on the device (Section V-C) equals the reference DP exactly, and
    the number of embeddings for a tree query with pairwise-distinct labels."""
    g = _c1()
    G = gpu_graph(g)
    from paper_2102_10768_amd import cstm

    for q in query_set(g, [3, 4, 5, 6, 7] * 3, 57):
        ref = cst_ref.build_cst(g, q.qlabel, q.qedges)
        _, w_ref = cst_ref.workload(ref)
        c = cstm.CST(ctx(), G, q.qlabel, q.qedges)
        w = c.workload()
        assert w == cst_ref.saturate_u64(w_ref)
        n = c.count()
        c.close()
        assert w >= n
        if cf.is_tree_with_distinct_labels(q):
            assert w == n
    # the worked example of Section V-C on the fixture graph
    fx = json.load(open(os.path.join(GOLDEN, "fig4_fixture.json")))
    gf = cf.graph_from_edges(fx["n"], [tuple(e) for e in fx["edges"]], fx["labels"])
    qf = cf.query(fx["query"]["qlabel"], [tuple(e) for e in fx["query"]["qedges"]])
    ref = cst_ref.build_cst(gf, qf.qlabel, qf.qedges)
    c = cstm.CST(ctx(), gpu_graph(gf), qf.qlabel, qf.qedges)
    assert c.workload() == cst_ref.workload(ref)[1] == 7
    c.close()


def test_workload_is_exact_beyond_double_precision_and_saturates():
    """W_CST of a star K_{1,s} (one label) in K_n is n (n-1)^s (root = centre):
    K_{1,6} in K_300 is 300 * 299^6 ~ 2.1e17 > 2^53, held exactly; K_{1,8} in
    K_400 is ~2.6e23 > 2^64 - 1, held as 2^64 - 1.  The reference DP
    (Python integers) agrees on the first."""
    from paper_2102_10768_amd import cstm

    for n, s_ in ((300, 6), (400, 8)):
        g = cf.complete(n)
        q = cf.star_query(s_)
        c = cstm.CST(ctx(), gpu_graph(g), q.qlabel, q.qedges)
        want = n * (n - 1) ** s_
        assert c.info()["root"] == 0
        assert c.workload() == cst_ref.saturate_u64(want)
        c.close()
        if n == 300:
            assert cst_ref.workload(cst_ref.build_cst(g, q.qlabel, q.qedges))[1] == want
    assert 300 * 299 ** 6 > 2 ** 53 and 400 * 399 ** 8 > 2 ** 64


def test_fig4_partition_counts_and_image_bytes_by_hand():
    """Algorithm 2 on the fixture graph under the path order u0, u1, u3, u2
    (Section V-B), values summed by hand: the full image is 352 B; at a
    320-byte budget the root splits into {v1} (320 B) and {v2} (304 B); at
    304 B {v1} splits again at u1 into two 288-byte images."""
    from paper_2102_10768_amd import cstm

    fx = json.load(open(os.path.join(GOLDEN, "fig4_fixture.json")))
    gf = cf.graph_from_edges(fx["n"], [tuple(e) for e in fx["edges"]], fx["labels"])
    qf = cf.query(fx["query"]["qlabel"], [tuple(e) for e in fx["query"]["qedges"]])
    G = gpu_graph(gf, "lds")
    for budget, sizes in ((1024, [352]), (320, [320, 304]), (304, [288, 288, 304])):
        c = cstm.CST(ctx("lds"), G, qf.qlabel, qf.qedges)
        assert c.info()["order"][:4] == [0, 1, 3, 2]
        assert c.partition(budget) == len(sizes)
        info = c.info()
        assert info["part_bytes"] == sum(sizes) and info["max_part_bytes"] == max(sizes)
        assert c.count() == 3
        c.close()


def test_batch_seeding_order_does_not_change_counts():
    g = _c1()
    G = gpu_graph(g, "hbm")
    from paper_2102_10768_amd import cstm

    qs = query_set(g, [3, 4, 5, 6] * 4, 73)
    csts = [cstm.CST(ctx("hbm"), G, q.qlabel, q.qedges) for q in qs]
    given = cstm.batch_count(ctx("hbm"), csts)
    ctx("hbm").tune = {"batch_order": 1}
    try:
        by_w = cstm.batch_count(ctx("hbm"), csts)
    finally:
        ctx("hbm").tune = {"batch_order": 0}
    alone = [c.count() for c in csts]
    for c in csts:
        c.close()
    assert by_w == given == alone


def _sorted_rows(c):
    n, rows = c.list(1 << 16)
    return n, sorted(tuple(int(x) for x in row) for row in rows.cpu().numpy())


def _tree_orders(parent, root, rng, n):
    """n random orders that start at the root and put every vertex after its
    tree parent (the orders Section VII-C varies)."""
    k = len(parent)
    out = []
    for _ in range(n):
        order, placed = [root], {root}
        while len(order) < k:
            ready = [u for u in range(k) if u not in placed and parent[u] in placed]
            u = int(rng.choice(ready))
            order.append(u)
            placed.add(u)
        out.append(order)
    return out


@pytest.mark.gpu
@pytest.mark.parametrize("mode", MODES)
def test_caller_matching_order_keeps_embeddings(mode):
    g = _c1()
    G = gpu_graph(g, mode)
    from paper_2102_10768_amd import cstm

    rng = np.random.default_rng(91)
    for q in query_set(g, [4, 5, 6, 7], 92):
        base = cstm.CST(ctx(mode), G, q.qlabel, q.qedges)
        info = base.info()
        want_n = base.count()
        want_rows = _sorted_rows(base)
        base.close()
        assert want_n == oracle.match(g, q).count
        for order in _tree_orders(info["parent"], info["root"], rng, 3):
            c = cstm.CST(ctx(mode), G, q.qlabel, q.qedges, order=order)
            assert c.info()["order"] == order
            assert c.count() == want_n
            assert _sorted_rows(c) == want_rows
            c.close()
        # an order that breaks the tree (root not first, or a child before its parent)
        bad = list(info["order"])
        bad[0], bad[1] = bad[1], bad[0]
        with pytest.raises(cstm.CstmError) as e:
            cstm.CST(ctx(mode), G, q.qlabel, q.qedges, order=bad)
        assert e.value.status == cstm.EINVAL
        with pytest.raises(cstm.CstmError):
            cstm.CST(ctx(mode), G, q.qlabel, q.qedges, order=[info["root"]] * q.k)


def _constraint_first(qedges, k, root, parent):
    """The order_rule = 1 matching order, restated: after the root, repeatedly
    the vertex whose tree parent is placed with the most placed query
    neighbours, then the larger query degree, then the smaller id."""
    adj = [set() for _ in range(k)]
    for a, b in np.asarray(qedges).reshape(-1, 2):
        adj[int(a)].add(int(b))
        adj[int(b)].add(int(a))
    order, placed = [root], {root}
    while len(order) < k:
        ready = [u for u in range(k) if u not in placed and parent[u] in placed]
        u = max(ready, key=lambda w: (len(adj[w] & placed), len(adj[w]), -w))
        order.append(u)
        placed.add(u)
    return order


def test_constraint_first_order_rule_keeps_every_embedding():
    """Built with order_rule = 1, a CST follows the restated rule and gives the
    oracle's count and sorted listing (Section VII-C: the order changes only
    the work).  Queries of 3..8 vertices with non-tree edges, on the small ER
    workload and on random tiny graphs."""
    from paper_2102_10768_amd import cstm
    from gpu_common import gpu_graph_in

    c = cstm.Context(0, tune={"enum_mode": cstm.MODE_HBM, "order_rule": 1})
    g = make_graph({"kind": "er", "n": 300, "p": 0.05, "seed": 9, "labels": {"kind": "uniform", "L": 3}})
    G = gpu_graph_in(c, g)
    qs = query_set(g, [3, 4, 5, 6, 7, 8] * 3, 91)
    assert sum(q.m_q > q.k - 1 for q in qs) >= 3  # some carry non-tree edges
    for q in qs:
        cs = cstm.CST(c, G, q.qlabel, q.qedges)
        info = cs.info()
        assert info["order"] == _constraint_first(q.qedges, q.k, info["root"], info["parent"])
        if q.k <= 5:
            n, rows = cs.list(1 << 20)
            want = oracle.match(g, q, list_rows=True)
            assert n == want.count
            assert sorted(tuple(int(x) for x in r) for r in rows.cpu().numpy()) == [
                tuple(int(x) for x in r) for r in want.rows]
        else:
            assert cs.count() == oracle.count(g, q)
        cs.close()
    G.close()
    for seed in range(12):
        rng = np.random.default_rng(8800 + seed)
        gt = random_tiny_graph(rng)
        q = random_connected_query(rng, L=int(gt.label.max()) + 1)
        Gt = gpu_graph_in(c, gt)
        cs = cstm.CST(c, Gt, q.qlabel, q.qedges)
        assert cs.count() == oracle.count(gt, q)
        cs.close()
        Gt.close()
    c.close()


def test_label_edge_table_matches_the_csr():
    """The per-graph count of edges between label pairs (which bounds the
    construction buffers) equals a count made directly from the CSR; above 128
    labels no table is made."""
    from synth.graphs import Graph, erdos_renyi, uniform_labels, zipf_labels

    graphs = [_c1()]
    for seed, L in ((51, 1), (52, 7), (53, 128), (54, 129)):
        row_ptr, col = erdos_renyi(600, 0.02, seed)
        lab = uniform_labels(600, L, seed) if L != 7 else zipf_labels(600, L, 1.0, seed)
        lab[0] = L - 1  # the largest label occurs
        graphs.append(Graph(600, row_ptr, col, lab, f"er{L}"))
    for g in graphs:
        G = gpu_graph(g)
        L = int(g.label.max()) + 1
        t = G.label_edges()
        say(f"{g.name}: L={L}, table {'none' if t is None else t.shape}")
        if L > 128:
            assert t is None
            continue
        src = np.repeat(np.arange(g.n), np.diff(g.row_ptr))
        want = np.zeros((L, L), dtype=np.uint64)
        np.add.at(want, (g.label[src], g.label[g.col]), 1)
        assert t.shape == (L, L) and np.array_equal(t, want)
        assert int(t.sum()) == int(g.row_ptr[-1])


def test_sparse_label_space_takes_the_64_bit_keys():
    """Labels up to 2^20 with a label group of 2,600 vertices need 21 + 12 = 33
    key bits, so G keeps 64-bit packed keys and 64-bit label-grouped rows (and
    no label-pair table): counts and sorted lists still equal the oracle's."""
    from synth.graphs import Graph, erdos_renyi

    rng = np.random.default_rng(61)
    n = 3000
    row_ptr, col = erdos_renyi(n, 10 / (n - 1), 61)
    lab = np.zeros(n, dtype=np.int32)
    lab[rng.choice(n, 300, replace=False)] = 1
    lab[rng.choice(n, 100, replace=False)] = 1 << 20
    g = Graph(n, row_ptr, col, lab, "sparse-labels")
    G = gpu_graph(g)
    assert G.label_edges() is None  # more than 128 labels
    from synth import Query

    big = 1 << 20  # queries that use the largest label too
    small = query_set(g, [2, 3, 3], 62) + [
        Query(np.array([big, 0], dtype=np.int32), np.array([[0, 1]], dtype=np.int32)),
        Query(np.array([0, big, 1], dtype=np.int32), np.array([[0, 1], [1, 2]], dtype=np.int32)),
    ]  # listed: at most a few 10^5 rows
    large = query_set(g, [4, 5], 63)     # counted
    for mode in MODES:
        Gm = gpu_graph(g, mode)
        for q in small:
            say(f"sparse labels ({mode}): k={q.k} labels={sorted(set(q.qlabel))} (lists)")
            want_n, want_rows = _oracle_rows(g, q)
            n_got, rows = gpu_rows(Gm, q)
            assert n_got == want_n and rows == want_rows
        for q in large:
            say(f"sparse labels ({mode}): k={q.k} labels={sorted(set(q.qlabel))} (counts)")
            want = oracle.match(g, q)
            assert want.status == oracle.OK
            assert gpu_count(Gm, q, partition=mode == "lds")[0] == want.count
