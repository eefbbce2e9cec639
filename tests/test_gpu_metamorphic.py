"""Metamorphic relations and failure injection through the C ABI.

Relations that hold for any correct matcher (Section II-A's definition):
renumbering G's vertices, renaming labels consistently in G and q, or
renumbering q's vertices leaves the count unchanged; the disjoint union of G
with itself doubles the count of a connected query; adding edges to G never
lowers it.  Every count is also compared with the oracle on the transformed
input.  Failure injection: an allocator callback that runs dry must surface
as CSTM_ENOMEM, and the context must keep working once memory returns.
"""

from __future__ import annotations

import ctypes
import json
import os

import numpy as np
import pytest

import closed_forms as cf
import oracle
from gpu_common import ctx, gpu_graph
from synth import Query, make_graph, query_set

pytestmark = pytest.mark.gpu


def _c1():
    W = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "c1.json")))
    return make_graph(W["workload"]["graph"])


def _edges(g):
    src = np.repeat(np.arange(g.n), np.diff(g.row_ptr))
    keep = src < g.col
    return np.stack([src[keep], g.col[keep]], axis=1)


def _count(G, q):
    from paper_2102_10768_amd import cstm

    c = cstm.CST(G.ctx, G, q.qlabel, q.qedges)
    n = c.count()
    c.close()
    return n


def _queries(g, seed):
    return query_set(g, [3, 4, 5, 6], seed)


def test_vertex_renumbering_and_label_renaming():
    g = _c1()
    qs = _queries(g, 501)
    base = [_count(gpu_graph(g, "hbm"), q) for q in qs]
    assert base == [oracle.count(g, q) for q in qs]
    rng = np.random.default_rng(502)
    perm = rng.permutation(g.n)
    e = _edges(g)
    lab = np.empty_like(g.label)
    lab[perm] = g.label
    gp = cf.graph_from_edges(g.n, perm[e], lab, "renumbered")
    Gp = gpu_graph(gp, "hbm")
    assert [_count(Gp, q) for q in qs] == base
    # labels renamed by a bijection, in G and in every query
    L = int(g.label.max()) + 1
    ren = rng.permutation(L).astype(np.int32)
    gr = cf.graph_from_edges(g.n, e, ren[g.label], "renamed")
    Gr = gpu_graph(gr, "lds")
    got = [_count(Gr, Query(qlabel=ren[q.qlabel], qedges=q.qedges)) for q in qs]
    assert got == base


def test_query_vertex_renumbering():
    g = _c1()
    G = gpu_graph(g, "auto")
    from paper_2102_10768_amd import cstm

    rng = np.random.default_rng(503)
    for q in _queries(g, 504):
        p = rng.permutation(q.k)  # new id of old vertex i is p[i]
        ql = np.empty_like(q.qlabel)
        ql[p] = q.qlabel
        qe = np.sort(p[q.qedges], axis=1).astype(np.int32)
        q2 = Query(qlabel=ql, qedges=qe)
        c1 = cstm.CST(ctx("auto"), G, q.qlabel, q.qedges)
        c2 = cstm.CST(ctx("auto"), G, q2.qlabel, q2.qedges)
        n1, r1 = c1.list(1 << 16)
        n2, r2 = c2.list(1 << 16)
        c1.close()
        c2.close()
        assert n1 == n2 == oracle.count(g, q)
        # row[u] of the renumbered query is row[p^-1(u)] of the original
        a = sorted(tuple(int(x) for x in row) for row in r1.cpu().numpy())
        b = sorted(tuple(int(x) for x in row[p]) for row in r2.cpu().numpy())
        assert a == b


def test_disjoint_union_doubles_and_added_edges_never_lower():
    g = _c1()
    qs = _queries(g, 505)
    base = [_count(gpu_graph(g, "hbm"), q) for q in qs]
    e = _edges(g)
    gu = cf.graph_from_edges(2 * g.n, np.concatenate([e, e + g.n]), np.concatenate([g.label, g.label]), "union")
    Gu = gpu_graph(gu, "hbm")
    assert [_count(Gu, q) for q in qs] == [2 * b for b in base]
    rng = np.random.default_rng(506)
    extra = rng.integers(0, g.n, size=(2000, 2))
    extra = extra[extra[:, 0] != extra[:, 1]]
    ga = cf.graph_from_edges(g.n, np.concatenate([e, np.sort(extra, axis=1)]), g.label, "more edges")
    Ga = gpu_graph(ga, "lds")
    more = [_count(Ga, q) for q in qs]
    assert all(m >= b for m, b in zip(more, base))
    assert more == [oracle.count(ga, q) for q in qs]


def test_allocator_running_dry_reports_enomem_and_recovers():
    import torch

    from paper_2102_10768_amd import cstm

    lib = cstm.load_library()
    state = {"left": 0, "live": 0}

    def _alloc(nbytes, user):
        if state["left"] <= 0:
            return None
        state["left"] -= 1
        state["live"] += 1
        return torch.cuda.caching_allocator_alloc(int(nbytes), 0)

    def _free(ptr, user):
        state["live"] -= 1
        torch.cuda.caching_allocator_delete(ptr)

    alloc, free = cstm.ALLOC_FN(_alloc), cstm.FREE_FN(_free)
    t = cstm.cstm_tune(enum_mode=cstm.MODE_HBM)
    h = ctypes.c_void_p()
    state["left"] = 1 << 30
    assert lib.cstm_ctx_create(0, alloc, free, None, ctypes.byref(t), ctypes.byref(h)) == 0
    g = _c1()
    rp = torch.from_numpy(g.row_ptr).cuda()
    col = torch.from_numpy(g.col).cuda()
    lab = torch.from_numpy(g.label).cuda()
    graph = ctypes.c_void_p()
    assert lib.cstm_graph_load(h, g.n, int(g.col.shape[0]), rp.data_ptr(), col.data_ptr(), lab.data_ptr(), 1,
                               None, ctypes.byref(graph)) == 0
    q = _queries(g, 507)[3]
    ql = np.ascontiguousarray(q.qlabel, dtype=np.int32)
    qe = np.ascontiguousarray(q.qedges, dtype=np.int32)
    want = oracle.count(g, q)
    torch.cuda.synchronize()
    failures = 0
    for budget in (0, 1, 2, 3, 5, 8, 13, 21, 34):
        state["left"] = budget
        cst = ctypes.c_void_p()
        st = lib.cstm_cst_build(h, graph, q.k, ql.ctypes.data, q.m_q, qe.ctypes.data, None, ctypes.byref(cst))
        if st == 0:
            n = ctypes.c_uint64()
            st = lib.cstm_enumerate(cst, 0, 0, None, 0, ctypes.byref(n), None, ctypes.c_double(0.0), None)
            if st == 0:
                assert n.value == want
            else:
                assert st == cstm.ENOMEM
                failures += 1
            lib.cstm_cst_free(cst)
        else:
            assert st == cstm.ENOMEM, (budget, st)
            assert not cst.value
            failures += 1
        torch.cuda.synchronize()
    assert failures >= 1
    # memory back: the same context builds and counts again
    state["left"] = 1 << 30
    cst = ctypes.c_void_p()
    assert lib.cstm_cst_build(h, graph, q.k, ql.ctypes.data, q.m_q, qe.ctypes.data, None, ctypes.byref(cst)) == 0
    n = ctypes.c_uint64()
    assert lib.cstm_enumerate(cst, 0, 0, None, 0, ctypes.byref(n), None, ctypes.c_double(0.0), None) == 0
    assert n.value == want
    lib.cstm_cst_free(cst)
    lib.cstm_graph_free(graph)
    lib.cstm_ctx_destroy(h)
    torch.cuda.synchronize()
    # every block taken through the callback, failed calls included, came back
    assert state["live"] == 0, state
