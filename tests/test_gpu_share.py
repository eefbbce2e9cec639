"""Host-core share (Algorithm 3, Section V-C) through ``cstm_enumerate_shared``.

The total must equal the oracle's count for every delta; the split must obey
the rule of Algorithm 3 (the host's workload stays below delta times the
whole, the two shares add up to W_CST) and delta = 0 must leave the host idle.
"""

from __future__ import annotations

from fractions import Fraction
from math import perm

import numpy as np
import pytest

import closed_forms as cf
import oracle
from oracle import cst_ref
from gpu_common import ctx, gpu_graph
from synth import make_graph, query_set
from test_oracle import random_connected_query, random_tiny_graph

pytestmark = pytest.mark.gpu

DELTAS = (0.0, 0.05, 0.3, 0.7, 1.0)


def _c1():
    import json
    import os

    W = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "c1.json")))
    return make_graph(W["workload"]["graph"])


def _check_split(c, delta, n, st):
    assert st["count_host"] + st["count_device"] == n
    w = c.workload()
    assert st["w_host"] + st["w_device"] == w
    if delta == 0.0:
        assert st["groups_host"] == 0 and st["count_host"] == 0 and st["w_host"] == 0
    if st["groups_host"]:
        assert Fraction(st["w_host"]) < Fraction(delta) * (st["w_host"] + st["w_device"])
    assert st["groups_device"] >= 1


@pytest.mark.parametrize("mode", ["lds", "hbm"])
def test_shared_counts_match_oracle(mode):
    from paper_2102_10768_amd import cstm

    g = _c1()
    G = gpu_graph(g, mode)
    for q in query_set(g, [3, 4, 5, 6, 7], 211):
        want = oracle.count(g, q)
        c = cstm.CST(ctx(mode), G, q.qlabel, q.qedges)
        for delta in DELTAS:
            for runs in (0, 1, 7):
                n, st = c.count_shared(delta, n_runs=runs, host_threads=3)
                assert n == want, (q.k, delta, runs, st)
                _check_split(c, delta, n, st)
        c.close()


def test_shared_on_tiny_graphs_and_closed_forms():
    from paper_2102_10768_amd import cstm

    for seed in range(6):
        rng = np.random.default_rng(4000 + seed)
        g = random_tiny_graph(rng, n=int(rng.integers(10, 60)), L=int(rng.integers(1, 4)),
                              p=float(rng.uniform(0.1, 0.4)))
        G = gpu_graph(g, "hbm")
        for j in range(4):
            q = random_connected_query(rng, L=int(g.label.max()) + 1)
            want = oracle.count(g, q)
            c = cstm.CST(ctx("hbm"), G, q.qlabel, q.qedges)
            for delta in (0.2, 0.9):
                n, st = c.count_shared(delta, n_runs=5, host_threads=2)
                assert n == want
                _check_split(c, delta, n, st)
            c.close()
    # one label everywhere: the host side must apply injectivity and the
    # non-tree checks (cliques have one non-tree edge per extra pair)
    G = gpu_graph(cf.complete(9), "hbm")
    for k in range(1, 7):
        q = cf.clique_query([0] * k)
        c = cstm.CST(ctx("hbm"), G, q.qlabel, q.qedges)
        n, st = c.count_shared(0.6, n_runs=9, host_threads=4)
        assert n == perm(9, k)
        _check_split(c, 0.6, n, st)
        if k > 1:
            assert st["groups_host"] > 0 and st["count_host"] > 0
        c.close()


def test_shared_rejects_bad_arguments():
    from paper_2102_10768_amd import cstm

    g = _c1()
    G = gpu_graph(g, "hbm")
    q = query_set(g, [4], 5)[0]
    c = cstm.CST(ctx("hbm"), G, q.qlabel, q.qedges)
    for bad in (dict(delta=-0.1), dict(delta=1.5), dict(delta=float("nan")), dict(delta=0.1, n_runs=-1),
                dict(delta=0.1, host_threads=-2), dict(delta=0.1, host_threads=1000)):
        with pytest.raises(cstm.CstmError) as e:
            c.count_shared(**bad)
        assert e.value.status == cstm.EINVAL
    # the CST still counts normally afterwards
    assert c.count() == oracle.count(g, q)
    c.close()


def test_split_equals_the_reference_rule():
    """The runs each side receives and W_C, W_F equal the reference
    restatement of Algorithm 3 on the reference DP's c_root values."""
    from paper_2102_10768_amd import cstm

    g = _c1()
    G = gpu_graph(g, "hbm")
    for q in query_set(g, [4, 5, 6, 7], 213):
        ref = cst_ref.build_cst(g, q.qlabel, q.qedges)
        cmap, W = cst_ref.workload(ref)
        c = cstm.CST(ctx("hbm"), G, q.qlabel, q.qedges)
        assert c.info()["root"] == ref.root
        roots = c.candidates(ref.root).tolist()
        assert roots == ref.cand[ref.root]
        weights = [cmap[ref.root].get(v, 0) for v in roots]
        assert c.workload() == W
        for delta in (0.05, 0.3, 0.7):
            for runs in (0, 3, 11):
                _, st = c.count_shared(delta, n_runs=runs, host_threads=2)
                host, dev, wc, wf = cst_ref.share_split(weights, delta, runs)
                assert (st["groups_host"], st["groups_device"]) == (len(host), len(dev)), (q.k, delta, runs)
                assert (st["w_host"], st["w_device"]) == (wc, wf)
        c.close()
