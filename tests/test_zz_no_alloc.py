"""The no-allocation entry point (``cstm_enumerate_noalloc``) against ``cstm_enumerate``.

Both are called through the C ABI on the same CSTs, two or more calls in a
row with the later inputs smaller than the first, so that anything the fixed
scratch array keeps from an earlier call would show.  Counts must be equal
(integers: bit-exact), equal to closed forms where one exists, and the
no-allocation calls must not reach the context's allocator.
"""

from __future__ import annotations

import ctypes
import json
import os

import pytest

import closed_forms as cf
from synth import Query, make_graph
from gpu_common import gpu_graph_in

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _counted_context(log):
    import torch
    from paper_2102_10768_amd import cstm

    def alloc(nbytes):
        log.append(nbytes)
        return torch.cuda.caching_allocator_alloc(nbytes, 0)

    def free(ptr):
        torch.cuda.caching_allocator_delete(ptr)

    return cstm.Context(0, tune={"enum_mode": cstm.MODE_HBM}, allocator=(alloc, free))


def _abi_counts(c, limit=0):
    """(cstm_enumerate count, cstm_enumerate_noalloc count), both raw C-ABI calls."""
    from paper_2102_10768_amd import cstm

    lib = cstm.load_library()
    stream = cstm._stream_ptr(None)
    a, w = ctypes.c_uint64(), ctypes.c_uint64()
    cstm._check(lib.cstm_enumerate(c.handle, 0, int(limit), None, 0, ctypes.byref(a), ctypes.byref(w), 0.0, stream))
    b = ctypes.c_uint64(12345)
    cstm._check(lib.cstm_enumerate_noalloc(c.handle, int(limit), ctypes.byref(b), 0.0, stream))
    return a.value, b.value


def test_noalloc_equals_enumerate_on_shrinking_inputs():
    from paper_2102_10768_amd import cstm

    log = []
    ctx = _counted_context(log)
    # first call: 4-cliques in K_200 (200 root candidates, 1.55e9 embeddings)
    big = gpu_graph_in(ctx, cf.complete(200))
    q = cf.clique_query([0] * 4)
    c = cstm.CST(ctx, big, q.qlabel, q.qedges)
    before = len(log)
    n_big = c.count_noalloc()
    assert len(log) == before, "the no-allocation entry point reached the allocator"
    assert n_big == cf.clique_host_count(200, 4) == 200 * 199 * 198 * 197
    got = _abi_counts(c)
    assert got == (n_big, n_big)
    # the same CST with a count limit: exactly min(total, limit)
    assert _abi_counts(c, limit=1000) == (1000, 1000)
    c.close()
    # then smaller inputs: the small ER workload's stored queries (fewer roots, small counts)
    W = json.load(open(os.path.join(GOLDEN, "c1.json")))
    g = make_graph(W["workload"]["graph"])
    small = gpu_graph_in(ctx, g)
    for d in W["queries"]:
        qq = Query.from_dict(d)
        cs = cstm.CST(ctx, small, qq.qlabel, qq.qedges)
        before = len(log)
        n = cs.count_noalloc()
        assert len(log) == before
        assert n == d["count"]
        assert _abi_counts(cs) == (d["count"], d["count"])
        cs.close()
    # a query with an empty candidate set, and a one-vertex query
    for qq, want in ((cf.query([99], []), 0), (cf.query([3], []), int((g.label == 3).sum()))):
        cs = cstm.CST(ctx, small, qq.qlabel, qq.qedges)
        assert cs.count_noalloc() == want
        assert _abi_counts(cs) == (want, want)
        cs.close()
    small.close()
    big.close()
    ctx.close()


def test_noalloc_rejects_null_arguments():
    from paper_2102_10768_amd import cstm

    lib = cstm.load_library()
    out = ctypes.c_uint64()
    assert lib.cstm_enumerate_noalloc(None, 0, ctypes.byref(out), 0.0, None) == cstm.EINVAL
