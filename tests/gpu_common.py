"""Shared helpers for the GPU tests: one device context per test session."""

from __future__ import annotations

import numpy as np
import pytest

_CTX = None


def ctx():
    global _CTX
    if _CTX is None:
        import torch

        if not torch.cuda.is_available():
            pytest.fail("GPU test collected on a machine without a GPU")
        from paper_2102_10768_amd import cstm

        _CTX = cstm.Context(0)
    return _CTX


def gpu_graph(g):
    """Load a synth.Graph through the device-pointer path (torch tensors)."""
    import torch
    from paper_2102_10768_amd import cstm

    rp = torch.from_numpy(np.ascontiguousarray(g.row_ptr)).cuda()
    col = torch.from_numpy(np.ascontiguousarray(g.col) if g.col.size else np.zeros(0, np.int32)).cuda()
    lab = torch.from_numpy(np.ascontiguousarray(g.label)).cuda()
    return cstm.Graph(ctx(), rp, col, lab)


def gpu_count(G, q, budget: int = 0, max_list: int = 0):
    from paper_2102_10768_amd import cstm

    c = cstm.CST(ctx(), G, q.qlabel, q.qedges)
    c.partition(budget, max_list)
    n = c.count()
    info = c.info()
    c.close()
    return n, info


def gpu_rows(G, q, cap: int = 1 << 20, budget: int = 0):
    from paper_2102_10768_amd import cstm

    c = cstm.CST(ctx(), G, q.qlabel, q.qedges)
    if budget:
        c.partition(budget)
    n, rows = c.list(cap)
    r = sorted(tuple(int(x) for x in row) for row in rows.cpu().numpy())
    c.close()
    return n, r
