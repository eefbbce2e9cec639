"""Shared helpers for the GPU tests: one device context per test session."""

from __future__ import annotations

import numpy as np
import pytest

_CTX = {}

MODES = ("auto", "lds", "hbm")
MODE_IDS = {"auto": 0, "lds": 1, "hbm": 2}


def ctx(mode: str = "auto"):
    if mode not in _CTX:
        import torch

        if not torch.cuda.is_available():
            pytest.fail("GPU test collected on a machine without a GPU")
        from paper_2102_10768_amd import cstm

        _CTX[mode] = cstm.Context(0, tune={"enum_mode": MODE_IDS[mode], "collect_stats": 1})
    return _CTX[mode]


def gpu_graph(g, mode: str = "auto"):
    """Load a synth.Graph through the device-pointer path (torch tensors)."""
    return gpu_graph_in(ctx(mode), g)


def gpu_graph_in(context, g):
    """Load a synth.Graph into the given context (torch tensors, borrowed)."""
    import torch
    from paper_2102_10768_amd import cstm

    rp = torch.from_numpy(np.ascontiguousarray(g.row_ptr)).cuda()
    col = torch.from_numpy(np.ascontiguousarray(g.col) if g.col.size else np.zeros(0, np.int32)).cuda()
    lab = torch.from_numpy(np.ascontiguousarray(g.label)).cuda()
    return cstm.Graph(context, rp, col, lab)


def gpu_count(G, q, budget: int = 0, max_list: int = 0, partition: bool = True):
    from paper_2102_10768_amd import cstm

    c = cstm.CST(G.ctx, G, q.qlabel, q.qedges)
    if partition:
        c.partition(budget, max_list)
    n = c.count()
    info = c.info()
    c.close()
    return n, info


def gpu_rows(G, q, cap: int = 1 << 20, budget: int = 0):
    from paper_2102_10768_amd import cstm

    c = cstm.CST(G.ctx, G, q.qlabel, q.qedges)
    if budget:
        c.partition(budget)
    n, rows = c.list(cap)
    r = sorted(tuple(int(x) for x in row) for row in rows.cpu().numpy())
    c.close()
    return n, r
