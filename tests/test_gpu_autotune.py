"""The autotuner on the device: it leaves counts unchanged and applies its choice."""

from __future__ import annotations

import json
import os

import pytest

from synth import Query, make_graph

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def test_autotune_choice_keeps_counts():
    from paper_2102_10768_amd import autotune, cstm

    W = json.load(open(os.path.join(GOLDEN, "c1.json")))
    g = make_graph(W["workload"]["graph"])
    import numpy as np
    import torch

    G_ctx = cstm.Context(0, tune={"collect_stats": 0})
    G = cstm.Graph(G_ctx, torch.from_numpy(np.ascontiguousarray(g.row_ptr)).cuda(),
                   torch.from_numpy(np.ascontiguousarray(g.col)).cuda(),
                   torch.from_numpy(np.ascontiguousarray(g.label)).cuda())
    qs = [Query.from_dict(d) for d in W["queries"]]
    rec = autotune.tune(G_ctx, G, qs, frac=0.5, repeats=1)
    assert rec["choice"]["enum_mode"] in (cstm.MODE_HBM, cstm.MODE_LDS)
    assert not [t for t in rec["trials"] if "error" in t and "differ" in t["error"]]
    tuned = G_ctx.tune
    for k, v in rec["choice"].items():
        if k != "part_budget_bytes":
            assert tuned[k] == v
    csts = [cstm.CST(G_ctx, G, q.qlabel, q.qedges) for q in qs]
    assert cstm.batch_count(G_ctx, csts) == [d["count"] for d in W["queries"]]
    for x in csts:
        x.close()
    G_ctx.close()
