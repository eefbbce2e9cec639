"""Brute force over all injective maps: the plain definition of an embedding, for tiny inputs.

Definition 1 (Section II-A): f: V(q) -> V(G) is an embedding iff it is injective,
keeps every label and maps every query edge onto an edge of G.  This module
tries every injective map (``itertools.permutations``), so it is only usable for
n <= 9 and k <= 5 (at most 15,120 maps).
"""

from __future__ import annotations

import itertools

import numpy as np


def edge_set(g) -> frozenset:
    out = set()
    for v in range(g.n):
        for w in g.col[g.row_ptr[v] : g.row_ptr[v + 1]]:
            out.add((int(v), int(w)))
    return frozenset(out)


def embeddings(g, q) -> list[tuple[int, ...]]:
    """Sorted list of all embeddings, each a tuple (f(0), ..., f(k-1))."""
    E = edge_set(g)
    lab = [int(x) for x in g.label]
    ql = [int(x) for x in q.qlabel]
    qe = [(int(a), int(b)) for a, b in np.asarray(q.qedges).reshape(-1, 2)]
    k = len(ql)
    out = []
    for f in itertools.permutations(range(g.n), k):
        if any(lab[f[u]] != ql[u] for u in range(k)):
            continue
        if any((f[a], f[b]) not in E for a, b in qe):
            continue
        out.append(tuple(f))
    out.sort()
    return out


def count(g, q) -> int:
    return len(embeddings(g, q))
