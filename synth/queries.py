"""Seeded query generation: connected queries extracted from a data graph by random walk.

A random-walk query of size k starts at a uniformly random vertex of degree at
least one and steps to uniformly random neighbours until k distinct vertices
were seen (restarting from a fresh start vertex after 100*k steps).  The query
is the subgraph of G induced on those vertices, with labels inherited and query
ids assigned in first-visit order; the visited tuple is recorded as ``source``
(one embedding the query is guaranteed to have).
"""

from __future__ import annotations

import dataclasses

import numpy as np

from .graphs import Graph, _rng

STREAM_QUERIES = 3


@dataclasses.dataclass
class Query:
    qlabel: np.ndarray  # int32[k]
    qedges: np.ndarray  # int32[m_q, 2], a < b
    source: np.ndarray | None = None  # int32[k]: data vertex of each query vertex
    qid: int = -1

    @property
    def k(self) -> int:
        return int(self.qlabel.shape[0])

    @property
    def m_q(self) -> int:
        return int(self.qedges.shape[0])

    @property
    def avg_degree(self) -> float:
        return 2.0 * self.m_q / self.k if self.k else 0.0

    def to_dict(self) -> dict:
        d = {"qlabel": self.qlabel.tolist(), "qedges": self.qedges.tolist()}
        if self.source is not None:
            d["source"] = self.source.tolist()
        if self.qid >= 0:
            d["qid"] = self.qid
        return d

    @staticmethod
    def from_dict(d: dict) -> "Query":
        qe = np.asarray(d["qedges"], dtype=np.int32).reshape(-1, 2)
        src = d.get("source")
        return Query(
            qlabel=np.asarray(d["qlabel"], dtype=np.int32),
            qedges=qe,
            source=None if src is None else np.asarray(src, dtype=np.int32),
            qid=int(d.get("qid", -1)),
        )


def induced_edges(g: Graph, verts: np.ndarray) -> np.ndarray:
    """All edges of G among ``verts``, as pairs of positions (i < j) into ``verts``."""
    out = []
    k = len(verts)
    for i in range(k):
        row = g.neighbors(int(verts[i]))
        for j in range(i + 1, k):
            t = int(verts[j])
            p = np.searchsorted(row, t)
            if p < row.shape[0] and row[p] == t:
                out.append((i, j))
    return np.asarray(out, dtype=np.int32).reshape(-1, 2)


def random_walk_query(g: Graph, k: int, rng: np.random.Generator, start_by_degree: bool = False) -> Query:
    deg = g.degree
    nz = np.flatnonzero(deg > 0)
    if nz.shape[0] == 0:
        raise ValueError("graph has no edges")
    if start_by_degree:
        cdf = np.cumsum(deg[nz].astype(np.float64))
        cdf /= cdf[-1]
    while True:
        if start_by_degree:
            v = int(nz[min(int(np.searchsorted(cdf, rng.random(), side="right")), nz.shape[0] - 1)])
        else:
            v = int(nz[rng.integers(0, nz.shape[0])])
        seen = [v]
        seen_set = {v}
        steps = 0
        while len(seen) < k and steps < 100 * k:
            row = g.neighbors(v)
            v = int(row[rng.integers(0, row.shape[0])])
            if v not in seen_set:
                seen_set.add(v)
                seen.append(v)
            steps += 1
        if len(seen) == k:
            verts = np.asarray(seen, dtype=np.int32)
            return Query(qlabel=g.label[verts].astype(np.int32), qedges=induced_edges(g, verts), source=verts)


def query_set(g: Graph, sizes, seed: int, start_by_degree: bool = False) -> list[Query]:
    """One random-walk query per entry of ``sizes``, from a single seeded stream."""
    rng = _rng(seed, STREAM_QUERIES)
    out = []
    for i, k in enumerate(sizes):
        q = random_walk_query(g, int(k), rng, start_by_degree=start_by_degree)
        q.qid = i
        out.append(q)
    return out
