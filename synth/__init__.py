"""Seeded synthetic inputs for subgraph matching: data graphs, vertex labels and queries.

This package holds input generation only. It contains none of the matching
method's arithmetic (no candidate filtering, no search, no counting), so both
the CPU oracle and the HIP path may take their inputs from it.

Every generator draws from ``numpy.random.Generator(PCG64(seed))`` and returns
plain numpy arrays:

* a data graph is ``(row_ptr int64[n+1], col int32[2m], label int32[n])``:
  undirected, simple (no self-loops, no duplicate edges), each row sorted
  ascending, every edge stored in both directions;
* a query is ``(qlabel int32[k], qedges int32[m_q, 2])`` with ``a < b`` per edge.
"""

from .graphs import (
    Graph,
    csr_from_edges,
    erdos_renyi,
    chung_lu,
    rmat,
    uniform_labels,
    zipf_labels,
    make_graph,
)
from .queries import Query, random_walk_query, query_set, induced_edges

__all__ = [
    "Graph",
    "csr_from_edges",
    "erdos_renyi",
    "chung_lu",
    "rmat",
    "uniform_labels",
    "zipf_labels",
    "make_graph",
    "Query",
    "random_walk_query",
    "query_set",
    "induced_edges",
]
