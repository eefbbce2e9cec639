"""Independent pins for embedding counts: small named graphs, closed forms and sparse-matrix identities.

Nothing here enumerates.  Each function states a count that mathematics fixes
without a search, so the CPU oracle (and through it the GPU path) can be checked
against something other than itself.
"""

from __future__ import annotations

import math

import numpy as np
import scipy.sparse as sp

from synth import Graph, Query, csr_from_edges


def graph_from_edges(n: int, edges, labels=None, name: str = "") -> Graph:
    e = np.asarray(list(edges), dtype=np.int64).reshape(-1, 2)
    row_ptr, col = csr_from_edges(n, e[:, 0], e[:, 1])
    lab = np.zeros(n, dtype=np.int32) if labels is None else np.asarray(labels, dtype=np.int32)
    return Graph(n=n, row_ptr=row_ptr, col=col, label=lab, name=name)


def complete(n: int, labels=None) -> Graph:
    return graph_from_edges(n, [(i, j) for i in range(n) for j in range(i + 1, n)], labels, f"K{n}")


def complete_bipartite(a: int, b: int) -> Graph:
    return graph_from_edges(a + b, [(i, a + j) for i in range(a) for j in range(b)], None, f"K{a},{b}")


def cycle(n: int) -> Graph:
    return graph_from_edges(n, [(i, (i + 1) % n) for i in range(n)], None, f"C{n}")


def path(n: int) -> Graph:
    return graph_from_edges(n, [(i, i + 1) for i in range(n - 1)], None, f"P{n}")


def query(labels, edges) -> Query:
    return Query(qlabel=np.asarray(labels, dtype=np.int32), qedges=np.asarray(list(edges), dtype=np.int32).reshape(-1, 2))


def path_query(k: int, label: int = 0) -> Query:
    return query([label] * k, [(i, i + 1) for i in range(k - 1)])


def cycle_query(k: int, label: int = 0) -> Query:
    return query([label] * k, [(i, (i + 1) % k) for i in range(k)])


def star_query(s: int, label: int = 0) -> Query:
    return query([label] * (s + 1), [(0, i) for i in range(1, s + 1)])


def clique_query(labels) -> Query:
    k = len(labels)
    return query(labels, [(i, j) for i in range(k) for j in range(i + 1, k)])


def falling(x: int, r: int) -> int:
    out = 1
    for i in range(r):
        out *= x - i
    return out


# ---- closed forms -------------------------------------------------------

def clique_host_count(n: int, k: int) -> int:
    """Any connected k-vertex single-label query in K_n: every injective map works."""
    return math.perm(n, k)


def labelled_clique_host_count(host_label_counts: dict, query_label_counts: dict) -> int:
    """Clique query with m_i vertices of label i in a complete graph with c_i vertices of label i."""
    out = 1
    for lab, m in query_label_counts.items():
        out *= falling(host_label_counts.get(lab, 0), m)
    return out


def edge_count(g: Graph) -> int:
    """Edge query: each undirected edge gives two maps."""
    return int(g.col.shape[0])


def wedge_count(g: Graph) -> int:
    """Path with 3 vertices: ordered pairs of distinct neighbours around each middle vertex."""
    d = np.diff(g.row_ptr).astype(object)
    return int(sum(x * (x - 1) for x in d))


def star_count(g: Graph, s: int) -> int:
    """Star K_{1,s}: centre to v, leaves to an ordered s-tuple of distinct neighbours."""
    d = np.diff(g.row_ptr)
    return int(sum(falling(int(x), s) for x in d))


def c4_in_complete_bipartite(a: int, b: int) -> int:
    """4-cycle in K_{a,b}: choose the side of query vertex 0, then ordered distinct pairs on each side."""
    return 2 * a * (a - 1) * b * (b - 1)


def path_in_cycle(n: int, k: int) -> int:
    """P_k in C_n (2 <= k <= n, n >= 3): a start vertex and a direction."""
    return 2 * n


def path_in_path(n: int, k: int) -> int:
    """P_k in P_n (2 <= k <= n): a start position and a direction."""
    return 2 * (n - k + 1)


# ---- sparse-matrix identities ------------------------------------------

def adjacency(g: Graph, dtype=np.int64) -> sp.csr_matrix:
    return sp.csr_matrix((np.ones(g.col.shape[0], dtype=dtype), g.col, g.row_ptr), shape=(g.n, g.n))


def triangle_count_single_label(g: Graph, label: int) -> int:
    """Triangle query with all three vertices labelled ``label``: trace((P A)^3)."""
    A = adjacency(g)
    p = (g.label == label).astype(np.int64)
    P = sp.diags(p)
    M = P @ A
    return int((M @ M @ M).diagonal().sum())


def triangle_count_labels(g: Graph, la: int, lb: int, lc: int) -> int:
    """Triangle query labelled (la, lb, lc): trace(P_a A P_b A P_c A)."""
    A = adjacency(g)
    Ps = [sp.diags((g.label == x).astype(np.int64)) for x in (la, lb, lc)]
    M = Ps[0] @ A @ Ps[1] @ A @ Ps[2] @ A
    return int(M.diagonal().sum())


def tree_homomorphism_count(g: Graph, q: Query, degree_filter: bool = False, exact: bool = True):
    """Number of label-preserving homomorphisms of a spanning tree of q into G.

    f_u(v) = [l(v) = l_q(u)] * prod_{children c} sum_{w in N(v)} f_c(w); the total
    is sum_v f_root(v).  For a tree query whose labels are pairwise distinct, a
    homomorphism is automatically injective, so this equals the embedding
    count.  For any query it is an upper bound on the embedding count.
    ``exact`` returns an int computed with int64 sparse products (checked first in
    float64 to fit); otherwise a float64 estimate.
    """
    k = q.k
    adj = [[] for _ in range(k)]
    for a, b in np.asarray(q.qedges).reshape(-1, 2):
        adj[int(a)].append(int(b))
        adj[int(b)].append(int(a))
    parent = [-1] * k
    order = [0]
    seen = {0}
    for u in order:
        for w in sorted(adj[u]):
            if w not in seen:
                seen.add(w)
                parent[w] = u
                order.append(w)
    if len(order) != k:
        raise ValueError("query is disconnected")
    deg = np.diff(g.row_ptr)

    def run(dtype):
        A = adjacency(g, dtype=dtype)
        f = [None] * k
        peak = 0
        for u in reversed(order):
            mask = g.label == q.qlabel[u]
            if degree_filter:
                mask &= deg >= len(adj[u])
            x = mask.astype(dtype)
            for c in range(k):
                if parent[c] == u:
                    s = A @ f[c]
                    x = x * s
                    if x.shape[0]:
                        peak = max(peak, float(s.max()), float(x.max()))
            f[u] = x
        return f[0].sum(), peak

    total, peak = run(np.float64)
    if not exact:
        return float(total)
    # int64 sparse products are exact when no intermediate value can overflow
    if peak < 2.0**62 and total < 2.0**62:
        t, _ = run(np.int64)
        return int(t)
    raise OverflowError("tree homomorphism count does not fit in int64")


def automorphism_count(q: Query) -> int:
    """#Aut(q) by brute force over vertex permutations of q (label-preserving)."""
    import itertools

    k = q.k
    E = set()
    for a, b in np.asarray(q.qedges).reshape(-1, 2):
        E.add((int(a), int(b)))
        E.add((int(b), int(a)))
    lab = [int(x) for x in q.qlabel]
    cnt = 0
    for p in itertools.permutations(range(k)):
        if any(lab[p[u]] != lab[u] for u in range(k)):
            continue
        if all((p[a], p[b]) in E for a, b in E):
            cnt += 1
    return cnt


def query_as_graph(q: Query) -> Graph:
    return graph_from_edges(q.k, [tuple(e) for e in np.asarray(q.qedges).reshape(-1, 2)], q.qlabel, "q")


def disjoint_union(g1: Graph, g2: Graph) -> Graph:
    e1 = [(v, int(w)) for v in range(g1.n) for w in g1.neighbors(v) if v < w]
    e2 = [(g1.n + v, g1.n + int(w)) for v in range(g2.n) for w in g2.neighbors(v) if v < w]
    return graph_from_edges(g1.n + g2.n, e1 + e2, np.concatenate([g1.label, g2.label]), "union")


def permute_graph(g: Graph, perm: np.ndarray) -> Graph:
    """Vertex v becomes perm[v]."""
    e = [(int(perm[v]), int(perm[w])) for v in range(g.n) for w in g.neighbors(v) if v < w]
    lab = np.zeros(g.n, dtype=np.int32)
    lab[perm] = g.label
    return graph_from_edges(g.n, e, lab, "perm")


def relabel_query(q: Query, perm) -> Query:
    """Query vertex u becomes perm[u]."""
    perm = np.asarray(perm)
    lab = np.zeros(q.k, dtype=np.int32)
    lab[perm] = q.qlabel
    e = [(int(min(perm[a], perm[b])), int(max(perm[a], perm[b]))) for a, b in np.asarray(q.qedges).reshape(-1, 2)]
    return query(lab, e)


class LabelBlocks:
    """Adjacency of G cut into label-by-label blocks, for fast labelled tree DPs.

    Block (a, b) holds the edges from label-a vertices to label-b vertices, so a
    product that only needs label-b values on label-a rows touches only those
    edges.
    """

    def __init__(self, g: Graph, dtype=np.float64):
        self.g = g
        L = int(g.label.max()) + 1 if g.n else 0
        self.L = L
        self.members = [np.flatnonzero(g.label == l) for l in range(L)]
        self.index = np.zeros(g.n, dtype=np.int64)
        for l in range(L):
            self.index[self.members[l]] = np.arange(self.members[l].shape[0])
        self.dtype = dtype
        A = adjacency(g, dtype=dtype).tocsr()
        self.rows = [A[self.members[l], :] for l in range(L)]
        self.blocks = {}
        self.deg = np.diff(g.row_ptr)

    def block(self, a: int, b: int):
        key = (a, b)
        if key not in self.blocks:
            self.blocks[key] = self.rows[a][:, self.members[b]].tocsr()
        return self.blocks[key]

    def tree_bound(self, q: Query, degree_filter: bool = True) -> float:
        """Labelled spanning-tree homomorphism count (float64): an upper bound on the embedding count."""
        k = q.k
        adj = [[] for _ in range(k)]
        for a, b in np.asarray(q.qedges).reshape(-1, 2):
            adj[int(a)].append(int(b))
            adj[int(b)].append(int(a))
        parent = [-1] * k
        order = [0]
        seen = {0}
        for u in order:
            for w in sorted(adj[u]):
                if w not in seen:
                    seen.add(w)
                    parent[w] = u
                    order.append(w)
        f = [None] * k
        for u in reversed(order):
            lu = int(q.qlabel[u])
            if lu >= self.L:
                return 0.0
            x = np.ones(self.members[lu].shape[0], dtype=self.dtype)
            if degree_filter:
                x *= (self.deg[self.members[lu]] >= len(adj[u])).astype(self.dtype)
            for c in range(k):
                if parent[c] == u:
                    x = x * (self.block(lu, int(q.qlabel[c])) @ f[c])
            f[u] = x
        if self.dtype == np.int64:
            return int(f[0].sum())
        return float(f[0].sum())


def is_tree_with_distinct_labels(q: Query) -> bool:
    return q.m_q == q.k - 1 and len(set(int(x) for x in q.qlabel)) == q.k


class ExactTreeCounter(LabelBlocks):
    """Exact embedding counts of tree queries with pairwise-distinct labels, at any graph size.

    For such a query an injective map is automatic, so the embeddings are the
    label-preserving homomorphisms of the tree: the DP of
    :func:`tree_homomorphism_count`, run on label blocks in int64 (checked to fit).
    """

    def __init__(self, g: Graph):
        super().__init__(g, dtype=np.int64)
        self.frows = [r.astype(np.float64) for r in self.rows]
        self.fblocks = {}

    def count(self, q: Query) -> int:
        if not is_tree_with_distinct_labels(q):
            raise ValueError("not a tree with pairwise-distinct labels")
        # a float64 pass first proves every intermediate fits in int64
        fl = LabelBlocks.__new__(LabelBlocks)
        fl.__dict__.update(self.__dict__)
        fl.dtype = np.float64
        fl.blocks = self.fblocks
        fl.rows = self.frows
        if fl.tree_bound(q, degree_filter=False) >= 2.0**60:
            raise OverflowError("count does not fit in int64")
        return int(self.tree_bound(q, degree_filter=False))
