"""Plain Python restatement of the CST method's own steps.  TEST INFRASTRUCTURE ONLY.

The count oracle (``oracle.c``) fixes *what* is computed; this module restates
*how* the paper computes it, so the CST-level invariants can be checked:

* :func:`build_cst` -- candidate search tree, Section V-A, Definition 2 and
  Algorithm 1 (top-down construction, bottom-up refinement, non-tree candidate
  edges), candidates filtered by label and degree ("local features").
* :func:`path_order` -- the path-based matching order of Section V-B.
* :func:`partition` -- the CST partition of Algorithm 2 (Section V-B).
* :func:`workload` -- the workload estimate c_u(v) / W_CST of Section V-C.
* :func:`share_split` -- Algorithm 3's host/accelerator split of the work
  (Section V-C), over runs of root candidates.
* :func:`fast_round` -- one Generator / Visited Validator / Edge Validator /
  Synchronizer round (Algorithms 5-8, Section VI-A), for the worked example.
* :func:`enumerate_cst` -- all embeddings found by traversing only the CST
  (the soundness theorem of Section V-A).

Where the paper leaves a choice open, the reading taken is stated at the
function that takes it.  Everything works on plain Python sets and lists.
"""

from __future__ import annotations

import dataclasses
import itertools
import math
from fractions import Fraction

import numpy as np


@dataclasses.dataclass
class CST:
    k: int
    qlabel: list
    qdeg: list
    qadj: list  # sorted neighbour lists of q
    root: int
    parent: list  # tree parent per query vertex, -1 at the root
    children: list  # tree children per query vertex, ascending
    bfs: list  # BFS order of t_q
    nontree: list  # non-tree edges (a, b), a < b
    cand: list  # C(u): data vertices, ordered by (degree desc, id asc)
    tree_adj: dict  # (u_p, u) -> {v_p: [v, ...]}  N^{u_p}_u(v_p), v ascending
    nt_adj: dict  # (u, u_n) -> {v: [v_n, ...]}    N^u_{u_n}(v), both directions

    def cand_set(self, u):
        return set(self.cand[u])


def _rank_key(g, v):
    return (-int(g.row_ptr[v + 1] - g.row_ptr[v]), int(v))


def local_candidates(g, label: int, min_degree: int) -> list:
    """C0(u): vertices with the query vertex's label and degree >= its query degree.

    Reading of "local features ... labels and degrees" (Sections IV and V-A):
    the label-and-degree filter.  Ordered by degree descending, then id.
    """
    deg = np.diff(g.row_ptr)
    vs = np.flatnonzero((g.label == label) & (deg >= min_degree))
    return sorted((int(v) for v in vs), key=lambda v: _rank_key(g, v))


def query_structure(k, qlabel, qedges):
    adj = [set() for _ in range(k)]
    for a, b in np.asarray(qedges).reshape(-1, 2):
        adj[int(a)].add(int(b))
        adj[int(b)].add(int(a))
    return [sorted(s) for s in adj]


def choose_root(g, k, qlabel, qadj) -> int:
    """Reading: the root minimises #C0(u) / d_q(u) (smaller id on ties); with k = 1 the only vertex."""
    if k == 1:
        return 0
    best, best_val = 0, None
    for u in range(k):
        c0 = len(local_candidates(g, int(qlabel[u]), len(qadj[u])))
        val = c0 / len(qadj[u])
        if best_val is None or val < best_val:
            best, best_val = u, val
    return best


def bfs_tree(k, qadj, root):
    """BFS spanning tree t_q; neighbours visited in ascending id, parent = first discoverer."""
    parent = [-1] * k
    order = [root]
    seen = {root}
    for u in order:
        for w in qadj[u]:
            if w not in seen:
                seen.add(w)
                parent[w] = u
                order.append(w)
    children = [sorted(c for c in range(k) if parent[c] == u) for u in range(k)]
    tree = {(min(c, parent[c]), max(c, parent[c])) for c in range(k) if parent[c] >= 0}
    nontree = sorted(
        (a, b) for a in range(k) for b in qadj[a] if a < b and (a, b) not in tree
    )
    return parent, children, order, nontree


def build_cst(g, qlabel, qedges, root: int | None = None) -> CST:
    """Algorithm 1: CST construction.

    Readings taken:
    * top-down: C(u) = C0(u) restricted to vertices adjacent to some candidate
      of the tree parent, and N^{u_p}_u(v_p) = N_G(v_p) intersected with C(u);
    * bottom-up (reverse BFS order): first drop from each child list the
      children removed below, then v stays iff every child list is non-empty
      (a parent exists by construction of the top-down pass);
    * the passes run once each, as written; non-tree lists are built last, for
      both directions of every non-tree edge.
    """
    k = len(qlabel)
    qlabel = [int(x) for x in qlabel]
    qadj = query_structure(k, qlabel, qedges)
    qdeg = [len(a) for a in qadj]
    if root is None:
        root = choose_root(g, k, qlabel, qadj)
    parent, children, bfs, nontree = bfs_tree(k, qadj, root)
    order_key = lambda v: _rank_key(g, v)

    cand = [None] * k
    tree_adj = {}
    # top-down construction
    cand[root] = local_candidates(g, qlabel[root], qdeg[root])
    for u in bfs[1:]:
        up = parent[u]
        c0 = set(local_candidates(g, qlabel[u], qdeg[u]))
        lists = {}
        union = set()
        for vp in cand[up]:
            nb = [int(w) for w in g.neighbors(vp) if int(w) in c0]
            lists[vp] = nb
            union.update(nb)
        cand[u] = sorted(union, key=order_key)
        tree_adj[(up, u)] = lists
    # bottom-up refinement
    for u in reversed(bfs):
        keep = []
        for v in cand[u]:
            ok = True
            for uc in children[u]:
                cs = set(cand[uc])
                lst = [w for w in tree_adj[(u, uc)][v] if w in cs]
                tree_adj[(u, uc)][v] = lst
                if not lst:
                    ok = False
            if ok:
                keep.append(v)
        if len(keep) != len(cand[u]):
            gone = set(cand[u]) - set(keep)
            for uc in children[u]:
                for v in gone:
                    tree_adj[(u, uc)].pop(v, None)
        cand[u] = keep
    # after refinement, lists only point at surviving children
    for u in range(k):
        for uc in children[u]:
            cs = set(cand[uc])
            for v in list(tree_adj[(u, uc)].keys()):
                tree_adj[(u, uc)][v] = [w for w in tree_adj[(u, uc)][v] if w in cs]
    # non-tree candidate edges
    nt_adj = {}
    for a, b in nontree:
        for u, un in ((a, b), (b, a)):
            cs = set(cand[un])
            nt_adj[(u, un)] = {v: [int(w) for w in g.neighbors(v) if int(w) in cs] for v in cand[u]}
    return CST(k, qlabel, qdeg, qadj, root, parent, children, bfs, nontree, cand, tree_adj, nt_adj)


def tree_paths(cst: CST) -> list:
    """Root-to-leaf paths of t_q (leaves in ascending id)."""
    out = []
    for leaf in range(cst.k):
        if cst.children[leaf] or (leaf == cst.root and cst.k > 1):
            continue
        p = [leaf]
        while cst.parent[p[-1]] >= 0:
            p.append(cst.parent[p[-1]])
        out.append(p[::-1])
    return out


def path_embeddings(cst: CST, path: list) -> int:
    """Number of candidate paths in the CST along a root-to-leaf path of t_q."""
    cnt = {v: 1 for v in cst.cand[path[-1]]}
    for i in range(len(path) - 2, -1, -1):
        u, uc = path[i], path[i + 1]
        cnt = {v: sum(cnt.get(w, 0) for w in cst.tree_adj[(u, uc)].get(v, [])) for v in cst.cand[u]}
    return sum(cnt.values())


def path_order(cst: CST) -> list:
    """Path-based matching order (Section V-B).

    Reading: root-to-leaf paths of t_q sorted by their number of CST path
    embeddings (ascending, smaller leaf id on ties); the order lists each path's
    not-yet-listed vertices in path order.  Parents always precede children.
    """
    paths = tree_paths(cst)
    if not paths:
        return [cst.root]
    keyed = sorted(paths, key=lambda p: (path_embeddings(cst, p), p[-1]))
    order = []
    for p in keyed:
        for u in p:
            if u not in order:
                order.append(u)
    return order


# ---------------------------------------------------------------- enumeration on the CST

def enumerate_cst(cst: CST, order: list, cand_override=None) -> list:
    """All embeddings reachable in the CST along ``order`` (sorted rows, query-id order).

    Each next vertex takes its candidates from its tree parent's list, checks
    that the data vertex is unused (visited validation) and that it is joined in
    the CST to every already-mapped non-tree neighbour (edge validation).
    ``cand_override`` restricts candidate sets (a partition).
    """
    k = cst.k
    cand = [set(c) for c in (cand_override or cst.cand)]
    pos = {u: i for i, u in enumerate(order)}
    out = []
    f = {}

    def rec(i):
        if i == k:
            out.append(tuple(f[u] for u in range(k)))
            return
        u = order[i]
        if i == 0:
            pool = [v for v in cst.cand[u] if v in cand[u]]
        else:
            pool = [v for v in cst.tree_adj[(cst.parent[u], u)].get(f[cst.parent[u]], []) if v in cand[u]]
        for v in pool:
            if v in f.values():
                continue
            ok = True
            for un in cst.qadj[u]:
                if un == cst.parent[u] or cst.parent[un] == u or pos[un] > i:
                    continue
                if f[un] not in cst.nt_adj[(u, un)].get(v, []):
                    ok = False
                    break
            if not ok:
                continue
            f[u] = v
            rec(i + 1)
            del f[u]

    rec(0)
    out.sort()
    return out


# ---------------------------------------------------------------- workload estimate

def workload(cst: CST, cand_override=None):
    """c_u(v) = prod over tree children u' of sum_{v' in N^u_{u'}(v)} c_{u'}(v'); W_CST = sum over root candidates.

    Section V-C.  Leaves have c = 1.  Exact Python integers.  Returns (c, W) with c[u][v].
    """
    cand = [set(c) for c in (cand_override or cst.cand)]
    c = [dict() for _ in range(cst.k)]
    for u in reversed(cst.bfs):
        for v in cst.cand[u]:
            if v not in cand[u]:
                continue
            val = 1
            for uc in cst.children[u]:
                val *= sum(c[uc].get(w, 0) for w in cst.tree_adj[(u, uc)].get(v, []) if w in cand[uc])
            c[u][v] = val
    W = sum(c[cst.root].values())
    return c, W


U64_MAX = (1 << 64) - 1


def saturate_u64(x: int) -> int:
    """min(x, 2^64 - 1): a value held in an unsigned 64-bit integer that saturates."""
    return min(int(x), U64_MAX)


def share_split(weights, delta: float, n_runs: int):
    """Algorithm 3 (Section V-C): the host takes a unit of work only while its
    share of the workload handed out so far, that unit included, stays below
    delta; every other unit goes to the accelerator.

    Reading: the units are runs of consecutive root candidates (the first
    split of Algorithm 2); run i of R covers root indices [i*n//R, (i+1)*n//R)
    and weighs w_i, the sum of c_root over them (``weights`` in root-candidate
    order).  With S_i = w_0 + ... + w_i (all work handed out once run i is)
    and H the host's part of S_{i-1}, run i goes to the host exactly when
    H + w_i < delta * S_i.  Integers are exact and delta is taken as the exact
    rational value of the float.

    Returns (host_runs, device_runs, W_C, W_F), runs as (lo, hi) pairs.
    """
    n = len(weights)
    R = min(n, n_runs if n_runs > 0 else 1024)
    runs = [(i * n // R, (i + 1) * n // R) for i in range(R)]
    w = [sum(int(x) for x in weights[lo:hi]) for lo, hi in runs]
    d = Fraction(delta)
    to_host = []
    H = 0
    for wi, Si in zip(w, itertools.accumulate(w)):
        to_host.append(H + wi < d * Si)
        H += wi if to_host[-1] else 0
    host = [r for r, t in zip(runs, to_host) if t]
    dev = [r for r, t in zip(runs, to_host) if not t]
    return host, dev, H, sum(w) - H


# ---------------------------------------------------------------- partition (Algorithm 2)

def restricted_sets(cst: CST, order: list, ranges: dict) -> list:
    """Candidate sets of a partition, top-down along ``order``.

    ``ranges[i] = (lo, hi)`` keeps only the candidates of ``order[i]`` whose
    index in the full C(order[i]) lies in [lo, hi).  Every later vertex keeps the
    candidates its (restricted) tree parent reaches: "can reach at least one
    candidate of the split set" read along the tree path; vertices not below a
    split keep what their parents reach, a sound superset.
    """
    sets = [None] * cst.k
    for i, u in enumerate(order):
        if i == 0:
            pool = list(cst.cand[u])
        else:
            up = cst.parent[u]
            reach = set()
            for vp in sets[up]:
                reach.update(cst.tree_adj[(up, u)].get(vp, []))
            pool = [v for v in cst.cand[u] if v in reach]
        if i in ranges:
            lo, hi = ranges[i]
            idx = {v: j for j, v in enumerate(cst.cand[u])}
            pool = [v for v in pool if lo <= idx[v] < hi]
        sets[u] = pool
    return sets


def image_bytes(cst: CST, order: list, sets: list) -> int:
    """size(CST) of a partition: bytes of its on-chip image.

    Reading of |CST| (Table I): 4 B per candidate (data vertex id); per tree edge
    4 B per parent candidate plus 4 B (list offsets) and 2 B per list entry,
    padded to 4 B; per non-tree edge a bit row of ceil(#C(b)/32) 4-byte words
    for each candidate of the endpoint a that comes first in the order; plus a
    fixed header; the total rounded up to 16 B.
    """
    pos = {u: i for i, u in enumerate(order)}
    k = cst.k
    total = image_header_bytes(k, len(cst.nontree))
    ss = [set(s) for s in sets]
    for u in range(k):
        total += 4 * len(sets[u])
    for u in range(k):
        if cst.parent[u] < 0:
            continue
        up = cst.parent[u]
        total += 4 * (len(sets[up]) + 1)
        entries = sum(len([w for w in cst.tree_adj[(up, u)].get(vp, []) if w in ss[u]]) for vp in sets[up])
        total += 4 * ((entries + 1) // 2)
    for a, b in cst.nontree:
        first, second = (a, b) if pos[a] < pos[b] else (b, a)
        total += 4 * len(sets[first]) * ((len(sets[second]) + 31) // 32)
    return _align(total, 16)


def _align(x, a):
    return (x + a - 1) // a * a


def image_header_bytes(k: int, n_nontree: int) -> int:
    """Fixed part of the on-chip image: per position 8 words, per non-tree edge 4 words."""
    return _align(64 + 32 * k + 16 * n_nontree, 16)


def max_list_len(cst: CST, sets: list) -> int:
    """D_CST: the longest tree or non-tree list inside the partition."""
    ss = [set(s) for s in sets]
    d = 0
    for (up, u), lists in cst.tree_adj.items():
        for vp in sets[up]:
            d = max(d, len([w for w in lists.get(vp, []) if w in ss[u]]))
    for (u, un), lists in cst.nt_adj.items():
        for v in sets[u]:
            d = max(d, len([w for w in lists.get(v, []) if w in ss[un]]))
    return d


def partition(cst: CST, order: list, delta_s: int, delta_d: int = 1 << 30, force_k: int | None = None):
    """Algorithm 2.  Returns a list of (ranges, sets) for partitions that fit.

    Readings: the factor is ceil(max(size/delta_S, D/delta_D)), at least 2 and
    at most #C(u); parts are contiguous runs of the current candidate list of
    u, in candidate order, with sizes differing by at most one (the first ones
    larger); a part whose candidate set for u has one vertex moves the split to
    the next vertex of the order; a part with an empty candidate set anywhere
    holds no embedding and is dropped.  ``force_k`` fixes the factor (the worked
    example uses k = 2).
    """
    out = []
    full = restricted_sets(cst, order, {})
    if any(len(s) == 0 for s in full):
        return out
    if image_bytes(cst, order, full) <= delta_s and max_list_len(cst, full) <= delta_d:
        return [({}, full)]

    def split_ranges(u_idx, ranges, sets):
        u = order[u_idx]
        idx = {v: j for j, v in enumerate(cst.cand[u])}
        members = [idx[v] for v in sets[u]]
        size = image_bytes(cst, order, sets)
        dmax = max_list_len(cst, sets)
        kp = force_k or max(2, math.ceil(max(size / delta_s, dmax / delta_d)))
        kp = min(kp, len(members))
        base, extra = divmod(len(members), kp)
        start = 0
        for i in range(kp):
            cnt = base + (1 if i < extra else 0)
            chunk = members[start : start + cnt]
            start += cnt
            r = dict(ranges)
            r[u_idx] = (chunk[0], chunk[-1] + 1)
            yield r

    def rec(u_idx, ranges, sets):
        while u_idx < cst.k and len(sets[order[u_idx]]) <= 1:
            u_idx += 1
        if u_idx == cst.k:
            # one candidate per vertex: nothing is left to split
            out.append((ranges, sets))
            return
        for r in split_ranges(u_idx, ranges, sets):
            s = restricted_sets(cst, order, r)
            if any(len(x) == 0 for x in s):
                continue
            if image_bytes(cst, order, s) <= delta_s and max_list_len(cst, s) <= delta_d:
                out.append((r, s))
            else:
                # a part left with one candidate moves on to the next vertex (top of rec)
                rec(u_idx, r, s)

    rec(0, {}, full)
    return out


# ---------------------------------------------------------------- one FAST round (Algorithms 5-8)

def fast_round(cst: CST, order: list, P: list, N_o: int, cand_override=None):
    """One Generator -> validators -> Synchronizer round on the partial results ``P``.

    Section VI-A restated from what each stage computes.  ``P`` holds partial
    results as tuples of data vertices in ``order`` positions, all of length n;
    u = order[n] is the vertex the round maps, u_p its tree parent.

    * The extensions of a partial result p are the candidates of u in the CST
      list of p's u_p candidate (within the candidate sets in force).
    * The round takes the longest prefix of P whose extensions together number
      at most N_o (the Generator's output budget; reading of its cut: a partial
      result whose extensions do not all fit stays in P for the next round).
      P_o is those extensions in order; T_v pairs each new vertex with the
      index (within the prefix) of the partial result it extends.
    * The backward non-tree neighbours of u are its query neighbours other
      than u_p and its tree children that are already mapped; T_n holds, for
      each of them in ascending id and then for each p_o, the triple
      (M(u), M(u_n), index of p_o).
    * B_v(p_o) = 1 iff the new vertex is not among p_o's earlier vertices;
      B_n(p_o) = 1 iff the CST joins the new vertex to the mapping of every
      backward non-tree neighbour.  The survivors are the p_o with both bits.

    Returns (P_o, T_v, T_n, B_v, B_n, survivors, rest), ``rest`` = P minus the
    prefix taken.
    """
    cand = [set(c) for c in (cand_override or cst.cand)]
    n = len(P[0])
    u = order[n]
    up = cst.parent[u]
    pos = {w: i for i, w in enumerate(order)}

    def extensions(p):
        return [v for v in cst.tree_adj[(up, u)].get(p[pos[up]], []) if v in cand[u]]

    ext = [extensions(p) for p in P]
    fits = [total <= N_o for total in itertools.accumulate(len(e) for e in ext)]
    taken = fits.index(False) if False in fits else len(P)
    P_o = [P[i] + (v,) for i in range(taken) for v in ext[i]]
    T_v = [(v, i) for i in range(taken) for v in ext[i]]
    back_nt = [un for un in cst.qadj[u] if un != up and cst.parent[un] != u and pos[un] < n]
    T_n = [(p_o[n], p_o[pos[un]], j) for un in back_nt for j, p_o in enumerate(P_o)]
    B_v = [int(p_o[n] not in p_o[:n]) for p_o in P_o]
    B_n = [int(all(p_o[pos[un]] in cst.nt_adj[(u, un)].get(p_o[n], []) for un in back_nt)) for p_o in P_o]
    survivors = [p for p, bv, bn in zip(P_o, B_v, B_n) if bv and bn]
    return P_o, T_v, T_n, B_v, B_n, survivors, list(P[taken:])
