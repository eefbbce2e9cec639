"""Seeded data-graph generators: Erdos-Renyi, Chung-Lu power law, R-MAT; iid labels.

All graphs are returned as CSR with int64 ``row_ptr`` and int32 ``col``.
Edges are undirected and simple: self-loops are dropped, duplicates merged and
each edge stored in both directions, rows sorted ascending.  Vertex labels are
int32, drawn iid and independent of degree.
"""

from __future__ import annotations

import dataclasses

import numpy as np


def _rng(seed: int, stream: int) -> np.random.Generator:
    """One independent PCG64 stream per (seed, purpose) pair."""
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence([int(seed), int(stream)])))


STREAM_EDGES = 0
STREAM_LABELS = 1
STREAM_PERM = 2


@dataclasses.dataclass
class Graph:
    n: int
    row_ptr: np.ndarray  # int64[n+1]
    col: np.ndarray  # int32[2m]
    label: np.ndarray  # int32[n]
    name: str = ""
    params: dict = dataclasses.field(default_factory=dict)

    @property
    def m(self) -> int:
        return int(self.col.shape[0] // 2)

    @property
    def degree(self) -> np.ndarray:
        return np.diff(self.row_ptr)

    @property
    def num_labels(self) -> int:
        return int(self.label.max()) + 1 if self.n else 0

    def neighbors(self, v: int) -> np.ndarray:
        return self.col[self.row_ptr[v] : self.row_ptr[v + 1]]

    def has_edge(self, a: int, b: int) -> bool:
        row = self.neighbors(a)
        i = np.searchsorted(row, b)
        return bool(i < row.shape[0] and row[i] == b)

    def summary(self) -> dict:
        d = self.degree
        return {
            "name": self.name,
            "n": int(self.n),
            "m": self.m,
            "max_degree": int(d.max()) if self.n else 0,
            "avg_degree": float(d.mean()) if self.n else 0.0,
            "labels": self.num_labels,
            **self.params,
        }


def _sorted_unique(keys: np.ndarray, bound: int, log=None) -> np.ndarray:
    """np.unique(keys) for non-negative keys below ``bound``; very large arrays
    are split into 64 ranges of the key space, each sorted on its own, so the
    work reports progress and needs less temporary memory (same result)."""
    if keys.shape[0] < (1 << 27):
        return np.unique(keys)
    shift = max(0, int(bound - 1).bit_length() - 6)
    parts = []
    for b in range(64):
        part = np.unique(keys[(keys >> shift) == b])
        parts.append(part)
        if log and b % 8 == 7:
            log(f"sorted {b + 1}/64 key ranges")
    return np.concatenate(parts)



def csr_from_edges(n: int, a: np.ndarray, b: np.ndarray, log=None) -> tuple[np.ndarray, np.ndarray]:
    """Simple undirected CSR from an endpoint list (loops dropped, duplicates merged)."""
    a = np.asarray(a, dtype=np.int64)
    b = np.asarray(b, dtype=np.int64)
    keep = a != b
    a, b = a[keep], b[keep]
    lo = np.minimum(a, b)
    hi = np.maximum(a, b)
    key = _sorted_unique(lo * n + hi, n * n, log)
    if log:
        log(f"csr: {key.shape[0]} distinct edges")
    lo = key // n
    hi = key % n
    del key
    src = np.concatenate([lo, hi])
    dst = np.concatenate([hi, lo])
    del lo, hi
    key2 = src * n + dst
    del src, dst
    key2 = _sorted_unique(key2, n * n, log)  # all distinct: a plain sort
    if log:
        log("csr: adjacency sorted")
    src = key2 // n
    col = (key2 % n).astype(np.int32)
    del key2
    counts = np.bincount(src, minlength=n)
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(counts, out=row_ptr[1:])
    return row_ptr, col


def erdos_renyi(n: int, p: float, seed: int):
    """G(n, p): every unordered pair is an edge independently with probability p.

    Pairs are visited in row-major upper-triangle order and the gaps between
    successive edges are geometric(p), which samples G(n, p) exactly.
    """
    rng = _rng(seed, STREAM_EDGES)
    total = n * (n - 1) // 2
    if total == 0 or p <= 0:
        return np.zeros(n + 1, dtype=np.int64), np.zeros(0, dtype=np.int32)
    picks = []
    pos = -1
    while True:
        batch = int(total * p * 1.05) + 1024
        gaps = rng.geometric(p, size=batch).astype(np.int64)
        idx = pos + np.cumsum(gaps)
        inside = idx[idx < total]
        picks.append(inside)
        if inside.shape[0] < idx.shape[0]:
            break
        pos = int(idx[-1])
    t = np.concatenate(picks)
    # row i of the upper triangle starts at linear index i*(n-1) - i*(i-1)/2
    i_all = np.arange(n, dtype=np.int64)
    starts = i_all * (n - 1) - i_all * (i_all - 1) // 2
    i = np.searchsorted(starts, t, side="right") - 1
    j = t - starts[i] + i + 1
    return csr_from_edges(n, i, j)


def chung_lu(n: int, m_target: int, gamma: float, seed: int, log=None):
    """Chung-Lu power-law graph, uncapped weights w_i ~ (i+1)^(-1/(gamma-1)).

    Both endpoints of an edge are drawn independently with probability
    proportional to their weight.  Draws continue until ``m_target`` distinct
    non-loop pairs were seen; the first ``m_target`` distinct pairs in draw order
    are kept.  Vertex ids are then shuffled so that id and degree are unrelated.
    Uniforms are drawn in chunks (the same stream as one draw per batch), so
    large graphs need little temporary memory; ``log`` receives progress lines.
    """
    rng = _rng(seed, STREAM_EDGES)
    w = np.power(np.arange(1, n + 1, dtype=np.float64), -1.0 / (gamma - 1.0))
    cdf = np.cumsum(w)
    cdf /= cdf[-1]
    del w
    chunk = 1 << 24
    itype = np.int32 if n < (1 << 31) else np.int64

    def endpoints(count):
        out = np.empty(count, dtype=itype)
        for i, s0 in enumerate(range(0, count, chunk)):
            s1 = min(count, s0 + chunk)
            out[s0:s1] = np.minimum(np.searchsorted(cdf, rng.random(s1 - s0), side="right"), n - 1)
            if log and i % 4 == 3:
                log(f"chung_lu: {s1} of {count} endpoints")
        return out

    all_keys = np.zeros(0, dtype=np.int64)
    while True:
        need = m_target - all_keys.shape[0]
        batch = int(need * 1.3) + 4096
        a = endpoints(batch)
        b = endpoints(batch)
        if log:
            log(f"chung_lu: {2 * batch} endpoints drawn")
        keep = a != b
        a, b = a[keep].astype(np.int64), b[keep].astype(np.int64)
        key = np.minimum(a, b) * n + np.maximum(a, b)
        del a, b, keep
        all_keys = np.concatenate([all_keys, key])
        del key
        # keep the distinct pairs in the order they were first drawn
        if log:
            log(f"chung_lu: deduplicating {all_keys.shape[0]} pairs")
        _, first = np.unique(all_keys, return_index=True)
        first.sort()
        if log:
            log(f"chung_lu: {all_keys.shape[0]} pairs drawn, {first.shape[0]} distinct of {m_target}")
        if first.shape[0] >= m_target:
            all_keys = all_keys[first[:m_target]]
            break
        all_keys = all_keys[first]
        del first
    lo = all_keys // n
    hi = all_keys % n
    del all_keys
    perm = _rng(seed, STREAM_PERM).permutation(n).astype(np.int64)
    out = csr_from_edges(n, perm[lo], perm[hi], log=log)
    if log:
        log("chung_lu: CSR built")
    return out


def rmat(scale: int, edge_factor: int, a: float, b: float, c: float, seed: int, chunk: int = 1 << 24, log=None):
    """R-MAT (Graph500 style): 2^scale vertices, edge_factor * 2^scale samples.

    Each sample picks one quadrant per bit level with probabilities a, b, c and
    d = 1 - a - b - c.  Samples are then deduplicated and symmetrised, self-loops
    dropped, and vertex ids shuffled by a seeded permutation.
    """
    n = 1 << scale
    samples = edge_factor * n
    rng = _rng(seed, STREAM_EDGES)
    keys = []
    done = 0
    ab = a + b
    abc = a + b + c
    while done < samples:
        cnt = min(chunk, samples - done)
        src = np.zeros(cnt, dtype=np.int64)
        dst = np.zeros(cnt, dtype=np.int64)
        for level in range(scale):
            u = rng.random(cnt, dtype=np.float32)
            sbit = u >= ab
            dbit = ((u >= a) & (u < ab)) | (u >= abc)
            src |= sbit.astype(np.int64) << level
            dst |= dbit.astype(np.int64) << level
        keep = src != dst
        lo = np.minimum(src[keep], dst[keep])
        hi = np.maximum(src[keep], dst[keep])
        keys.append(np.unique(lo * n + hi))
        done += cnt
        if log and (done // cnt) % 8 == 0:
            log(f"rmat: {done} of {samples} samples")
    key = _sorted_unique(np.concatenate(keys), n * n, log)
    del keys
    perm = _rng(seed, STREAM_PERM).permutation(n).astype(np.int64)
    return csr_from_edges(n, perm[key // n], perm[key % n], log=log)


def uniform_labels(n: int, num_labels: int, seed: int) -> np.ndarray:
    rng = _rng(seed, STREAM_LABELS)
    return rng.integers(0, num_labels, size=n).astype(np.int32)


def zipf_labels(n: int, num_labels: int, s: float, seed: int) -> np.ndarray:
    """P(label = r-1) proportional to r^-s for r = 1..num_labels."""
    rng = _rng(seed, STREAM_LABELS)
    p = np.power(np.arange(1, num_labels + 1, dtype=np.float64), -s)
    p /= p.sum()
    return rng.choice(num_labels, size=n, p=p).astype(np.int32)


def make_graph(spec: dict, log=None) -> Graph:
    """Build a graph from a plain dict spec.

    ``{"kind": "er", "n", "p"}``, ``{"kind": "chung_lu" | "chung_lu_native", "n", "m", "gamma"}`` or
    ``{"kind": "rmat" | "rmat_native", "scale", "edge_factor", "a", "b", "c"}``, each with
    ``"seed"`` and ``"labels": {"kind": "uniform"|"zipf", "L", ["s"]}``.
    """
    kind = spec["kind"]
    seed = int(spec["seed"])
    if kind == "er":
        n = int(spec["n"])
        row_ptr, col = erdos_renyi(n, float(spec["p"]), seed)
    elif kind == "chung_lu":
        n = int(spec["n"])
        row_ptr, col = chung_lu(n, int(spec["m"]), float(spec["gamma"]), seed, log=log)
    elif kind == "chung_lu_native":
        from . import native

        n = int(spec["n"])
        if log:
            log(f"chung_lu (native): n {n}, m {spec['m']}")
        row_ptr, col = native.chung_lu_csr(n, int(spec["m"]), float(spec["gamma"]), seed)
        if log:
            log(f"chung_lu (native): {col.shape[0] // 2} edges")
    elif kind == "rmat_native":
        from . import native

        n = 1 << int(spec["scale"])
        if log:
            log(f"rmat (native): scale {spec['scale']}")
        row_ptr, col = native.rmat_csr(int(spec["scale"]), int(spec.get("edge_factor", 16)),
                                       float(spec.get("a", 0.57)), float(spec.get("b", 0.19)),
                                       float(spec.get("c", 0.19)), seed)
        if log:
            log(f"rmat (native): {col.shape[0] // 2} edges")
    elif kind == "rmat":
        n = 1 << int(spec["scale"])
        row_ptr, col = rmat(
            int(spec["scale"]),
            int(spec.get("edge_factor", 16)),
            float(spec.get("a", 0.57)),
            float(spec.get("b", 0.19)),
            float(spec.get("c", 0.19)),
            seed,
            log=log,
        )
    else:
        raise ValueError(f"unknown graph kind {kind!r}")
    lab = spec["labels"]
    if lab["kind"] == "uniform":
        label = uniform_labels(n, int(lab["L"]), seed)
    elif lab["kind"] == "zipf":
        label = zipf_labels(n, int(lab["L"]), float(lab["s"]), seed)
    else:
        raise ValueError(f"unknown label kind {lab['kind']!r}")
    return Graph(n=n, row_ptr=row_ptr, col=col, label=label, name=spec.get("name", kind), params=dict(spec))
