"""CPU oracle for subgraph matching.  TEST INFRASTRUCTURE ONLY.

Only ``tests/``, the smoke check in ``__graft_entry__`` and the CPU-baseline leg
of ``bench.py`` may import this package.  It shares no code with the HIP path.

* :func:`match` -- C backtracking matcher on G (``oracle.c``): the exact count
  and, for small cases, the sorted list of all embeddings (Section II-A,
  Definition 1).
* :mod:`oracle.cst_ref` -- plain Python restatement of the CST construction
  (Algorithm 1), the partition rule (Algorithm 2), the workload estimate and one
  generator/validator/synchronizer round, used to pin the CST-level invariants.
"""

from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")

OK, EINVAL, ENOMEM, ETIMEOUT, EOVERFLOW = 0, 1, 2, 4, 5

_lib = None


def build(force: bool = True) -> str:
    """Compile ``oracle.c`` into ``liboracle.so`` next to it (gcc, -O3, pthreads)."""
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp"
        subprocess.check_call(
            ["gcc", "-O3", "-std=gnu11", "-Wall", "-Wextra", "-shared", "-fPIC", "-pthread", _SRC, "-o", tmp]
        )
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build()
        lib = ctypes.CDLL(_LIB_PATH)
        p = ctypes.c_void_p
        lib.oracle_match.restype = ctypes.c_int
        lib.oracle_match.argtypes = [
            ctypes.c_int64, p, p, p, p,  # n, row_ptr, col, label, label-grouped col
            ctypes.c_int32, p, ctypes.c_int32, p,  # k, qlabel, m_q, qedges
            ctypes.c_int, ctypes.c_int, ctypes.c_double, ctypes.c_uint64,  # degfilter, threads, deadline, budget
            ctypes.c_uint64,  # limit
            ctypes.c_int, p, ctypes.c_uint64, ctypes.c_int,  # list, rows, cap, mutate
            p, p, p, p,  # count, nodes, rows_written, threads_used
        ]
        lib.oracle_num_cores.restype = ctypes.c_int
        lib.oracle_label_group.restype = ctypes.c_int
        lib.oracle_label_group.argtypes = [ctypes.c_int64, p, p, p, p, ctypes.c_int]
        _lib = lib
    return _lib


def num_cores() -> int:
    return int(_load().oracle_num_cores())


class MatchResult:
    __slots__ = ("status", "count", "nodes", "rows", "threads")

    def __init__(self, status, count, nodes, rows, threads):
        self.status = status
        self.count = count
        self.nodes = nodes
        self.rows = rows
        self.threads = threads

    def __repr__(self):
        return f"MatchResult(status={self.status}, count={self.count}, nodes={self.nodes}, threads={self.threads})"


def label_grouped_col(g, threads: int = 0) -> np.ndarray:
    """G's rows regrouped by (neighbour label, neighbour id), same row_ptr.

    Passing it to :func:`match` lets the matcher visit only the neighbours of
    the label it needs; the result is the same.  Computed by ``oracle.c``
    (rows sorted independently on host threads), so it scales to
    billion-edge graphs; :func:`label_grouped_col_numpy` is the plain form."""
    lib = _load()
    row_ptr = _c(g.row_ptr, np.int64)
    col = _c(g.col, np.int32)
    label = _c(g.label, np.int32)
    out = np.empty_like(col)
    st = lib.oracle_label_group(int(g.n), row_ptr.ctypes.data, col.ctypes.data, label.ctypes.data,
                                out.ctypes.data, int(threads))
    if st != OK:
        raise MemoryError("label grouping ran out of host memory")
    return out


def label_grouped_col_numpy(g) -> np.ndarray:
    """The same regrouping as :func:`label_grouped_col`, by one numpy stable sort."""
    row_ptr = np.asarray(g.row_ptr, dtype=np.int64)
    col = np.asarray(g.col, dtype=np.int32)
    label = np.asarray(g.label, dtype=np.int64)
    L = int(label.max()) + 1 if label.size else 1
    row_of = np.repeat(np.arange(row_ptr.shape[0] - 1, dtype=np.int64), np.diff(row_ptr))
    key = row_of * L + label[col]
    del row_of
    # stable: ids stay ascending inside each (row, label) run
    idx = np.argsort(key, kind="stable")
    del key
    return np.ascontiguousarray(col[idx])


def _c(a, dtype):
    return np.ascontiguousarray(a, dtype=dtype)


def match(g, q, *, list_rows: bool = False, cap: int | None = None, degree_filter: bool = True,
          threads: int = 0, deadline_s: float = 0.0, node_budget: int = 0, mutate: int = 0,
          lcol: np.ndarray | None = None, limit: int = 0) -> MatchResult:
    """Count (and with ``list_rows`` list, sorted) all embeddings of ``q`` in ``g``.

    ``g`` has ``n``, ``row_ptr``, ``col``, ``label``; ``q`` has ``qlabel``, ``qedges``.
    ``lcol`` (optional) is :func:`label_grouped_col` of ``g``: same result, less scanning.
    ``limit`` > 0 (counting only) stops once that many embeddings were found;
    the count is then exactly min(total, limit).
    Raises ``ValueError`` on an invalid query.  A ``TIMEOUT`` status means the
    count is only a lower bound.
    """
    lib = _load()
    row_ptr = _c(g.row_ptr, np.int64)
    col = _c(g.col, np.int32)
    label = _c(g.label, np.int32)
    if lcol is not None:
        lcol = _c(lcol, np.int32)
        assert lcol.shape == col.shape
    qlabel = _c(q.qlabel, np.int32)
    qedges = _c(np.asarray(q.qedges).reshape(-1, 2), np.int32)
    k = int(qlabel.shape[0])
    if list_rows and cap is None:
        cap = 1 << 22
    cap = int(cap or 0)
    rows = np.zeros((cap, k), dtype=np.int32) if list_rows else None
    cnt = ctypes.c_uint64(0)
    nodes = ctypes.c_uint64(0)
    written = ctypes.c_uint64(0)
    used = ctypes.c_int(0)
    st = lib.oracle_match(
        int(g.n), row_ptr.ctypes.data, col.ctypes.data, label.ctypes.data,
        lcol.ctypes.data if lcol is not None else None, k, qlabel.ctypes.data, int(qedges.shape[0]), qedges.ctypes.data,
        int(bool(degree_filter)), int(threads), float(deadline_s), int(node_budget), int(limit),
        int(bool(list_rows)), rows.ctypes.data if rows is not None else None, cap, int(mutate),
        ctypes.byref(cnt), ctypes.byref(nodes), ctypes.byref(written), ctypes.byref(used),
    )
    if st == EINVAL:
        raise ValueError("invalid query (k out of range, bad label or edge, or disconnected)")
    out_rows = rows[: written.value] if rows is not None else None
    return MatchResult(st, int(cnt.value), int(nodes.value), out_rows, int(used.value))


def count(g, q, **kw) -> int:
    """Exact embedding count; raises if the search did not finish."""
    r = match(g, q, **kw)
    if r.status != OK:
        raise RuntimeError(f"oracle did not finish: status {r.status}")
    return r.count
