"""ctypes binding of ``libcstm.so`` (see ``include/cstm.h``).

Argument marshalling only: every step of the matching path runs in the HIP
library.  PyTorch provides device memory and streams.  Loading fails with an
ImportError when the library has not been built; there is no fallback.
"""

from __future__ import annotations

import ctypes
import os
import weakref

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libcstm.so")

MAX_K = 32

OK, EINVAL, ENOMEM, EDEVICE, ETIMEOUT, EOVERFLOW, ECANCELLED = range(7)
STATUS_NAMES = {0: "OK", 1: "EINVAL", 2: "ENOMEM", 3: "EDEVICE", 4: "ETIMEOUT", 5: "EOVERFLOW", 6: "ECANCELLED"}


class CstmError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


class cstm_tune(ctypes.Structure):
    _fields_ = [
        ("part_budget_bytes", ctypes.c_uint64),
        ("max_list_len", ctypes.c_int32),
        ("waves_per_wg", ctypes.c_int32),
        ("wgs_per_cu", ctypes.c_int32),
        ("collect_stats", ctypes.c_int32),
        ("enum_mode", ctypes.c_int32),
        ("max_replication", ctypes.c_int32),
        ("deadline_ms", ctypes.c_int32),
        ("hbm_wgs_per_cu", ctypes.c_int32),
        ("hbm_donate_period", ctypes.c_int32),
        ("hbm_flat_max", ctypes.c_int32),
        ("hbm_donate_last_min", ctypes.c_int32),
        ("last_level_sum", ctypes.c_int32),
        ("hbm_donate_min", ctypes.c_int32),
        ("batch_order", ctypes.c_int32),
        ("hbm_idle_ms", ctypes.c_int32),
        ("order_rule", ctypes.c_int32),
        ("serve_wgs_per_cu", ctypes.c_int32),
    ]


MODE_AUTO, MODE_LDS, MODE_HBM = 0, 1, 2


class cstm_enum_stats(ctypes.Structure):
    _fields_ = [
        ("kernel_ms", ctypes.c_double),
        ("mode", ctypes.c_int32),
        ("launches", ctypes.c_int32),
        ("images", ctypes.c_uint64),
        ("image_bytes", ctypes.c_uint64),
        ("extensions", ctypes.c_uint64),
        ("edge_checks", ctypes.c_uint64),
        ("pushed", ctypes.c_uint64),
        ("busy_frac", ctypes.c_double),
        ("summed", ctypes.c_uint64),
        ("chunks", ctypes.c_uint64),
    ]


class cstm_share_stats(ctypes.Structure):
    _fields_ = [
        ("delta", ctypes.c_double),
        ("w_host", ctypes.c_uint64),
        ("w_device", ctypes.c_uint64),
        ("groups_host", ctypes.c_int64),
        ("groups_device", ctypes.c_int64),
        ("count_host", ctypes.c_uint64),
        ("count_device", ctypes.c_uint64),
        ("copy_ms", ctypes.c_double),
        ("host_ms", ctypes.c_double),
        ("device_ms", ctypes.c_double),
        ("wall_ms", ctypes.c_double),
        ("host_threads", ctypes.c_int32),
        ("reserved", ctypes.c_int32),
    ]


class cstm_request_result(ctypes.Structure):
    _fields_ = [
        ("done", ctypes.c_int32),
        ("status", ctypes.c_int32),
        ("count", ctypes.c_uint64),
        ("submit_s", ctypes.c_double),
        ("admit_s", ctypes.c_double),
        ("built_s", ctypes.c_double),
        ("launch_s", ctypes.c_double),
        ("done_s", ctypes.c_double),
        ("batch_size", ctypes.c_int32),
        ("lane", ctypes.c_int32),
    ]


class cstm_server_stats(ctypes.Structure):
    _fields_ = [
        ("submitted", ctypes.c_uint64),
        ("completed", ctypes.c_uint64),
        ("failed", ctypes.c_uint64),
        ("launches", ctypes.c_uint64),
        ("batched", ctypes.c_uint64),
        ("peak_bytes", ctypes.c_uint64),
        ("in_use_bytes", ctypes.c_uint64),
        ("max_overlap", ctypes.c_int32),
        ("reserved", ctypes.c_int32),
        ("admission_bytes", ctypes.c_uint64),
        ("kernel_ms", ctypes.c_double),
        ("extensions", ctypes.c_uint64),
        ("edge_checks", ctypes.c_uint64),
        ("pushed", ctypes.c_uint64),
        ("summed", ctypes.c_uint64),
        ("chunks", ctypes.c_uint64),
    ]


class cstm_cst_info(ctypes.Structure):
    _fields_ = [
        ("k", ctypes.c_int32),
        ("root", ctypes.c_int32),
        ("parent", ctypes.c_int32 * MAX_K),
        ("order", ctypes.c_int32 * MAX_K),
        ("cand", ctypes.c_int64 * MAX_K),
        ("tree_entries", ctypes.c_int64),
        ("nontree_entries", ctypes.c_int64),
        ("bytes", ctypes.c_uint64),
        ("d_cst", ctypes.c_int32),
        ("n_nontree", ctypes.c_int32),
        ("n_parts", ctypes.c_int64),
        ("part_bytes", ctypes.c_uint64),
        ("max_part_bytes", ctypes.c_uint64),
    ]


ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p)
FREE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p)

EXPORTS = [
    "cstm_ctx_create", "cstm_ctx_destroy", "cstm_ctx_get_tune", "cstm_ctx_set_tune", "cstm_ctx_lds_bytes",
    "cstm_graph_load", "cstm_graph_free", "cstm_graph_info", "cstm_graph_label_edges",
    "cstm_cst_build", "cstm_cst_partition", "cstm_cst_info_get", "cstm_cst_candidates",
    "cstm_enumerate", "cstm_batch_enumerate", "cstm_cst_times", "cstm_cst_free",
    "cstm_last_error", "cstm_version", "cstm_ctx_last_enum_stats", "cstm_cst_estimate",
    "cstm_server_create", "cstm_server_submit", "cstm_server_poll", "cstm_server_wait", "cstm_server_get_stats",
    "cstm_server_destroy", "cstm_cst_workload", "cstm_cst_build_ordered", "cstm_enumerate_shared",
    "cstm_enumerate_noalloc",
]

# bytes of the fixed device array cstm_enumerate_noalloc works in (CSTM_NOALLOC_SCRATCH_BYTES)
NOALLOC_SCRATCH_BYTES = 12 << 20

_lib = None


def load_library():
    """Load ``libcstm.so``; raises ImportError if it was not built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_2102_10768_amd.build`")
    # PyTorch ships its own HIP runtime with the same soname as the system one.
    # Loading torch first makes the library bind to that runtime, so one process
    # never holds two HIP runtimes (the second would see no device).
    import torch  # noqa: F401

    lib = ctypes.CDLL(LIB_PATH)
    P = ctypes.c_void_p
    I32, I64, U64 = ctypes.c_int32, ctypes.c_int64, ctypes.c_uint64
    st = ctypes.c_int
    sig = {
        "cstm_ctx_create": (st, [ctypes.c_int, ALLOC_FN, FREE_FN, P, ctypes.POINTER(cstm_tune), ctypes.POINTER(P)]),
        "cstm_ctx_destroy": (None, [P]),
        "cstm_ctx_get_tune": (st, [P, ctypes.POINTER(cstm_tune)]),
        "cstm_ctx_set_tune": (st, [P, ctypes.POINTER(cstm_tune)]),
        "cstm_ctx_lds_bytes": (st, [P, ctypes.POINTER(I64)]),
        "cstm_graph_load": (st, [P, I64, I64, P, P, P, ctypes.c_int, P, ctypes.POINTER(P)]),
        "cstm_graph_free": (None, [P]),
        "cstm_graph_info": (st, [P, ctypes.POINTER(I64), ctypes.POINTER(I64), ctypes.POINTER(I32), ctypes.POINTER(I64)]),
        "cstm_graph_label_edges": (st, [P, P, I64, ctypes.POINTER(I64)]),
        "cstm_cst_build": (st, [P, P, I32, P, I32, P, P, ctypes.POINTER(P)]),
        "cstm_cst_partition": (st, [P, U64, I32, U64, ctypes.POINTER(I64)]),
        "cstm_cst_info_get": (st, [P, ctypes.POINTER(cstm_cst_info)]),
        "cstm_cst_candidates": (st, [P, I32, P, I64, ctypes.POINTER(I64)]),
        "cstm_enumerate": (st, [P, ctypes.c_int, U64, P, U64, ctypes.POINTER(U64), ctypes.POINTER(U64),
                                ctypes.c_double, P]),
        "cstm_batch_enumerate": (st, [P, I32, P, P, P, P]),
        "cstm_cst_times": (st, [P, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double),
                                ctypes.POINTER(ctypes.c_double)]),
        "cstm_cst_free": (None, [P]),
        "cstm_ctx_last_enum_stats": (st, [P, ctypes.POINTER(cstm_enum_stats)]),
        "cstm_cst_estimate": (st, [P, I32, P, I32, P, ctypes.POINTER(U64)]),
        "cstm_server_create": (st, [P, P, U64, I32, I32, I32, I32, ctypes.POINTER(P)]),
        "cstm_server_submit": (st, [P, I32, P, I32, P, U64, ctypes.POINTER(U64)]),
        "cstm_server_poll": (st, [P, U64, ctypes.POINTER(cstm_request_result)]),
        "cstm_server_wait": (st, [P, U64, ctypes.c_double, ctypes.POINTER(cstm_request_result)]),
        "cstm_server_get_stats": (st, [P, ctypes.POINTER(cstm_server_stats)]),
        "cstm_server_destroy": (None, [P]),
        "cstm_cst_workload": (st, [P, ctypes.POINTER(ctypes.c_uint64)]),
        "cstm_cst_build_ordered": (st, [P, P, I32, P, I32, P, P, P, ctypes.POINTER(P)]),
        "cstm_enumerate_shared": (st, [P, ctypes.c_double, I64, I32, ctypes.POINTER(U64),
                                       ctypes.POINTER(cstm_share_stats), P]),
        "cstm_enumerate_noalloc": (st, [P, U64, ctypes.POINTER(U64), ctypes.c_double, P]),
        "cstm_last_error": (ctypes.c_char_p, []),
        "cstm_version": (ctypes.c_char_p, []),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def _check(status: int):
    if status != OK:
        msg = load_library().cstm_last_error().decode(errors="replace")
        raise CstmError(status, msg)


def _stream_ptr(stream):
    if stream is None:
        import torch

        return torch.cuda.current_stream().cuda_stream
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream


# ---------------------------------------------------------------- thin object wrappers


class Context:
    """A device context (``cstm_ctx_create``).  ``tune`` is a dict of cstm_tune fields."""

    def __init__(self, device: int = 0, tune: dict | None = None, torch_allocator: bool = False, allocator=None):
        """``allocator``: optional (alloc(nbytes) -> device pointer or 0, free(ptr)) pair
        of Python callables used for every device allocation of the library."""
        lib = load_library()
        self._keep = []
        alloc = ALLOC_FN()
        free = FREE_FN()
        if allocator is not None:
            user_alloc, user_free = allocator

            def _alloc_cb(nbytes, user):
                return user_alloc(int(nbytes)) or None

            def _free_cb(ptr, user):
                user_free(ptr)

            alloc, free = ALLOC_FN(_alloc_cb), FREE_FN(_free_cb)
            self._keep += [alloc, free]
        elif torch_allocator:
            import torch

            def _alloc(nbytes, user):
                try:
                    return torch.cuda.caching_allocator_alloc(int(nbytes), device)
                except Exception:
                    return None

            def _free(ptr, user):
                torch.cuda.caching_allocator_delete(ptr)

            alloc, free = ALLOC_FN(_alloc), FREE_FN(_free)
            self._keep += [alloc, free]
        t = cstm_tune(**(tune or {}))
        h = ctypes.c_void_p()
        _check(lib.cstm_ctx_create(device, alloc, free, None, ctypes.byref(t), ctypes.byref(h)))
        self.handle = h
        self.device = device
        # graphs and CSTs made in this context; closed before it (they return memory to it)
        self._children = weakref.WeakSet()

    @property
    def tune(self) -> dict:
        t = cstm_tune()
        _check(load_library().cstm_ctx_get_tune(self.handle, ctypes.byref(t)))
        return {f: getattr(t, f) for f, _ in cstm_tune._fields_}

    @tune.setter
    def tune(self, values: dict):
        cur = self.tune
        cur.update(values)
        t = cstm_tune(**cur)
        _check(load_library().cstm_ctx_set_tune(self.handle, ctypes.byref(t)))

    def last_enum_stats(self) -> dict:
        v = cstm_enum_stats()
        _check(load_library().cstm_ctx_last_enum_stats(self.handle, ctypes.byref(v)))
        return {f: getattr(v, f) for f, _ in cstm_enum_stats._fields_}

    def lds_bytes(self) -> int:
        v = ctypes.c_int64()
        _check(load_library().cstm_ctx_lds_bytes(self.handle, ctypes.byref(v)))
        return v.value

    def close(self):
        if getattr(self, "handle", None):
            for child in sorted(list(self._children), key=lambda c: isinstance(c, Graph)):
                child.close()
            load_library().cstm_ctx_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Graph:
    """A resident data graph (``cstm_graph_load``).

    Pass torch CUDA tensors (borrowed: the tensors are kept referenced here) or
    numpy / CPU arrays (copied to the device).
    """

    def __init__(self, ctx: Context, row_ptr, col, label, stream=None):
        lib = load_library()
        self.ctx = ctx
        on_device = _is_cuda(row_ptr)
        if on_device:
            import torch

            self._tensors = (row_ptr.contiguous(), col.contiguous(), label.contiguous())
            assert self._tensors[0].dtype == torch.int64 and self._tensors[1].dtype == torch.int32
            ptrs = [t.data_ptr() for t in self._tensors]
            n = self._tensors[2].numel()
            nnz = self._tensors[1].numel()
        else:
            self._tensors = (
                np.ascontiguousarray(row_ptr, dtype=np.int64),
                np.ascontiguousarray(col, dtype=np.int32),
                np.ascontiguousarray(label, dtype=np.int32),
            )
            ptrs = [a.ctypes.data for a in self._tensors]
            n = self._tensors[2].shape[0]
            nnz = self._tensors[1].shape[0]
        h = ctypes.c_void_p()
        _check(lib.cstm_graph_load(ctx.handle, n, nnz, ptrs[0], ptrs[1], ptrs[2], int(on_device),
                                   _stream_ptr(stream) if on_device else None, ctypes.byref(h)))
        self.handle = h
        ctx._children.add(self)
        if not on_device:
            self._tensors = None

    def estimate_bytes(self, qlabel, qedges) -> int:
        """Upper bound on the device bytes a CST build for this query would use."""
        ql = np.ascontiguousarray(qlabel, dtype=np.int32)
        qe = np.ascontiguousarray(np.asarray(qedges, dtype=np.int32).reshape(-1, 2))
        out = ctypes.c_uint64()
        _check(load_library().cstm_cst_estimate(self.handle, int(ql.shape[0]), ql.ctypes.data, int(qe.shape[0]),
                                                qe.ctypes.data if qe.size else None, ctypes.byref(out)))
        return out.value

    def info(self) -> dict:
        n, nnz, L, md = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int32(), ctypes.c_int64()
        _check(load_library().cstm_graph_info(self.handle, ctypes.byref(n), ctypes.byref(nnz), ctypes.byref(L),
                                              ctypes.byref(md)))
        return {"n": n.value, "nnz": nnz.value, "num_labels": L.value, "max_degree": md.value}

    def label_edges(self):
        """(L, L) uint64 array of edges between label pairs, or None when not made."""
        n = ctypes.c_int64()
        _check(load_library().cstm_graph_label_edges(self.handle, None, 0, ctypes.byref(n)))
        if n.value == 0:
            return None
        out = np.zeros(n.value, dtype=np.uint64)
        _check(load_library().cstm_graph_label_edges(self.handle, out.ctypes.data, n.value, ctypes.byref(n)))
        L = int(round(n.value ** 0.5))
        return out.reshape(L, L)

    def close(self):
        if getattr(self, "handle", None):
            load_library().cstm_graph_free(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class CST:
    """One query's candidate search tree (``cstm_cst_build``)."""

    def __init__(self, ctx: Context, graph: Graph, qlabel, qedges, stream=None, order=None):
        """``order``: the matching order (a permutation of the query vertices
        that starts at the CST root and puts every vertex after its BFS-tree
        parent); None keeps the path-based order of Section V-B."""
        lib = load_library()
        self.ctx, self.graph = ctx, graph
        ql = np.ascontiguousarray(qlabel, dtype=np.int32)
        qe = np.ascontiguousarray(np.asarray(qedges, dtype=np.int32).reshape(-1, 2))
        self.k = int(ql.shape[0])
        h = ctypes.c_void_p()
        if order is None:
            _check(lib.cstm_cst_build(ctx.handle, graph.handle, self.k, ql.ctypes.data, int(qe.shape[0]),
                                      qe.ctypes.data if qe.size else None, _stream_ptr(stream),
                                      ctypes.byref(h)))
        else:
            od = np.ascontiguousarray(order, dtype=np.int32)
            if od.shape != (self.k,):
                raise ValueError(f"order must hold {self.k} vertices, got shape {od.shape}")
            _check(lib.cstm_cst_build_ordered(ctx.handle, graph.handle, self.k, ql.ctypes.data,
                                              int(qe.shape[0]), qe.ctypes.data if qe.size else None,
                                              od.ctypes.data, _stream_ptr(stream), ctypes.byref(h)))
        self.handle = h
        ctx._children.add(self)

    def partition(self, budget_bytes: int = 0, max_list_len: int = 0, max_total_bytes: int = 0) -> int:
        """Algorithm 2; returns the number of partitions.  Raises ``CstmError``
        (ENOMEM) when the images would exceed ``max_total_bytes`` (0: no limit)."""
        n = ctypes.c_int64()
        _check(load_library().cstm_cst_partition(self.handle, int(budget_bytes), int(max_list_len),
                                                 int(max_total_bytes), ctypes.byref(n)))
        return n.value

    def workload(self) -> int:
        """W_CST of the workload DP (Section V-C), exactly min(W_CST, 2^64 - 1)."""
        w = ctypes.c_uint64()
        _check(load_library().cstm_cst_workload(self.handle, ctypes.byref(w)))
        return w.value

    def count_shared(self, delta: float, n_runs: int = 0, host_threads: int = 0, stream=None):
        """Algorithm 3: count with a share of at most ``delta`` of W_CST on the
        host cores and the rest on the GPU.  Returns (count, stats dict)."""
        c = ctypes.c_uint64()
        st = cstm_share_stats()
        _check(load_library().cstm_enumerate_shared(self.handle, float(delta), int(n_runs), int(host_threads),
                                                    ctypes.byref(c), ctypes.byref(st), _stream_ptr(stream)))
        return int(c.value), {name: getattr(st, name) for name, _ in cstm_share_stats._fields_ if name != "reserved"}

    def info(self) -> dict:
        i = cstm_cst_info()
        _check(load_library().cstm_cst_info_get(self.handle, ctypes.byref(i)))
        k = i.k
        return {
            "k": k, "root": i.root, "parent": list(i.parent[:k]), "order": list(i.order[:k]),
            "cand": list(i.cand[:k]), "tree_entries": i.tree_entries, "nontree_entries": i.nontree_entries,
            "bytes": i.bytes, "d_cst": i.d_cst, "n_nontree": i.n_nontree, "n_parts": i.n_parts,
            "part_bytes": i.part_bytes, "max_part_bytes": i.max_part_bytes,
        }

    def candidates(self, u: int) -> np.ndarray:
        lib = load_library()
        n = ctypes.c_int64()
        _check(lib.cstm_cst_candidates(self.handle, u, None, 0, ctypes.byref(n)))
        out = np.zeros(n.value, dtype=np.int32)
        _check(lib.cstm_cst_candidates(self.handle, u, out.ctypes.data, n.value, ctypes.byref(n)))
        return out

    def count(self, stream=None, limit: int = 0, deadline_s: float = 0.0) -> int:
        """Number of embeddings; with ``limit`` > 0, exactly min(total, limit)."""
        c, w = ctypes.c_uint64(), ctypes.c_uint64()
        _check(load_library().cstm_enumerate(self.handle, 0, int(limit), None, 0, ctypes.byref(c), ctypes.byref(w),
                                             float(deadline_s), _stream_ptr(stream)))
        return c.value

    def count_noalloc(self, stream=None, limit: int = 0, deadline_s: float = 0.0) -> int:
        """As :meth:`count`, through ``cstm_enumerate_noalloc`` (no device allocation)."""
        c = ctypes.c_uint64()
        _check(load_library().cstm_enumerate_noalloc(self.handle, int(limit), ctypes.byref(c), float(deadline_s),
                                                     _stream_ptr(stream)))
        return c.value

    def list(self, cap: int, stream=None, allow_overflow: bool = False, limit: int = 0, deadline_s: float = 0.0):
        """Returns (count, rows): rows is a (min(count, cap), k) int32 CUDA tensor.

        Raises on overflow (count > cap) unless ``allow_overflow``; the count is exact either way.
        With ``limit`` > 0 the count is min(total, limit) and at most that many rows are returned.
        """
        import torch

        rows = torch.empty((max(cap, 1), self.k), dtype=torch.int32, device=f"cuda:{self.ctx.device}")
        c, w = ctypes.c_uint64(), ctypes.c_uint64()
        st = load_library().cstm_enumerate(self.handle, 1, int(limit), rows.data_ptr(), int(cap), ctypes.byref(c),
                                           ctypes.byref(w), float(deadline_s), _stream_ptr(stream))
        if not (allow_overflow and st == EOVERFLOW):
            _check(st)
        return c.value, rows[: w.value]

    def times(self) -> dict:
        b, p, e = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
        _check(load_library().cstm_cst_times(self.handle, ctypes.byref(b), ctypes.byref(p), ctypes.byref(e)))
        return {"build_ms": b.value, "partition_ms": p.value, "enumerate_ms": e.value}

    def close(self):
        if getattr(self, "handle", None):
            load_library().cstm_cst_free(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Server:
    """``cstm_server_*``: the library's request loop over a resident graph.

    ``submit`` queues a query and returns a ticket; ``wait``/``poll`` return a
    dict (``done``, ``status``, ``count``, ``submit_s``, ``done_s`` on the
    server's clock, ``batch_size``, ``lane``) once, when the request is done.
    """

    def __init__(self, ctx: Context, graph: "Graph", mem_budget: int = 64 << 30, lanes: int = 2,
                 builders: int = 2, max_batch: int = 256, batch_wait_us: int = 0):
        self.ctx = ctx
        self.graph = graph
        h = ctypes.c_void_p()
        _check(load_library().cstm_server_create(ctx.handle, graph.handle, int(mem_budget), int(lanes),
                                                 int(builders), int(max_batch), int(batch_wait_us),
                                                 ctypes.byref(h)))
        self.handle = h
        ctx._children.add(self)

    def submit(self, qlabel, qedges, limit: int = 0) -> int:
        ql = np.ascontiguousarray(qlabel, dtype=np.int32)
        qe = np.ascontiguousarray(np.asarray(qedges, dtype=np.int32).reshape(-1, 2))
        t = ctypes.c_uint64()
        _check(load_library().cstm_server_submit(self.handle, int(ql.shape[0]), ql.ctypes.data, int(qe.shape[0]),
                                                 qe.ctypes.data if qe.size else None, int(limit), ctypes.byref(t)))
        return t.value

    @staticmethod
    def _result(r: cstm_request_result) -> dict:
        return {f: getattr(r, f) for f, _ in cstm_request_result._fields_}

    def poll(self, ticket: int) -> dict:
        r = cstm_request_result()
        _check(load_library().cstm_server_poll(self.handle, int(ticket), ctypes.byref(r)))
        return self._result(r)

    def wait(self, ticket: int, timeout_s: float = 0.0) -> dict:
        r = cstm_request_result()
        _check(load_library().cstm_server_wait(self.handle, int(ticket), float(timeout_s), ctypes.byref(r)))
        return self._result(r)

    def stats(self) -> dict:
        v = cstm_server_stats()
        _check(load_library().cstm_server_get_stats(self.handle, ctypes.byref(v)))
        return {f: getattr(v, f) for f, _ in cstm_server_stats._fields_}

    def close(self):
        """Finish every submitted request, then free the server."""
        if getattr(self, "handle", None):
            load_library().cstm_server_destroy(self.handle)
            self.handle = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def batch_count(ctx: Context, csts: list, stream=None, limits=None) -> list[int]:
    """``cstm_batch_enumerate``: counts of many CSTs from one persistent launch.

    ``limits`` (optional, one per CST, 0 = all): each count is min(total, limit)."""
    n = len(csts)
    arr = (ctypes.c_void_p * max(n, 1))(*[c.handle.value for c in csts])
    out = (ctypes.c_uint64 * max(n, 1))()
    lim = None
    if limits is not None:
        assert len(limits) == n
        lim = (ctypes.c_uint64 * max(n, 1))(*[int(x) for x in limits])
    _check(load_library().cstm_batch_enumerate(ctx.handle, n, arr, lim, out, _stream_ptr(stream)))
    return [int(out[i]) for i in range(n)]


def _is_cuda(x) -> bool:
    try:
        import torch

        return isinstance(x, torch.Tensor) and x.is_cuda
    except ImportError:
        return False
