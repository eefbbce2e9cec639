"""Native (C, pthreads) generators for very large R-MAT and Chung-Lu graphs.

``rmat_csr`` and ``chung_lu_csr`` build the same kinds of graph as
:func:`synth.graphs.rmat` and :func:`synth.graphs.chung_lu` (loops dropped,
duplicates merged, ids permuted, rows sorted) from a counter-based SplitMix64
stream instead of PCG64, using all host threads; they are how the largest
configurations are generated in seconds rather than the minutes numpy needs.
Input generation only.
"""

from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "rmat_native.c")
_LIB = os.path.join(_HERE, "librmat_native.so")
_lib = None


def build(force: bool = True) -> str:
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O3", "-std=gnu11", "-Wall", "-Wextra", "-shared", "-fPIC", "-pthread",
                               _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        lib = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        lib.rmat_csr.restype = ctypes.c_int
        lib.rmat_csr.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                 ctypes.c_uint64, ctypes.c_int, ctypes.POINTER(P), ctypes.POINTER(P),
                                 ctypes.POINTER(ctypes.c_int64)]
        lib.chung_lu_csr.restype = ctypes.c_int
        lib.chung_lu_csr.argtypes = [ctypes.c_int64, ctypes.c_int64, ctypes.c_double, ctypes.c_uint64, ctypes.c_int,
                                     ctypes.POINTER(P), ctypes.POINTER(P), ctypes.POINTER(ctypes.c_int64)]
        lib.rmat_free.restype = None
        lib.rmat_free.argtypes = [P]
        _lib = lib
    return _lib


def rmat_csr(scale: int, edge_factor: int, a: float, b: float, c: float, seed: int, threads: int = 0):
    """(row_ptr int64[n+1], col int32[nnz]) of the R-MAT graph; see the module docstring."""
    lib = _load()
    nt = threads or min(64, os.cpu_count() or 1)
    rp, col = ctypes.c_void_p(), ctypes.c_void_p()
    nnz = ctypes.c_int64()
    st = lib.rmat_csr(int(scale), int(edge_factor), float(a), float(b), float(c), int(seed) & (2**64 - 1), int(nt),
                      ctypes.byref(rp), ctypes.byref(col), ctypes.byref(nnz))
    if st == 1:
        raise ValueError("bad R-MAT parameters")
    if st != 0:
        raise MemoryError("R-MAT generation ran out of memory")
    n = 1 << int(scale)
    try:
        row_ptr = np.ctypeslib.as_array(ctypes.cast(rp, ctypes.POINTER(ctypes.c_int64)), shape=(n + 1,)).copy()
        c_arr = np.ctypeslib.as_array(ctypes.cast(col, ctypes.POINTER(ctypes.c_int32)), shape=(max(nnz.value, 1),))
        col_out = c_arr[: nnz.value].copy()
    finally:
        lib.rmat_free(rp)
        lib.rmat_free(col)
    return row_ptr, col_out


def chung_lu_csr(n: int, m: int, gamma: float, seed: int, threads: int = 0):
    """(row_ptr int64[n+1], col int32[2m]) of the Chung-Lu graph; see the module docstring."""
    lib = _load()
    nt = threads or min(64, os.cpu_count() or 1)
    rp, col = ctypes.c_void_p(), ctypes.c_void_p()
    nnz = ctypes.c_int64()
    st = lib.chung_lu_csr(int(n), int(m), float(gamma), int(seed) & (2**64 - 1), int(nt), ctypes.byref(rp),
                          ctypes.byref(col), ctypes.byref(nnz))
    if st == 1:
        raise ValueError("bad Chung-Lu parameters")
    if st != 0:
        raise MemoryError("Chung-Lu generation ran out of memory")
    try:
        row_ptr = np.ctypeslib.as_array(ctypes.cast(rp, ctypes.POINTER(ctypes.c_int64)), shape=(int(n) + 1,)).copy()
        c_arr = np.ctypeslib.as_array(ctypes.cast(col, ctypes.POINTER(ctypes.c_int32)), shape=(max(nnz.value, 1),))
        col_out = c_arr[: nnz.value].copy()
    finally:
        lib.rmat_free(rp)
        lib.rmat_free(col)
    return row_ptr, col_out
