"""ORACLE -- TEST INFRASTRUCTURE ONLY.

Sequential CPU union-find that defines the answers of the bulk incremental
connectivity problem (Section 1 model; Algorithm 1; the Section 4 union-find;
the Section 6 "UF with path compression" baseline).  Only the tests, the smoke
check and the benchmark's CPU-baseline leg may import this package; the GPU
library never does, and shares no code with it.

The arithmetic lives in ``uf_oracle.c`` (plain C, built with gcc); this file
only marshals numpy arrays to it.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "uf_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")


def build_lib(force: bool = False) -> str:
    """Compile uf_oracle.c (single-threaded, -O2) into liboracle.so."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fPIC", "-shared", "-std=c11", "-o", tmp, _SRC])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def load_lib(path: str):
    """Load a compiled oracle library and declare its C signatures."""
    L = ctypes.CDLL(path)
    vp, i64, i32 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32
    L.uf_create.restype = vp
    L.uf_create.argtypes = [i64]
    L.uf_destroy.argtypes = [vp]
    L.uf_bulk_update.restype = i64
    L.uf_bulk_update.argtypes = [vp, vp, i64]
    L.uf_bulk_query.restype = i64
    L.uf_bulk_query.argtypes = [vp, vp, i64, vp]
    L.uf_labels.restype = ctypes.c_int
    L.uf_labels.argtypes = [vp, vp]
    for f in ("uf_num_components", "uf_unions", "uf_invalid", "uf_count_roots"):
        getattr(L, f).restype = i64
        getattr(L, f).argtypes = [vp]
    L.uf_max_height.restype = i32
    L.uf_max_height.argtypes = [vp]
    L.uf_parents.argtypes = [vp, vp]
    return L


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build_lib()
        _lib = load_lib(_LIB)
    return _lib


def _pairs(a) -> np.ndarray:
    a = np.ascontiguousarray(np.asarray(a, dtype=np.int32))
    if a.size == 0:
        return a.reshape(0, 2)
    assert a.ndim == 2 and a.shape[1] == 2, "pairs must be int32[k][2]"
    return a


class UnionFind:
    """Sequential union-find oracle over vertices [0, n)."""

    def __init__(self, n: int, _lib=None):
        self.n = int(n)
        self._L = _lib if _lib is not None else lib()
        self._h = self._L.uf_create(self.n)
        if not self._h:
            raise ValueError("uf_create(%d) failed" % n)

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            self._L.uf_destroy(h)
            self._h = None

    def bulk_update(self, edges) -> int:
        """Apply a minibatch of edges; returns the number of skipped (out-of-range) edges."""
        e = _pairs(edges)
        return int(self._L.uf_bulk_update(self._h, e.ctypes.data, e.shape[0]))

    def bulk_query(self, pairs) -> np.ndarray:
        """uint8 answers, 1 iff the pair is connected; out-of-range pairs answer 0."""
        p = _pairs(pairs)
        out = np.empty(p.shape[0], np.uint8)
        self._L.uf_bulk_query(self._h, p.ctypes.data, p.shape[0], out.ctypes.data)
        return out

    def labels(self) -> np.ndarray:
        """int32 label[v] = smallest vertex id in v's component."""
        out = np.empty(self.n, np.int32)
        if self._L.uf_labels(self._h, out.ctypes.data) != 0:
            raise MemoryError("uf_labels")
        return out

    def num_components(self) -> int:
        return int(self._L.uf_num_components(self._h))

    def unions(self) -> int:
        return int(self._L.uf_unions(self._h))

    def invalid(self) -> int:
        return int(self._L.uf_invalid(self._h))

    def count_roots(self) -> int:
        return int(self._L.uf_count_roots(self._h))

    def max_height(self) -> int:
        return int(self._L.uf_max_height(self._h))

    def parents(self) -> np.ndarray:
        out = np.empty(self.n, np.int32)
        self._L.uf_parents(self._h, out.ctypes.data)
        return out
