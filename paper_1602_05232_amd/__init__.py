"""Bulk-parallel incremental graph connectivity on AMD MI355X (gfx950).

Hot path: Bulk-Update and Bulk-Query over a union-find parent array in HBM,
as hand-written HIP kernels behind the C ABI of include/cc.h (libcc.so).
"""
from .cc import QUERY, UPDATE, CCError, Graph, Pool, PreparedOps, lib  # noqa: F401
