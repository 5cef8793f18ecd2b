"""Python binding of libcc.so (include/cc.h): argument marshalling only.

Every step of Bulk-Update, Bulk-Query and the label pass runs in the HIP
kernels of libcc.so; this module only turns torch device tensors into raw
pointers and HIP streams into handles.  There is no fallback: if the library
is not built, importing this module raises.
"""
from __future__ import annotations

import ctypes
import os

import torch  # loads torch's HIP runtime first, so libcc.so binds to the same one

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libcc.so")

CC_OK, CC_EINVAL, CC_ENOMEM, CC_ERANGE, CC_EDEVICE, CC_ECORRUPT = 0, -1, -2, -3, -4, -5
OPT_UPDATE_MODE, OPT_BLOCK, OPT_ITEMS, OPT_QUERY_HALVING = 1, 2, 3, 4
OPT_COMPRESS_EVERY, OPT_HOOK, OPT_GRID_CAP, OPT_COMPRESS_LINKED, OPT_SPIN_LIMIT, OPT_FIND = 5, 6, 7, 8, 9, 10
OPT_ONE_LAUNCH, OPT_FILTER, OPT_QUERY_ITEMS, OPT_SPLIT_BELOW = 11, 12, 13, 14
_OPT_NAMES = {"update_mode": OPT_UPDATE_MODE, "block": OPT_BLOCK, "items": OPT_ITEMS,
              "query_halving": OPT_QUERY_HALVING, "compress_every": OPT_COMPRESS_EVERY,
              "hook": OPT_HOOK, "grid_cap": OPT_GRID_CAP, "compress_linked": OPT_COMPRESS_LINKED,
              "spin_limit": OPT_SPIN_LIMIT, "find": OPT_FIND, "one_launch": OPT_ONE_LAUNCH,
              "filter": OPT_FILTER, "query_items": OPT_QUERY_ITEMS, "split_below": OPT_SPLIT_BELOW}

# Every symbol include/cc.h declares, with (restype, argtypes).
_vp, _i64, _i32 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int
SIGNATURES = {
    "cc_create": (_vp, [_i64]),
    "cc_destroy": (_i32, [_vp]),
    "cc_set_stream": (_i32, [_vp, _vp]),
    "cc_set_option": (_i32, [_vp, _i32, _i64]),
    "cc_get_option": (_i32, [_vp, _i32, ctypes.POINTER(_i64)]),
    "cc_reserve": (_i32, [_vp, _i64]),
    "cc_reset": (_i32, [_vp]),
    "cc_bulk_update": (_i32, [_vp, _vp, _i64]),
    "cc_bulk_update_noalloc": (_i32, [_vp, _vp, _i64]),
    "cc_bulk_query": (_i32, [_vp, _vp, _i64, _vp]),
    "cc_bulk_stream": (_i32, [_vp, _i64, _vp, _vp, _vp, _vp, _vp, _i64]),
    "cc_labels": (_i32, [_vp, _vp]),
    "cc_num_components": (_i32, [_vp, ctypes.POINTER(_i64)]),
    "cc_count_roots": (_i32, [_vp, ctypes.POINTER(_i64)]),
    "cc_filter_state": (_i32, [_vp, ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32), _vp]),
    "cc_sync": (_i32, [_vp]),
    "cc_state_bytes": (_i64, [_vp]),
    "cc_save": (_i32, [_vp, _vp]),
    "cc_load": (_i32, [_vp, _vp]),
    "cc_num_vertices": (_i64, [_vp]),
    "cc_capture_begin": (_i32, [_vp]),
    "cc_capture_end": (_i32, [_vp, ctypes.POINTER(_vp)]),
    "cc_exec_launch": (_i32, [_vp]),
    "cc_exec_destroy": (_i32, [_vp]),
    "cc_strerror": (ctypes.c_char_p, [_i32]),
    "cc_last_error": (ctypes.c_char_p, []),
}

# include/cc_pool.h (many graphs in one arena)
POOL_SIGNATURES = {
    "cc_pool_create": (_vp, [_i64, _i32]),
    "cc_pool_destroy": (_i32, [_vp]),
    "cc_pool_set_stream": (_i32, [_vp, _vp]),
    "cc_pool_set_option": (_i32, [_vp, _i32, _i64]),
    "cc_pool_add": (_i32, [_vp, _i64, ctypes.POINTER(ctypes.c_int32)]),
    "cc_pool_remove": (_i32, [_vp, _i32]),
    "cc_pool_reset": (_i32, [_vp, _i32]),
    "cc_pool_reset_all": (_i32, [_vp]),
    "cc_pool_graph_vertices": (_i64, [_vp, _i32]),
    "cc_pool_free_vertices": (_i64, [_vp]),
    "cc_pool_largest_gap": (_i64, [_vp]),
    "cc_pool_graph_base": (_i64, [_vp, _i32]),
    "cc_pool_gaps": (_i32, [_vp, _vp, _vp, _i32]),
    "cc_pool_run": (_i32, [_vp, _vp, _i32]),
    "cc_pool_labels": (_i32, [_vp, _i32, _vp]),
    "cc_pool_num_components": (_i32, [_vp, _i32, ctypes.POINTER(_i64)]),
    "cc_pool_sync": (_i32, [_vp]),
    "cc_pool_state_bytes": (_i64, [_vp, _i32]),
    "cc_pool_save": (_i32, [_vp, _i32, _vp]),
    "cc_pool_load": (_i32, [_vp, _i32, _vp]),
}


class CcOp(ctypes.Structure):
    """struct cc_op of include/cc_pool.h."""
    _fields_ = [("graph", ctypes.c_int32), ("kind", ctypes.c_int32), ("count", ctypes.c_int64),
                ("items", ctypes.c_void_p), ("out", ctypes.c_void_p)]


UPDATE, QUERY = 0, 1

# include/cc_bench.h (memory-system microbenchmarks for roofline denominators)
BENCH_SIGNATURES = {
    "ccb_gather": (_i32, [_vp, _i64, _i64, ctypes.c_uint32, _vp, _vp]),
    "ccb_stream_read": (_i32, [_vp, _i64, _vp, _vp]),
    "ccb_copy": (_i32, [_vp, _vp, _i64, _vp]),
    "ccb_cas": (_i32, [_vp, _i64, _i64, ctypes.c_uint32, _vp]),
    "ccb_event_create": (_i32, [_vp]),
    "ccb_event_record": (_i32, [_vp, _vp]),
    "ccb_event_elapsed_ms": (_i32, [_vp, _vp, _vp]),
    "ccb_event_destroy": (_i32, [_vp]),
}


class CCError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__("%s (%d): %s" % (_name(code), code, msg))
        self.code = code


def _name(code):
    return {0: "CC_OK", -1: "CC_EINVAL", -2: "CC_ENOMEM", -3: "CC_ERANGE", -4: "CC_EDEVICE",
            -5: "CC_ECORRUPT"}.get(code, "CC_?")


def load_library(path: str = LIB_PATH, declare=None):
    declare = declare if declare is not None else {**SIGNATURES, **POOL_SIGNATURES, **BENCH_SIGNATURES}
    if not os.path.exists(path):
        raise ImportError("%s is not built; run __graft_entry__.build() first" % path)
    L = ctypes.CDLL(path)
    for name, (res, args) in declare.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    return L


_lib = None


def lib():
    global _lib
    if _lib is None:
        _lib = load_library()
    return _lib


def _check(rc: int):
    if rc != CC_OK:
        raise CCError(rc, lib().cc_last_error().decode(errors="replace"))
    return rc


def _pairs_ptr(t: torch.Tensor, what: str) -> int:
    if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == torch.int32):
        raise TypeError("%s must be a CUDA int32 tensor" % what)
    if t.numel() and not (t.dim() == 2 and t.shape[1] == 2 and t.is_contiguous()):
        raise ValueError("%s must be a contiguous [k, 2] tensor" % what)
    if t.numel() and t.data_ptr() % 8:
        raise ValueError("%s must start on an 8-byte boundary (one pair per 8-byte load)" % what)
    return t.data_ptr()


def stream_handle(stream) -> int:
    if stream is None:
        stream = torch.cuda.current_stream()
    return int(stream.cuda_stream)


class Graph:
    """A union-find forest over vertices [0, n) in device memory.

    Calls are asynchronous and ordered on `stream` (default: the current
    torch stream at construction)."""

    def __init__(self, n: int, stream=None, **options):
        self._h = None
        L = lib()
        h = L.cc_create(int(n))
        if not h:
            raise CCError(CC_EINVAL, L.cc_last_error().decode(errors="replace"))
        self._h = h
        self.n = int(n)
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        _check(L.cc_set_stream(h, stream_handle(self.stream)))
        for k, v in options.items():
            self.set_option(k, v)

    def close(self):
        if self._h:
            lib().cc_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def handle(self) -> int:
        return self._h

    def set_option(self, key, value: int):
        k = _OPT_NAMES[key] if isinstance(key, str) else int(key)
        _check(lib().cc_set_option(self._h, k, int(value)))

    def get_option(self, key) -> int:
        k = _OPT_NAMES[key] if isinstance(key, str) else int(key)
        v = ctypes.c_int64()
        _check(lib().cc_get_option(self._h, k, ctypes.byref(v)))
        return v.value

    def reserve(self, max_batch: int):
        _check(lib().cc_reserve(self._h, int(max_batch)))

    def reset(self):
        _check(lib().cc_reset(self._h))

    def bulk_update(self, edges: torch.Tensor):
        p = _pairs_ptr(edges, "edges")
        _check(lib().cc_bulk_update(self._h, p, edges.shape[0] if edges.numel() else 0))

    def bulk_update_noalloc(self, edges: torch.Tensor):
        """Bulk-Update through cc_bulk_update_noalloc (no device allocation;
        at most 2^22 edges per call)."""
        p = _pairs_ptr(edges, "edges")
        _check(lib().cc_bulk_update_noalloc(self._h, p, edges.shape[0] if edges.numel() else 0))

    def bulk_query(self, pairs: torch.Tensor, out: torch.Tensor | None = None) -> torch.Tensor:
        p = _pairs_ptr(pairs, "pairs")
        q = pairs.shape[0] if pairs.numel() else 0
        if out is None:
            out = torch.empty(q, dtype=torch.uint8, device=pairs.device)
        assert out.dtype == torch.uint8 and out.is_cuda and out.numel() >= q and out.is_contiguous()
        _check(lib().cc_bulk_query(self._h, p, q, out.data_ptr()))
        return out

    def bulk_stream(self, edges: torch.Tensor, eoff: torch.Tensor, pairs: torch.Tensor, qoff: torch.Tensor,
                    out: torch.Tensor, max_items: int | None = None):
        """Every (update k, query k) of a stream in one launch; eoff/qoff are
        CUDA int64 offsets (length batches + 1) into edges/pairs."""
        for t, name in ((eoff, "eoff"), (qoff, "qoff")):
            if not (t.is_cuda and t.dtype == torch.int64 and t.dim() == 1 and t.is_contiguous()):
                raise TypeError("%s must be a contiguous CUDA int64 vector" % name)
        batches = eoff.numel() - 1
        assert qoff.numel() == batches + 1 and out.dtype == torch.uint8 and out.is_cuda
        if max_items is None:
            max_items = int(max(torch.diff(eoff).max().item(), torch.diff(qoff).max().item(), 1))
        _check(lib().cc_bulk_stream(self._h, batches, _pairs_ptr(edges, "edges"), eoff.data_ptr(),
                                    _pairs_ptr(pairs, "pairs"), qoff.data_ptr(), out.data_ptr(), int(max_items)))

    def labels(self, out: torch.Tensor | None = None) -> torch.Tensor:
        if out is None:
            out = torch.empty(self.n, dtype=torch.int32, device="cuda")
        assert out.dtype == torch.int32 and out.is_cuda and out.numel() >= self.n and out.is_contiguous()
        _check(lib().cc_labels(self._h, out.data_ptr()))
        return out

    def num_components(self) -> int:
        v = ctypes.c_int64()
        _check(lib().cc_num_components(self._h, ctypes.byref(v)))
        return v.value

    def count_roots(self) -> int:
        v = ctypes.c_int64()
        _check(lib().cc_count_roots(self._h, ctypes.byref(v)))
        return v.value

    def filter_state(self):
        """(anchor, touched_complete, membership bitmap, touched bitmap) of the
        membership filter, the bitmaps as numpy uint32 arrays of ceil(n/32)
        words; waits for the stream."""
        import numpy as np
        a, c = ctypes.c_int32(), ctypes.c_int32()
        w = (self.n + 31) // 32
        bits = np.zeros(2 * w, np.uint32)
        _check(lib().cc_filter_state(self._h, ctypes.byref(a), ctypes.byref(c), bits.ctypes.data))
        return a.value, bool(c.value), bits[:w], bits[w:]

    def sync(self) -> int:
        """Wait for the stream; returns CC_OK, CC_ERANGE or CC_ECORRUPT
        (latched since the last sync) and raises on a device error."""
        rc = lib().cc_sync(self._h)
        if rc in (CC_OK, CC_ERANGE, CC_ECORRUPT):
            return rc
        return _check(rc)

    def capture(self):
        """Context manager: calls on this graph inside the block are recorded
        into a replayable sequence (the returned Recording after exit)."""
        return _Capture(self)

    def save(self) -> bytearray:
        buf = bytearray(int(lib().cc_state_bytes(self._h)))
        cbuf = (ctypes.c_char * len(buf)).from_buffer(buf)
        _check(lib().cc_save(self._h, ctypes.addressof(cbuf)))
        return buf

    def load(self, buf) -> None:
        buf = bytearray(buf)
        cbuf = (ctypes.c_char * len(buf)).from_buffer(buf)
        if len(buf) != lib().cc_state_bytes(self._h):
            raise CCError(CC_EINVAL, "state image has the wrong size")
        _check(lib().cc_load(self._h, ctypes.addressof(cbuf)))


class Recording:
    """A captured sequence of calls on one graph (cc_exec)."""

    def __init__(self, h):
        self._h = h

    def launch(self):
        _check(lib().cc_exec_launch(self._h))

    def close(self):
        if self._h:
            lib().cc_exec_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class _Capture:
    def __init__(self, g: Graph):
        self.g = g
        self.recording = None

    def __enter__(self):
        _check(lib().cc_capture_begin(self.g.handle))
        return self

    def __exit__(self, et, ev, tb):
        x = ctypes.c_void_p()
        rc = lib().cc_capture_end(self.g.handle, ctypes.byref(x))
        if et is None:
            _check(rc)
            self.recording = Recording(x.value)
        elif rc == CC_OK:
            lib().cc_exec_destroy(x.value)
        return False


class PreparedOps:
    """An operation list for Pool.run as the cc_op array of cc_pool_run.  It
    keeps the item and output tensors alive; their contents may change
    between runs, their storage must not."""

    def __init__(self, ops):
        ops = list(ops)
        arr = (CcOp * max(1, len(ops)))()
        keep = []
        for i, (gid, kind, items, out) in enumerate(ops):
            cnt = items.shape[0] if items is not None and items.numel() else 0
            arr[i].graph = int(gid)
            arr[i].kind = int(kind)
            arr[i].count = cnt
            arr[i].items = _pairs_ptr(items, "items") if cnt else None
            if kind == QUERY and cnt:
                assert out is not None and out.dtype == torch.uint8 and out.is_cuda and out.numel() >= cnt
                arr[i].out = out.data_ptr()
            else:
                arr[i].out = None
            keep.append((items, out))
        self.array, self.count, self._keep = arr, len(ops), keep


class Pool:
    """Many independent graphs in one device arena (include/cc_pool.h).

    run() takes a list of (graph, kind, items, out) with kind UPDATE (items =
    int32 [k, 2] edges, out None) or QUERY (items = pairs, out = uint8 [k]);
    operations on one graph apply in list order, one launch per round."""

    def __init__(self, capacity: int, max_graphs: int, stream=None, **options):
        self._h = None
        L = lib()
        h = L.cc_pool_create(int(capacity), int(max_graphs))
        if not h:
            raise CCError(CC_ENOMEM, L.cc_last_error().decode(errors="replace"))
        self._h = h
        self.capacity = int(capacity)
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        _check(L.cc_pool_set_stream(h, stream_handle(self.stream)))
        for k, v in options.items():
            self.set_option(k, v)

    def close(self):
        if self._h:
            lib().cc_pool_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_stream(self, stream):
        self.stream = stream
        _check(lib().cc_pool_set_stream(self._h, stream_handle(stream)))

    def set_option(self, key, value: int):
        k = _OPT_NAMES[key] if isinstance(key, str) else int(key)
        _check(lib().cc_pool_set_option(self._h, k, int(value)))

    def add(self, n: int) -> int:
        gid = ctypes.c_int32()
        _check(lib().cc_pool_add(self._h, int(n), ctypes.byref(gid)))
        return gid.value

    def remove(self, gid: int):
        _check(lib().cc_pool_remove(self._h, int(gid)))

    def reset(self, gid: int):
        _check(lib().cc_pool_reset(self._h, int(gid)))

    def reset_all(self):
        _check(lib().cc_pool_reset_all(self._h))

    def vertices(self, gid: int) -> int:
        return int(lib().cc_pool_graph_vertices(self._h, int(gid)))

    def free_vertices(self) -> int:
        return int(lib().cc_pool_free_vertices(self._h))

    def largest_gap(self) -> int:
        return int(lib().cc_pool_largest_gap(self._h))

    def gaps(self):
        """Free ranges as (base, length), ascending."""
        k = int(lib().cc_pool_gaps(self._h, None, None, 0))
        b = (ctypes.c_int64 * max(1, k))()
        ln = (ctypes.c_int64 * max(1, k))()
        lib().cc_pool_gaps(self._h, b, ln, k)
        return [(b[i], ln[i]) for i in range(k)]

    def gaps_after_removing(self, gids):
        """Lengths of the free ranges if the graphs `gids` were removed."""
        ranges = sorted(self.gaps() + [(int(lib().cc_pool_graph_base(self._h, int(g))), self.vertices(g))
                                       for g in gids])
        merged = []
        for b, ln in ranges:
            if merged and merged[-1][0] + merged[-1][1] == b:
                merged[-1] = (merged[-1][0], merged[-1][1] + ln)
            else:
                merged.append((b, ln))
        return [ln for _, ln in merged]

    @staticmethod
    def prepare(ops) -> "PreparedOps":
        """Marshal an operation list once, for runs that repeat it."""
        return PreparedOps(ops)

    def run(self, ops):
        """One cc_pool_run over ops: a list of (graph, kind, items, out) or a
        PreparedOps."""
        p = ops if isinstance(ops, PreparedOps) else PreparedOps(ops)
        _check(lib().cc_pool_run(self._h, p.array, p.count))

    def labels(self, gid: int, out: torch.Tensor | None = None) -> torch.Tensor:
        n = self.vertices(gid)
        if out is None:
            out = torch.empty(n, dtype=torch.int32, device="cuda")
        _check(lib().cc_pool_labels(self._h, int(gid), out.data_ptr()))
        return out

    def num_components(self, gid: int) -> int:
        v = ctypes.c_int64()
        _check(lib().cc_pool_num_components(self._h, int(gid), ctypes.byref(v)))
        return v.value

    def sync(self) -> int:
        rc = lib().cc_pool_sync(self._h)
        if rc in (CC_OK, CC_ERANGE, CC_ECORRUPT):
            return rc
        return _check(rc)

    def save(self, gid: int) -> bytearray:
        buf = bytearray(int(lib().cc_pool_state_bytes(self._h, int(gid))))
        cbuf = (ctypes.c_char * len(buf)).from_buffer(buf)
        _check(lib().cc_pool_save(self._h, int(gid), ctypes.addressof(cbuf)))
        return buf

    def load(self, gid: int, buf):
        buf = bytearray(buf)
        if len(buf) != lib().cc_pool_state_bytes(self._h, int(gid)):
            raise CCError(CC_EINVAL, "state image has the wrong size")
        cbuf = (ctypes.c_char * len(buf)).from_buffer(buf)
        _check(lib().cc_pool_load(self._h, int(gid), ctypes.addressof(cbuf)))
