"""Measured roofline denominators for the connectivity kernels.

Thin wrappers over include/cc_bench.h, timed with HIP events on the current
torch stream:
  G(N)  random 4-byte gathers per second from an N-entry int32 table,
  B_s   streaming read bandwidth (bytes/s),
  C     random device-scope compare-and-swaps per second.
The per-edge Bulk-Update bound is E_roof = 1 / (2/G + 8/B_s): two random
parent reads (one find per endpoint at depth one) plus 8 streamed bytes.
"""
from __future__ import annotations

import ctypes

import torch

from .cc import lib, stream_handle


def _time(fn, reps=3):
    s = torch.cuda.current_stream()
    best = None
    for _ in range(reps + 1):  # first call warms up
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(s)
        fn()
        b.record(s)
        b.synchronize()
        t = a.elapsed_time(b) / 1e3
        best = t if best is None else min(best, t)
    return best


def gather_rate(n_table: int, count: int = 1 << 28, table: torch.Tensor | None = None) -> float:
    """Random 4-byte gathers per second from an n_table-entry table."""
    t = table if table is not None else torch.arange(n_table, dtype=torch.int32, device="cuda")
    sink = torch.zeros(1, dtype=torch.int32, device="cuda")
    h = stream_handle(None)

    def run():
        rc = lib().ccb_gather(t.data_ptr(), n_table, count, 0x1234567, sink.data_ptr(), h)
        assert rc == 0, rc
    return count / _time(run)


def stream_bandwidth(nbytes: int = 1 << 31) -> float:
    buf = torch.ones(nbytes // 4, dtype=torch.int32, device="cuda")
    sink = torch.zeros(1, dtype=torch.int32, device="cuda")
    h = stream_handle(None)

    def run():
        assert lib().ccb_stream_read(buf.data_ptr(), nbytes, sink.data_ptr(), h) == 0
    t = _time(run)
    del buf
    return nbytes / t


def cas_rate(n_table: int, count: int = 1 << 26) -> float:
    t = torch.arange(n_table, dtype=torch.int32, device="cuda")
    h = stream_handle(None)

    def run():
        assert lib().ccb_cas(t.data_ptr(), n_table, count, 0x7654321, h) == 0
    return count / _time(run)


class TimingEvent:
    """A HIP event for timing only (created by ccb_event_create, without the
    system-scope fence of a default event), recorded on a torch stream.
    elapsed_time(stop) returns milliseconds, as torch.cuda.Event does."""

    def __init__(self):
        h = ctypes.c_void_p()
        rc = lib().ccb_event_create(ctypes.byref(h))
        if rc != 0:
            raise RuntimeError("ccb_event_create failed (%d)" % rc)
        self.handle = h.value

    def record(self, stream=None):
        rc = lib().ccb_event_record(self.handle, stream_handle(stream))
        if rc != 0:
            raise RuntimeError("ccb_event_record failed (%d)" % rc)

    def elapsed_time(self, stop: "TimingEvent") -> float:
        ms = ctypes.c_float()
        rc = lib().ccb_event_elapsed_ms(self.handle, stop.handle, ctypes.byref(ms))
        if rc != 0:
            raise RuntimeError("ccb_event_elapsed_ms failed (%d)" % rc)
        return ms.value

    def close(self):
        """Release the event now (before interpreter shutdown, when the
        runtime may already be tearing down)."""
        h, self.handle = getattr(self, "handle", None), None
        if h:
            lib().ccb_event_destroy(h)

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def copy_bytes(dst: torch.Tensor, src: torch.Tensor, nbytes: int):
    assert lib().ccb_copy(dst.data_ptr(), src.data_ptr(), nbytes, stream_handle(None)) == 0


def edge_roofline(G: float, Bs: float) -> float:
    """Bulk-Update edges/s bound: 2 random parent reads + 8 streamed bytes per edge."""
    return 1.0 / (2.0 / G + 8.0 / Bs)


def _main():
    """Command line: `python -m paper_1602_05232_amd.roofline copy [bytes]` runs
    one plain copy kernel of known size (the reference point for traffic
    counters); `... gather [log2 table]` prints G for one table size."""
    import sys
    what = sys.argv[1] if len(sys.argv) > 1 else "gather"
    if what == "copy":
        nbytes = int(sys.argv[2]) if len(sys.argv) > 2 else 1 << 30
        src = torch.ones(nbytes // 4, dtype=torch.int32, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        copy_bytes(dst, src, nbytes)
        torch.cuda.synchronize()
        assert torch.equal(src, dst)
        print("copied %d bytes with one ccb_copy launch" % nbytes, flush=True)
    else:
        lg = int(sys.argv[2]) if len(sys.argv) > 2 else 24
        print("G(2^%d) = %.4g gathers/s" % (lg, gather_rate(1 << lg)), flush=True)


if __name__ == "__main__":
    _main()
