"""Serving loop: continuous batching of Bulk-Update / Bulk-Query requests over
many resident graph streams.

Requests arrive over time, each for one graph stream.  The loop keeps one
FIFO per stream and at most one operation per stream on the device, which
keeps the rule that a bulk operation completes before the next begins
(Section 1, Model) per stream; each query therefore sees exactly the updates
that arrived before it on its stream, alone or in any mix.  Whenever a launch
slot is free, the heads of all idle streams that have work are packed into one
pool round (one kernel for many graphs, include/cc_pool.h) on the next HIP
stream, so rounds overlap on the device and requests that arrive while others
run join the next round (continuous batching, not a queue in front of a
serial server).  Graph state lives in a pool arena under a memory budget;
streams are admitted as room frees up and idle streams are evicted (state
saved to host, restored on return) when it does not.

The executor is pluggable: GpuExecutor runs the pool on the device;
tests drive the same scheduler with a CPU executor built on the oracle.
"""
from __future__ import annotations

import collections
import dataclasses
import time

import numpy as np

UPDATE, QUERY = 0, 1


@dataclasses.dataclass
class Request:
    rid: int
    stream: int
    kind: int           # UPDATE or QUERY
    arrival: float      # seconds, trace time
    items: object       # edges or pairs (executor-specific array/tensor, [k, 2])
    out: object = None  # query answers buffer (executor-specific)
    size: int = 0
    done_at: float = None

    @property
    def latency(self):
        return None if self.done_at is None else self.done_at - self.arrival


class Scheduler:
    """Continuous-batching request loop.

    executor: admit(stream, n) / evict(stream) / resident(stream) /
    free_vertices() / launch(list of (stream, kind, items, out)) -> handle /
    poll(handle) -> bool / now() -> float / idle_wait().
    """

    def __init__(self, executor, stream_sizes, max_inflight=2, max_items_per_round=1 << 26,
                 max_requests_per_round=1 << 30):
        self.ex = executor
        self.sizes = list(stream_sizes)
        self.max_inflight = max_inflight
        self.max_items = max_items_per_round
        self.max_reqs = max_requests_per_round
        self.fifo = collections.defaultdict(collections.deque)
        self.busy = set()
        self.inflight = []          # (handle, [requests])
        self.last_use = {}          # stream -> round counter (for LRU eviction)
        self.rounds = 0
        self.round_sizes = []
        self.evictions = 0
        self.admissions = 0

    def _make_room(self, s, allow_waiting_victims):
        """Make stream s resident.  Idle streams are evicted to make room:
        first those with no queued work, least recently used first; streams
        that still have queued requests only if `allow_waiting_victims`.
        Returns False if it cannot right now (nothing is changed then)."""
        if self.ex.resident(s):
            return True
        need = self.sizes[s]
        idle = [t for t in self.ex.resident_streams() if t not in self.busy and t != s]
        idle.sort(key=lambda t: (len(self.fifo[t]) > 0, self.last_use.get(t, -1)))
        if not allow_waiting_victims:
            idle = [t for t in idle if not self.fifo[t]]
        plan = []
        while not self.ex.can_admit_after(need, plan):
            if not idle:
                return False
            plan.append(idle.pop(0))
        for victim in plan:
            self.ex.evict(victim)
            self.evictions += 1
        self.ex.admit(s, need)
        self.admissions += 1
        return True

    def _complete(self):
        still = []
        for h, reqs in self.inflight:
            if self.ex.poll(h):
                t = self.ex.now()
                for r in reqs:
                    r.done_at = t
                    self.busy.discard(r.stream)
            else:
                still.append((h, reqs))
        self.inflight = still

    def _launch_round(self):
        ready = [s for s, q in self.fifo.items() if q and s not in self.busy]
        if not ready:
            return False
        # resident streams first (no transfer), each group oldest head first
        ready.sort(key=lambda s: (not self.ex.resident(s), self.fifo[s][0].arrival))
        picked, items = [], 0
        for s in ready:
            if len(picked) >= self.max_reqs:
                break
            r = self.fifo[s][0]
            if picked and items + r.size > self.max_items:
                continue
            # evicting a stream that has queued work only pays when nothing else can run
            if not self._make_room(s, allow_waiting_victims=not picked and not self.inflight):
                continue
            self.fifo[s].popleft()
            picked.append(r)
            items += r.size
            self.busy.add(s)
            self.last_use[s] = self.rounds
        if not picked:
            return False
        h = self.ex.launch([(r.stream, r.kind, r.items, r.out) for r in picked])
        self.inflight.append((h, picked))
        self.rounds += 1
        self.round_sizes.append(len(picked))
        return True

    def run(self, requests):
        """Serve `requests` (sorted by arrival); returns them with done_at set."""
        reqs = sorted(requests, key=lambda r: r.arrival)
        i = 0
        t0 = self.ex.now()
        while i < len(reqs) or self.inflight or any(self.fifo.values()):
            now = self.ex.now() - t0
            while i < len(reqs) and reqs[i].arrival <= now:
                self.fifo[reqs[i].stream].append(reqs[i])
                i += 1
            self._complete()
            launched = False
            while len(self.inflight) < self.max_inflight and self._launch_round():
                launched = True
            if not launched:
                nxt = reqs[i].arrival + t0 if i < len(reqs) else None
                self.ex.idle_wait(nxt)
        for r in reqs:
            r.done_at -= t0
        return reqs


class SerialScheduler(Scheduler):
    """The plain baseline: one request per launch, one launch at a time, in
    arrival order (a FIFO in front of a serial server)."""

    def __init__(self, executor, stream_sizes):
        super().__init__(executor, stream_sizes, max_inflight=1, max_requests_per_round=1)

    def _launch_round(self):
        ready = [s for s, q in self.fifo.items() if q and s not in self.busy]
        if not ready:
            return False
        s = min(ready, key=lambda t: self.fifo[t][0].arrival)
        if not self._make_room(s, allow_waiting_victims=True):
            return False
        r = self.fifo[s].popleft()
        self.busy.add(s)
        self.last_use[s] = self.rounds
        self.inflight.append((self.ex.launch([(r.stream, r.kind, r.items, r.out)]), [r]))
        self.rounds += 1
        self.round_sizes.append(1)
        return True


def serial_scheduler(executor, stream_sizes):
    return SerialScheduler(executor, stream_sizes)


class GpuExecutor:
    """Runs rounds on a cc_pool with `nstreams` HIP streams in rotation;
    admission and eviction run on a separate stream and wait for it."""

    def __init__(self, budget_vertices, max_graphs, nstreams=2, **options):
        import torch

        from .cc import Pool
        self.torch = torch
        self.pool = Pool(budget_vertices, max_graphs, **options)
        self.streams = [torch.cuda.Stream() for _ in range(nstreams)]
        self.admin = torch.cuda.Stream()
        self.next = 0
        self.gid = {}      # stream -> pool graph id
        self.images = {}   # stream -> host state image of an evicted graph
        self.sizes = {}

    def now(self):
        return time.perf_counter()

    def idle_wait(self, until):
        pass  # spin: completion is detected by polling events

    def resident(self, s):
        return s in self.gid

    def resident_streams(self):
        return list(self.gid)

    def can_admit(self, n):
        return self.pool.largest_gap() >= n

    def can_admit_after(self, n, victims):
        """Would a graph of n vertices fit once `victims` are evicted?"""
        if not victims:
            return self.can_admit(n)
        gaps = self.pool.gaps_after_removing([self.gid[v] for v in victims])
        return max(gaps, default=0) >= n

    def admit(self, s, n):
        # the entries taken belonged to graphs with no work left in flight
        self.pool.set_stream(self.admin)
        self.gid[s] = self.pool.add(n)
        self.sizes[s] = n
        if s in self.images:
            self.pool.load(self.gid[s], self.images.pop(s))
        self.admin.synchronize()  # initialised before any round on another stream

    def evict(self, s):
        # only idle streams are evicted: their last round has completed
        self.pool.set_stream(self.admin)
        gid = self.gid.pop(s)
        self.images[s] = self.pool.save(gid)
        self.pool.remove(gid)

    def checkpoint(self):
        """State images of every stream seen so far (resident ones are saved
        from the pool, evicted ones are already images).  Call when nothing
        is in flight."""
        self.torch.cuda.synchronize()
        out = dict(self.images)
        self.pool.set_stream(self.admin)
        for s, gid in self.gid.items():
            out[s] = self.pool.save(gid)
        return out

    def restore(self, images):
        """Take over the images of a checkpoint: each stream is loaded from
        its image when it is next admitted."""
        self.images.update(images)

    def launch(self, ops):
        st = self.streams[self.next]
        self.next = (self.next + 1) % len(self.streams)
        self.pool.set_stream(st)
        self.pool.run([(self.gid[s], k, items, out) for s, k, items, out in ops])
        ev = self.torch.cuda.Event()
        ev.record(st)
        return ev

    def poll(self, ev):
        return ev.query()

    def close(self):
        self.pool.close()


def latency_summary(reqs):
    lat = np.array([r.latency for r in reqs if r.latency is not None])
    if lat.size == 0:
        return {}
    return {"p50_ms": float(np.percentile(lat, 50) * 1e3), "p99_ms": float(np.percentile(lat, 99) * 1e3),
            "mean_ms": float(lat.mean() * 1e3), "max_ms": float(lat.max() * 1e3)}
