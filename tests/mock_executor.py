"""A CPU executor for the serving scheduler: applies each round through one
oracle per stream and completes it on a simulated clock (launch cost plus a
per-item cost), so the scheduler's admission, eviction, ordering and batching
can be tested without a GPU."""
import numpy as np

import oracle


class OracleExecutor:
    def __init__(self, budget, launch_cost=5e-6, item_cost=1e-9):
        self.t = 0.0
        self.budget = budget
        self.used = 0
        self.launch_cost = launch_cost
        self.item_cost = item_cost
        self.state = {}      # stream -> UnionFind (resident)
        self.evicted = {}    # stream -> UnionFind kept aside (its state image)
        self.images = {}     # stream -> parent array from a checkpoint, loaded when admitted
        self.nsize = {}
        self.done = {}       # handle -> completion time
        self.next_handle = 0
        self.max_concurrent = 0
        self.log = []        # (stream, kind, launch time)

    # clock
    def now(self):
        return self.t

    def idle_wait(self, until):
        cands = [d for d in self.done.values() if d > self.t]
        if until is not None and until > self.t:
            cands.append(until)
        self.t = min(cands) if cands else self.t + 1e-6

    # residency
    def resident(self, s):
        return s in self.state

    def resident_streams(self):
        return list(self.state)

    def can_admit(self, n):
        return self.used + n <= self.budget

    def can_admit_after(self, n, victims):
        return self.used - sum(self.nsize[v] for v in victims) + n <= self.budget

    def admit(self, s, n):
        assert self.can_admit(n)
        self.used += n
        self.nsize[s] = n
        if s in self.evicted:
            self.state[s] = self.evicted.pop(s)
        elif s in self.images:
            self.state[s] = self._from_image(self.images.pop(s))
        else:
            self.state[s] = oracle.UnionFind(n)

    # checkpoint / restore: an image is a stream's parent array; restoring
    # rebuilds a union-find with the same components from its edges (v, parent[v])
    def checkpoint(self):
        out = {s: img.copy() for s, img in self.images.items()}
        for s, uf in list(self.state.items()) + list(self.evicted.items()):
            out[s] = uf.parents()
        return out

    def restore(self, images):
        self.images.update({s: np.asarray(img, np.int32).copy() for s, img in images.items()})

    @staticmethod
    def _from_image(img):
        uf = oracle.UnionFind(len(img))
        uf.bulk_update(np.stack([np.arange(len(img), dtype=np.int32), img], 1))
        return uf

    def evict(self, s):
        self.evicted[s] = self.state.pop(s)
        self.used -= self.nsize[s]

    # work
    def launch(self, ops):
        busy = sum(1 for d in self.done.values() if d > self.t)
        self.max_concurrent = max(self.max_concurrent, busy + 1)
        items = 0
        for s, kind, arr, out in ops:
            uf = self.state[s]
            if kind == 0:
                uf.bulk_update(arr)
            else:
                out[:] = uf.bulk_query(arr)
            items += len(arr)
            self.log.append((s, kind, self.t))
        h = self.next_handle
        self.next_handle += 1
        self.done[h] = self.t + self.launch_cost + self.item_cost * items
        return h

    def poll(self, h):
        return self.t >= self.done[h]
