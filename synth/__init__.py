"""Seeded synthetic graph streams (inputs only; no connectivity arithmetic).

Both sides of every parity check -- the CPU oracle and the GPU library -- take
their inputs from this module.  It wraps the counter-based C generators in
``streamgen.c`` (splitmix64 keyed by (seed, stream, purpose, index)) and builds
the five workload recipes: uniform random, R-MAT power-law, many independent
graphs, a high-diameter mesh and a serving trace.  The shapes follow the
paper's evaluation datasets (Section 6.2, Table 1) scaled to one GPU.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "streamgen.c")
_LIB = os.path.join(_HERE, "libsynth.so")

BASE_SEED = 0x16020523

# purpose codes of the named random streams
P_EDGES, P_QUERIES, P_SIZES, P_PERM, P_PROBES, P_SHUFFLE, P_LONGRANGE = 1, 2, 3, 4, 5, 6, 7
P_GRAPH_N, P_CUTS, P_ARRIVALS, P_REQ_STREAM, P_REQ_TYPE, P_REQ_SIZE = 8, 9, 10, 11, 12, 13

RMAT_ABC = (0.57, 0.19, 0.19)


def build_lib(force: bool = False) -> str:
    """Compile streamgen.c into libsynth.so (gcc, OpenMP)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O3", "-fopenmp", "-fPIC", "-shared", "-std=c11",
                               "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build_lib()
        L = ctypes.CDLL(_LIB)
        u64, i64, i32, dbl, vp = (ctypes.c_uint64, ctypes.c_int64, ctypes.c_int,
                                  ctypes.c_double, ctypes.c_void_p)
        L.sg_key.restype = u64
        L.sg_key.argtypes = [u64, u64, u64]
        L.sg_draw.restype = u64
        L.sg_draw.argtypes = [u64, u64]
        L.sg_draws.argtypes = [u64, i64, i64, vp]
        L.sg_unit_doubles.argtypes = [u64, i64, i64, vp]
        L.sg_uniform_pairs.argtypes = [u64, i64, i64, i64, vp]
        L.sg_rmat_edges.argtypes = [u64, i64, i64, i32, dbl, dbl, dbl, i64, vp, vp]
        L.sg_permutation.argtypes = [u64, i64, vp]
        L.sg_shuffle_pairs.argtypes = [u64, i64, vp]
        L.sg_grid_edge_count.restype = i64
        L.sg_grid_edge_count.argtypes = [i64, i64]
        L.sg_grid_stream.restype = i64
        L.sg_grid_stream.argtypes = [i64, i64, i64, u64, u64, vp]
        L.sg_apply_perm.argtypes = [vp, i64, vp]
        L.sg_grid3d_edge_count.restype = i64
        L.sg_grid3d_edge_count.argtypes = [i64]
        L.sg_grid3d_stream.restype = i64
        L.sg_grid3d_stream.argtypes = [i64, u64, vp]
        L.sg_local_pairs.argtypes = [u64, i64, i64, i64, dbl, vp]
        L.sg_lognormal_counts.argtypes = [u64, i64, dbl, dbl, i64, i64, vp]
        L.sg_poisson_arrivals.argtypes = [u64, i64, dbl, vp]
        _lib = L
    return _lib


def _ptr(a) -> int:
    if isinstance(a, np.ndarray):
        assert a.flags["C_CONTIGUOUS"]
        return a.ctypes.data
    return int(a.data_ptr())  # a CPU torch tensor


def key(seed: int, stream: int, purpose: int) -> int:
    return int(lib().sg_key(seed & (2**64 - 1), stream, purpose))


def draws(k: int, start: int, count: int) -> np.ndarray:
    out = np.empty(count, np.uint64)
    lib().sg_draws(k, start, count, _ptr(out))
    return out


def unit_doubles(k: int, start: int, count: int) -> np.ndarray:
    out = np.empty(count, np.float64)
    lib().sg_unit_doubles(k, start, count, _ptr(out))
    return out


def uniform_pairs(k: int, start: int, count: int, n: int, out=None) -> np.ndarray:
    if out is None:
        out = np.empty((count, 2), np.int32)
    lib().sg_uniform_pairs(k, start, count, n, _ptr(out))
    return out


def permutation(k: int, n: int) -> np.ndarray:
    out = np.empty(n, np.int32)
    lib().sg_permutation(k, n, _ptr(out))
    return out


def rmat_edges(k: int, start: int, count: int, scale: int, n: int, perm=None,
               abc=RMAT_ABC, out=None) -> np.ndarray:
    if out is None:
        out = np.empty((count, 2), np.int32)
    p = None if perm is None else _ptr(perm)
    lib().sg_rmat_edges(k, start, count, scale, abc[0], abc[1], abc[2], n, p, _ptr(out))
    return out


def shuffle_pairs(k: int, pairs: np.ndarray) -> np.ndarray:
    lib().sg_shuffle_pairs(k, pairs.shape[0], _ptr(pairs))
    return pairs


def grid_stream(W: int, H: int, extra: int, lkey: int, skey: int) -> np.ndarray:
    cnt = int(lib().sg_grid_edge_count(W, H)) + extra
    out = np.empty((cnt, 2), np.int32)
    got = lib().sg_grid_stream(W, H, extra, lkey, skey, _ptr(out))
    assert got == cnt
    return out


def grid3d_edges(L: int, skey: int) -> np.ndarray:
    cnt = int(lib().sg_grid3d_edge_count(L))
    out = np.empty((cnt, 2), np.int32)
    assert lib().sg_grid3d_stream(L, skey, _ptr(out)) == cnt
    return out


def local_pairs(k: int, start: int, count: int, n: int, window: int, out=None) -> np.ndarray:
    if out is None:
        out = np.empty((count, 2), np.int32)
    lib().sg_local_pairs(k, start, count, n, float(np.log2(max(2, window))), _ptr(out))
    return out


def lognormal_counts(k: int, count: int, mu: float, sigma: float, lo: int, hi: int) -> np.ndarray:
    out = np.empty(count, np.int64)
    lib().sg_lognormal_counts(k, count, mu, sigma, lo, hi, _ptr(out))
    return out


def poisson_arrivals(k: int, count: int, lam: float) -> np.ndarray:
    out = np.empty(count, np.float64)
    lib().sg_poisson_arrivals(k, count, lam, _ptr(out))
    return out


# ---------------------------------------------------------------------------
# Stream recipes
# ---------------------------------------------------------------------------

@dataclass
class Stream:
    """One graph stream: minibatch i is edges[eoff[i]:eoff[i+1]], and the query
    batch that follows it is queries[qoff[i]:qoff[i+1]].  `probes` is a fixed
    pair set asked after every minibatch (answers may only go 0 -> 1)."""
    name: str
    n: int
    edges: np.ndarray
    eoff: np.ndarray
    queries: np.ndarray
    qoff: np.ndarray
    probes: np.ndarray = field(default_factory=lambda: np.empty((0, 2), np.int32))
    meta: dict = field(default_factory=dict)

    @property
    def num_batches(self) -> int:
        return len(self.eoff) - 1

    def batch(self, i: int) -> np.ndarray:
        return self.edges[self.eoff[i]:self.eoff[i + 1]]

    def query(self, i: int) -> np.ndarray:
        return self.queries[self.qoff[i]:self.qoff[i + 1]]


def _offsets(sizes) -> np.ndarray:
    off = np.zeros(len(sizes) + 1, np.int64)
    np.cumsum(np.asarray(sizes, np.int64), out=off[1:])
    return off


def er_stream(n=1 << 16, batches=16, batch=1 << 14, qbatch=1 << 14, probes=1 << 10,
              seed=BASE_SEED + 1, stream=0, name="er") -> Stream:
    """Uniform random (Erdos-Renyi) endpoints, self-loops and repeats kept."""
    m = batches * batch
    edges = uniform_pairs(key(seed, stream, P_EDGES), 0, m, n)
    queries = uniform_pairs(key(seed, stream, P_QUERIES), 0, batches * qbatch, n)
    pr = uniform_pairs(key(seed, stream, P_PROBES), 0, probes, n)
    return Stream(name, n, edges, _offsets([batch] * batches), queries,
                  _offsets([qbatch] * batches), pr,
                  dict(kind="uniform", batch=batch, qbatch=qbatch))


def rmat_batch_sizes(total: int, lo: float, hi: float, k: int) -> list:
    """Log-uniform minibatch sizes floor(2^U), U ~ U[lo, hi], drawn until the
    sum reaches `total`; the last one is truncated."""
    sizes, acc, start = [], 0, 0
    while acc < total:
        chunk = loguniform_sizes_from(k, start, 256, lo, hi)
        start += 256
        for s in chunk:
            s = int(min(s, total - acc))
            sizes.append(s)
            acc += s
            if acc >= total:
                break
    return sizes


def loguniform_sizes_from(k: int, start: int, count: int, lo: float, hi: float) -> np.ndarray:
    u = unit_doubles(k, start, count)
    return np.floor(np.exp2(lo + (hi - lo) * u)).astype(np.int64)


def rmat_stream(scale=24, edge_factor=16, size_lo=16.0, size_hi=24.0, qbatch=1 << 20,
                probes=1 << 10, seed=BASE_SEED + 2, stream=0, name="rmat",
                edges_out=None) -> Stream:
    """R-MAT (a=.57, b=.19, c=.19, d=.05) with ids randomly permuted, streamed
    as log-uniform minibatches, each followed by `qbatch` uniform pairs."""
    n = 1 << scale
    m = edge_factor * n
    perm = permutation(key(seed, stream, P_PERM), n)
    edges = rmat_edges(key(seed, stream, P_EDGES), 0, m, scale, n, perm, out=edges_out)
    sizes = rmat_batch_sizes(m, size_lo, size_hi, key(seed, stream, P_SIZES))
    nb = len(sizes)
    queries = uniform_pairs(key(seed, stream, P_QUERIES), 0, nb * qbatch, n)
    pr = uniform_pairs(key(seed, stream, P_PROBES), 0, probes, n)
    return Stream(name, n, edges, _offsets(sizes), queries, _offsets([qbatch] * nb), pr,
                  dict(kind="rmat", scale=scale, edge_factor=edge_factor,
                       size_lo=size_lo, size_hi=size_hi, qbatch=qbatch))


def grid_stream_cfg(W=4096, H=4096, long_frac=0.01, batch=1 << 12, qbatch=1 << 10,
                    probes=1 << 10, seed=BASE_SEED + 4, stream=0, name="grid") -> Stream:
    """W x H 4-neighbour mesh (row-major ids) plus floor(long_frac * mesh edges)
    uniform long-range edges, all shuffled, delivered in minibatches of
    `batch` (every edge delivered; the last batch is ragged)."""
    n = W * H
    mesh = int(lib().sg_grid_edge_count(W, H))
    extra = int(np.floor(long_frac * mesh))
    edges = grid_stream(W, H, extra, key(seed, stream, P_LONGRANGE), key(seed, stream, P_SHUFFLE))
    m = edges.shape[0]
    nb = (m + batch - 1) // batch
    sizes = [batch] * (nb - 1) + [m - batch * (nb - 1)]
    queries = uniform_pairs(key(seed, stream, P_QUERIES), 0, nb * qbatch, n)
    pr = uniform_pairs(key(seed, stream, P_PROBES), 0, probes, n)
    return Stream(name, n, edges, _offsets(sizes), queries, _offsets([qbatch] * nb), pr,
                  dict(kind="grid", W=W, H=H, extra=extra, batch=batch, qbatch=qbatch))


def grid3d_stream_cfg(L=256, batch=1 << 22, qbatch=1 << 20, probes=1 << 10, seed=BASE_SEED + 6, stream=0,
                      name="grid3d") -> Stream:
    """L^3 6-neighbour mesh (stands in for the paper's 3Dgrid), shuffled,
    in minibatches of `batch` (the last ragged), each followed by uniform pairs."""
    n = L ** 3
    edges = grid3d_edges(L, key(seed, stream, P_SHUFFLE))
    m = edges.shape[0]
    nb = (m + batch - 1) // batch
    sizes = [batch] * (nb - 1) + [m - batch * (nb - 1)]
    queries = uniform_pairs(key(seed, stream, P_QUERIES), 0, nb * qbatch, n)
    pr = uniform_pairs(key(seed, stream, P_PROBES), 0, probes, n)
    return Stream(name, n, edges, _offsets(sizes), queries, _offsets([qbatch] * nb), pr,
                  dict(kind="grid3d", L=L, batch=batch, qbatch=qbatch))


def local_stream(n=1 << 24, degree=5, window=1 << 12, batch=1 << 22, qbatch=1 << 20, probes=1 << 10,
                 seed=BASE_SEED + 7, stream=0, name="local") -> Stream:
    """degree * n locality-biased random edges (stands in for the paper's
    local5 / local16 "small separator" graphs), in minibatches of `batch`."""
    m = degree * n
    edges = local_pairs(key(seed, stream, P_EDGES), 0, m, n, window)
    nb = (m + batch - 1) // batch
    sizes = [batch] * (nb - 1) + [m - batch * (nb - 1)]
    queries = uniform_pairs(key(seed, stream, P_QUERIES), 0, nb * qbatch, n)
    pr = uniform_pairs(key(seed, stream, P_PROBES), 0, probes, n)
    return Stream(name, n, edges, _offsets(sizes), queries, _offsets([qbatch] * nb), pr,
                  dict(kind="local", degree=degree, window=window, batch=batch, qbatch=qbatch))


def multi_graph_sizes(G=1024, mu=14.0, sigma=2.0, lo=1 << 10, hi=1 << 20,
                      seed=BASE_SEED + 3) -> np.ndarray:
    """Vertex counts of the independent graphs: clip(round(2^X), lo, hi), X ~ N(mu, sigma)."""
    return lognormal_counts(key(seed, 0, P_GRAPH_N), G, mu, sigma, lo, hi)


def multi_graph_stream(g: int, n: int, edges_per_vertex=8, steps=4, qbatch=1 << 12,
                       rmat_from=512, seed=BASE_SEED + 3, name="multi") -> Stream:
    """Graph g of the many-graph workload: m = edges_per_vertex * n edges split
    at steps-1 sorted uniform cut points (empty parts allowed); uniform
    endpoints for g < rmat_from, else R-MAT at scale ceil(log2 n) with
    out-of-range draws redrawn and ids permuted.  `qbatch` uniform query pairs
    follow each step."""
    m = edges_per_vertex * n
    if g < rmat_from:
        edges = uniform_pairs(key(seed, g + 1, P_EDGES), 0, m, n)
        kind = "uniform"
    else:
        scale = max(1, int(np.ceil(np.log2(n))))
        perm = permutation(key(seed, g + 1, P_PERM), n)
        edges = rmat_edges(key(seed, g + 1, P_EDGES), 0, m, scale, n, perm)
        kind = "rmat"
    cuts = np.sort((unit_doubles(key(seed, g + 1, P_CUTS), 0, steps - 1) * m).astype(np.int64))
    eoff = np.concatenate([[0], cuts, [m]]).astype(np.int64)
    queries = uniform_pairs(key(seed, g + 1, P_QUERIES), 0, steps * qbatch, n)
    return Stream("%s[%d]" % (name, g), n, edges, eoff, queries,
                  _offsets([qbatch] * steps), meta=dict(kind=kind, graph=g))


@dataclass
class TraceRequest:
    """One request of a serving trace: `items` are int32 [size, 2] edges
    (kind 0, update) or pairs (kind 1, query) of graph `stream`."""
    rid: int
    stream: int
    kind: int
    size: int
    items: np.ndarray


def serving_trace(S=64, scale=22, R=1024, upd_frac=0.7, size_lo=8.0, size_hi=22.0,
                  seed=BASE_SEED + 5) -> list:
    """The serving workload: R requests over S graph streams, each graph an
    R-MAT stream at `scale` (a=.57 b=.19 c=.19, ids permuted per graph).
    Request i goes to a uniform stream; it is an update with probability
    upd_frac, else a query; its size is floor(2^U), U ~ U[size_lo, size_hi].
    An update takes the next `size` edges of its graph's stream, a query the
    next `size` uniform pairs of the graph's query stream.  Arrival times are
    drawn separately (poisson_arrivals with key P_ARRIVALS)."""
    n = 1 << scale
    kind_u = unit_doubles(key(seed, 0, P_REQ_TYPE), 0, R)
    strm = np.minimum((unit_doubles(key(seed, 0, P_REQ_STREAM), 0, R) * S).astype(np.int64), S - 1)
    sizes = np.floor(np.exp2(size_lo + (size_hi - size_lo) *
                             unit_doubles(key(seed, 0, P_REQ_SIZE), 0, R))).astype(np.int64)
    perms = {}
    ecur = np.zeros(S, np.int64)
    qcur = np.zeros(S, np.int64)
    out = []
    for i in range(R):
        st, size = int(strm[i]), int(sizes[i])
        if kind_u[i] < upd_frac:
            if st not in perms:
                perms[st] = permutation(key(seed, st + 1, P_PERM), n)
            items = rmat_edges(key(seed, st + 1, P_EDGES), int(ecur[st]), size, scale, n, perms[st])
            ecur[st] += size
            out.append(TraceRequest(i, st, 0, size, items))
        else:
            items = uniform_pairs(key(seed, st + 1, P_QUERIES), int(qcur[st]), size, n)
            qcur[st] += size
            out.append(TraceRequest(i, st, 1, size, items))
    return out


def tiny_stream(n: int, edges, batches: list, queries=None) -> Stream:
    """A hand-written stream (tests)."""
    e = np.ascontiguousarray(np.asarray(edges, np.int32).reshape(-1, 2))
    q = np.ascontiguousarray(np.asarray(queries if queries is not None else np.empty((0, 2)),
                                        np.int32).reshape(-1, 2))
    return Stream("tiny", n, e, _offsets(batches), q, _offsets([q.shape[0]] + [0] * (len(batches) - 1)))


def chain_forest(n: int, L: int, seed=BASE_SEED + 9):
    """A forest image of n // L paths of L vertices each (L divides n): the
    vertices of a path are drawn at random and ordered so that every parent
    id is below its child's, which an id-order forest may hold.  Returns
    (parent int32[n], path int64[n]): path[v] is the index of v's path, so
    u and v are connected iff path[u] == path[v]."""
    if L < 1 or n % L:
        raise ValueError("L must divide n")
    rows = permutation(key(seed, 0, P_PERM), n).reshape(n // L, L)
    rows.sort(axis=1)
    parent = np.empty(n, np.int32)
    parent[rows[:, 0]] = rows[:, 0]
    parent[rows[:, 1:].ravel()] = rows[:, :-1].ravel()
    path = np.empty(n, np.int64)
    path[rows.ravel()] = np.repeat(np.arange(n // L, dtype=np.int64), L)
    return parent, path
