"""Pins of the CPU oracle against things other than itself.

* brute force: BFS components, exhaustively on every edge set of K_5 and on
  seeded random graphs up to 2^10 vertices;
* a library routine: scipy.sparse.csgraph.connected_components on the
  uniform-random tiny workload after every minibatch;
* the paper's worked example: the star minibatch of Section 4.2;
* closed forms: mesh, perfect matching, self-loops, reversed path;
* invariants: components == n - unions == #roots, monotone answers, label
  properties, the union-by-rank height bound of the Section 4 lemma;
* order independence (Section 4.2 correctness lemma);
* planted mistakes: mutated copies of the oracle must fail these pins.
"""
import itertools
import os
import subprocess

import numpy as np
import pytest
import scipy.sparse as sp
from scipy.sparse.csgraph import connected_components

import oracle
import synth
from bruteforce import bfs_answers, bfs_labels

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def all_pairs(n):
    return np.array([(a, b) for a in range(n) for b in range(n)], np.int32).reshape(-1, 2)


def check_stream_against_bfs(n, batches, uf_factory=oracle.UnionFind):
    """Apply the batches one by one; after each compare every pair's answer,
    every label and the component count with BFS on all edges so far."""
    uf = uf_factory(n)
    seen = []
    pairs = all_pairs(n)
    for b in batches:
        b = np.asarray(b, np.int32).reshape(-1, 2)
        uf.bulk_update(b)
        seen.extend(map(tuple, b))
        lab = bfs_labels(n, seen)
        np.testing.assert_array_equal(uf.labels(), lab)
        np.testing.assert_array_equal(uf.bulk_query(pairs), bfs_answers(lab, pairs))
        assert uf.num_components() == len(set(lab.tolist()))


def test_exhaustive_k5(built_libs):
    n = 5
    kn = [(a, b) for a in range(n) for b in range(a + 1, n)]
    for mask in range(1 << len(kn)):
        es = [kn[i] if (i % 2 == 0) else kn[i][::-1] for i in range(len(kn)) if mask >> i & 1]
        half = len(es) // 2
        check_stream_against_bfs(n, [es[:half], es[half:]])


@pytest.mark.parametrize("seed", range(12))
def test_random_small_vs_bfs(built_libs, seed):
    rng = np.random.default_rng(seed)
    n = int(rng.integers(2, 1 << 10))
    m = int(rng.integers(0, 2 * n))
    e = rng.integers(0, n, size=(m, 2)).astype(np.int32)
    cuts = np.sort(rng.integers(0, m + 1, size=3))
    batches = np.split(e, cuts)
    uf = oracle.UnionFind(n)
    seen = []
    q = rng.integers(0, n, size=(256, 2)).astype(np.int32)
    for b in batches:
        uf.bulk_update(b)
        seen.extend(map(tuple, b))
        lab = bfs_labels(n, seen)
        np.testing.assert_array_equal(uf.labels(), lab)
        np.testing.assert_array_equal(uf.bulk_query(q), bfs_answers(lab, q))
        assert uf.num_components() == len(np.unique(lab))


def scipy_min_labels(n, edges):
    """Component labels from scipy, re-mapped to the smallest id per component."""
    e = np.asarray(edges, np.int64).reshape(-1, 2)
    g = sp.coo_matrix((np.ones(len(e), np.int8), (e[:, 0], e[:, 1])), shape=(n, n))
    k, lab = connected_components(g, directed=False)
    mins = np.full(k, n, np.int64)
    np.minimum.at(mins, lab, np.arange(n))
    return k, mins[lab].astype(np.int32)


def test_er_tiny_vs_scipy(built_libs):
    s = synth.er_stream()
    uf = oracle.UnionFind(s.n)
    for i in range(s.num_batches):
        uf.bulk_update(s.batch(i))
        k, lab = scipy_min_labels(s.n, s.edges[: s.eoff[i + 1]])
        assert uf.num_components() == k
        np.testing.assert_array_equal(uf.labels(), lab)
        q = s.query(i)
        np.testing.assert_array_equal(uf.bulk_query(q), (lab[q[:, 0]] == lab[q[:, 1]]).astype(np.uint8))


def test_small_rmat_vs_scipy(built_libs):
    s = synth.rmat_stream(scale=14, size_lo=8, size_hi=14, qbatch=1 << 10)
    uf = oracle.UnionFind(s.n)
    for i in range(s.num_batches):
        uf.bulk_update(s.batch(i))
    k, lab = scipy_min_labels(s.n, s.edges)
    assert uf.num_components() == k
    np.testing.assert_array_equal(uf.labels(), lab)


def load_golden(name):
    d = {"edges": []}
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.split("#")[0].split()
            if not line:
                continue
            if line[0] == "edge":
                d["edges"].append((int(line[1]), int(line[2])))
            elif line[0] in ("n", "components"):
                d[line[0]] = int(line[1])
            else:
                d[line[0]] = [int(x) for x in line[1:]]
    return d


def test_star_worked_example(built_libs):
    g = load_golden("star_section4_2.txt")
    uf = oracle.UnionFind(g["n"])
    uf.bulk_update(g["edges"])
    assert uf.num_components() == g["components"]
    c = g["connected"]
    ans = uf.bulk_query([(a, b) for a in c for b in c])
    assert ans.all()
    iso = g["isolated"]
    ans = uf.bulk_query([(a, b) for a in iso for b in c + iso if a != b])
    assert not ans.any()
    lab = uf.labels()
    assert (lab[c] == min(c)).all() and (lab[iso] == iso).all()


def test_closed_form_mesh(built_libs):
    W, H = 64, 48
    e = synth.grid_stream(W, H, 0, synth.key(1, 0, synth.P_LONGRANGE), synth.key(1, 0, synth.P_SHUFFLE))
    assert e.shape[0] == H * (W - 1) + (H - 1) * W
    uf = oracle.UnionFind(W * H)
    for b in np.array_split(e, 7):
        uf.bulk_update(b)
    assert uf.num_components() == 1
    assert (uf.labels() == 0).all()


def test_closed_form_matching_and_selfloops(built_libs):
    n = 1 << 12
    uf = oracle.UnionFind(n)
    uf.bulk_update(np.stack([np.arange(n), np.arange(n)], 1))
    assert uf.num_components() == n
    np.testing.assert_array_equal(uf.labels(), np.arange(n))
    ev = np.arange(0, n, 2)
    uf.bulk_update(np.stack([ev + 1, ev], 1))
    assert uf.num_components() == n // 2
    lab = uf.labels()
    np.testing.assert_array_equal(lab[1::2], ev)
    np.testing.assert_array_equal(lab[0::2], ev)


def test_closed_form_reversed_path(built_libs):
    n = 1 << 16
    i = np.arange(n - 2, -1, -1)
    uf = oracle.UnionFind(n)
    uf.bulk_update(np.stack([i, i + 1], 1))
    assert uf.num_components() == 1
    assert (uf.labels() == 0).all()


def test_invariants_along_stream(built_libs):
    s = synth.rmat_stream(scale=16, size_lo=8, size_hi=15, qbatch=1 << 12)
    uf = oracle.UnionFind(s.n)
    prev = np.zeros(len(s.probes), np.uint8)
    for i in range(s.num_batches):
        uf.bulk_update(s.batch(i))
        assert uf.num_components() == s.n - uf.unions() == uf.count_roots()
        a = uf.bulk_query(s.probes)
        assert (a >= prev).all(), "an answer went from connected to disconnected"
        prev = a
        lab = uf.labels()
        v = np.arange(s.n)
        assert (lab <= v).all()
        assert (lab[lab] == lab).all()
        assert ((lab == v).sum()) == uf.num_components()
        q = s.query(i)
        np.testing.assert_array_equal(uf.bulk_query(q), (lab[q[:, 0]] == lab[q[:, 1]]).astype(np.uint8))
        assert uf.max_height() <= int(np.floor(np.log2(s.n)))


def test_height_bound_is_tight_and_kept(built_libs):
    # root-to-root unions in a binomial pattern reach height exactly log2 n
    k = 10
    n = 1 << k
    uf = oracle.UnionFind(n)
    for r in range(k):
        i = np.arange(0, n, 2 << r)
        uf.bulk_update(np.stack([i, i + (1 << r)], 1))
    assert uf.max_height() == k
    # a path added in order stays within the bound (linking by rank, not by argument order)
    uf = oracle.UnionFind(n)
    i = np.arange(n - 1)
    uf.bulk_update(np.stack([i, i + 1], 1))
    assert uf.max_height() <= k


def test_order_independence(built_libs):
    s = synth.rmat_stream(scale=13, size_lo=8, size_hi=13, qbatch=16)
    rng = np.random.default_rng(7)
    ref = oracle.UnionFind(s.n)
    ref.bulk_update(s.edges)
    for trial in range(3):
        e = s.edges[rng.permutation(len(s.edges))]
        e = np.where(rng.random((len(e), 1)) < 0.5, e, e[:, ::-1])  # undirected
        uf = oracle.UnionFind(s.n)
        for b in np.array_split(e, 1 + trial * 5):
            uf.bulk_update(b)
        np.testing.assert_array_equal(uf.labels(), ref.labels())


def test_invalid_ids_skipped(built_libs):
    n = 10
    uf = oracle.UnionFind(n)
    bad = uf.bulk_update([(0, 1), (-1, 2), (2, 10), (3, 4), (11, -5), (4, 5)])
    assert bad == 3 and uf.invalid() == 3
    assert uf.num_components() == n - 3
    ans = uf.bulk_query([(0, 1), (3, 5), (0, 10), (-1, -1), (7, 7), (1, 3)])
    np.testing.assert_array_equal(ans, [1, 1, 0, 0, 1, 0])
    assert uf.invalid() == 5


def test_empty_minibatch(built_libs):
    uf = oracle.UnionFind(4)
    assert uf.bulk_update(np.empty((0, 2), np.int32)) == 0
    assert uf.num_components() == 4
    assert uf.bulk_query(np.empty((0, 2), np.int32)).shape == (0,)


# --- planted mistakes ---------------------------------------------------------

MUTANTS = {
    "no_link": ("  u->parent[rb] = ra;\n", "\n"),
    "find_one_step": ("while (u->parent[r] != r) r = u->parent[r];",
                      "if (u->parent[r] != r) r = u->parent[r];"),
    "query_negated": ("uf_find(u, a) == uf_find(u, b) ? 1 : 0", "uf_find(u, a) != uf_find(u, b) ? 1 : 0"),
    "label_last_seen": ("if (first[r] < 0) first[r] = (int32_t)v;", "first[r] = (int32_t)v;"),
    "range_drops_zero": ("return x >= 0 && (int64_t)x < u->n;", "return x > 0 && (int64_t)x < u->n;"),
    "no_union_count": ("  u->unions++;\n", "\n"),
    "link_second_arg": ("u->parent[rb] = ra;", "u->parent[ra] = rb;"),
}


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_pins_catch_planted_mistake(built_libs, tmp_path, name):
    src = open(os.path.join(os.path.dirname(oracle.__file__), "uf_oracle.c")).read()
    old, new = MUTANTS[name]
    assert old in src, name
    mpath = tmp_path / "mutant.c"
    mpath.write_text(src.replace(old, new, 1))
    so = tmp_path / "libmutant.so"
    subprocess.check_call(["gcc", "-O1", "-fPIC", "-shared", "-std=c11", "-o", str(so), str(mpath)])
    L = oracle.load_lib(str(so))
    factory = lambda n: oracle.UnionFind(n, _lib=L)  # noqa: E731
    caught = False
    try:
        n = 5
        kn = [(a, b) for a in range(n) for b in range(a + 1, n)]
        for mask in range(0, 1 << len(kn), 7):
            es = [kn[i] for i in range(len(kn)) if mask >> i & 1]
            check_stream_against_bfs(n, [es[: len(es) // 2], es[len(es) // 2:]], factory)
        # the invariants and the height bound
        uf = factory(1 << 10)
        i = np.arange((1 << 10) - 1)
        uf.bulk_update(np.stack([i, i + 1], 1))
        assert uf.num_components() == (1 << 10) - uf.unions() == uf.count_roots() == 1
        assert uf.max_height() <= 10
    except AssertionError:
        caught = True
    assert caught, "mutant %s survived the pins" % name


def component_trace(s, points=10):
    uf = oracle.UnionFind(s.n)
    out = []
    for i in range(s.num_batches):
        uf.bulk_update(s.batch(i))
        out.append((s.eoff[i + 1] / len(s.edges), uf.num_components()))
    return out


def test_stream_shapes_match_the_component_trends_of_section_6(built_libs):
    """Section 6.2 describes the component counts along the paper's streams
    (Fig. 2, whose curves are not in the text): local16 is connected around
    the middle of the stream, rMat keeps many components to the end, and
    random and local5 are almost indistinguishable until the end.  The
    synthetic stand-ins reproduce those shapes (n = 2^16)."""
    n = 1 << 16
    loc16 = component_trace(synth.local_stream(n=n, degree=16, window=1 << 8, batch=1 << 14, qbatch=1))
    first_one = next(f for f, c in loc16 if c == 1)
    assert 0.3 <= first_one <= 0.7
    rmat = component_trace(synth.rmat_stream(scale=16, size_lo=10, size_hi=14, qbatch=1))
    assert rmat[-1][1] > 0.25 * n
    rnd = component_trace(synth.er_stream(n=n, batches=20, batch=5 * n // 20, qbatch=1, probes=0))
    loc5 = component_trace(synth.local_stream(n=n, degree=5, window=1 << 8, batch=5 * n // 20, qbatch=1))
    for (f1, c1), (f2, c2) in zip(rnd[:-4], loc5[:-4]):
        assert abs(f1 - f2) < 1e-9 and abs(c1 - c2) <= 0.05 * max(c1, c2) + 50
