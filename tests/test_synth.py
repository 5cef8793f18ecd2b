"""The seeded input generators: determinism, ranges, shapes and the R-MAT
quadrant frequencies."""
import numpy as np

import synth


def test_splitmix64_reference_values(built_libs):
    # splitmix64 started at state 0: published first outputs of Vigna's generator
    assert synth.draws(0, 0, 3).tolist() == [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4,
                                              0x06C45D188009454F]


def test_counter_based_slices(built_libs):
    k = synth.key(5, 1, synth.P_EDGES)
    full = synth.uniform_pairs(k, 0, 1000, 12345)
    part = synth.uniform_pairs(k, 400, 300, 12345)
    np.testing.assert_array_equal(full[400:700], part)
    assert full.min() >= 0 and full.max() < 12345
    assert not np.array_equal(full, synth.uniform_pairs(synth.key(6, 1, synth.P_EDGES), 0, 1000, 12345))


def test_rmat_quadrants_and_range(built_libs):
    scale = 12
    e = synth.rmat_edges(synth.key(1, 0, 1), 0, 200000, scale, 1 << scale)
    assert e.min() >= 0 and e.max() < (1 << scale)
    top_u = (e[:, 0] >> (scale - 1)) & 1
    top_v = (e[:, 1] >> (scale - 1)) & 1
    # P(u msb = 1) = c + d = 0.24, P(v msb = 1) = b + d = 0.24, P(both) = d = 0.05
    assert abs(top_u.mean() - 0.24) < 0.005
    assert abs(top_v.mean() - 0.24) < 0.005
    assert abs((top_u & top_v).mean() - 0.05) < 0.003


def test_rmat_non_power_of_two_redraw(built_libs):
    n = 3000
    e = synth.rmat_edges(synth.key(2, 0, 1), 0, 50000, 12, n)
    assert e.min() >= 0 and e.max() < n


def test_permutation_and_stream_shapes(built_libs):
    p = synth.permutation(synth.key(3, 0, synth.P_PERM), 1 << 14)
    assert np.array_equal(np.sort(p), np.arange(1 << 14))
    s = synth.rmat_stream(scale=12, size_lo=6, size_hi=12, qbatch=100)
    assert s.eoff[-1] == 16 << 12 and len(s.edges) == 16 << 12
    sizes = np.diff(s.eoff)
    assert sizes.min() >= 0 and sizes[:-1].min() >= 64 and sizes.max() <= 4096
    assert s.qoff[-1] == 100 * s.num_batches
    g = synth.grid_stream_cfg(W=64, H=32, batch=100)
    mesh = 32 * 63 + 31 * 64
    assert g.edges.shape[0] == mesh + mesh // 100
    assert np.diff(g.eoff)[:-1].min() == 100 and g.eoff[-1] == g.edges.shape[0]


def test_multi_graph_recipe(built_libs):
    ns = synth.multi_graph_sizes(G=64)
    assert ns.min() >= 1 << 10 and ns.max() <= 1 << 20
    s0 = synth.multi_graph_stream(0, int(ns[0]))
    s1 = synth.multi_graph_stream(600, int(ns[1]))
    for s, n in ((s0, ns[0]), (s1, ns[1])):
        assert s.num_batches == 4 and s.eoff[-1] == 8 * n
        assert s.edges.max() < n and (np.diff(s.eoff) >= 0).all()
    assert s1.meta["kind"] == "rmat" and s0.meta["kind"] == "uniform"


def test_grid3d_and_local_recipes(built_libs):
    import oracle
    L = 12
    e = synth.grid3d_edges(L, synth.key(1, 0, synth.P_SHUFFLE))
    assert e.shape[0] == 3 * L * L * (L - 1)
    d = np.abs(e[:, 0].astype(np.int64) - e[:, 1])
    assert set(d.tolist()) == {1, L, L * L}
    assert len({tuple(sorted(x)) for x in e.tolist()}) == e.shape[0]  # no repeats
    uf = oracle.UnionFind(L ** 3)
    uf.bulk_update(e)
    assert uf.num_components() == 1  # closed form: the mesh is connected
    n, w = 1 << 14, 1 << 6
    s = synth.local_stream(n=n, degree=5, window=w, batch=1 << 12, qbatch=64)
    dd = np.abs(s.edges[:, 0].astype(np.int64) - s.edges[:, 1])
    dd = np.minimum(dd, n - dd)
    assert len(s.edges) == 5 * n and dd.max() < w and s.edges.min() >= 0 and s.edges.max() < n


def test_chain_forest_shape(built_libs):
    n, L = 1 << 12, 64
    parent, path = synth.chain_forest(n, L)
    v = np.arange(n)
    assert parent.dtype == np.int32 and (parent <= v).all()  # an image id-order linking accepts
    roots = parent == v
    assert roots.sum() == n // L
    # every vertex reaches its path's root in at most L - 1 steps, and the
    # deepest takes exactly L - 1
    x, depth = v.copy(), np.zeros(n, np.int64)
    for _ in range(L):
        nx = parent[x]
        depth += nx != x
        x = nx
    assert (parent[x] == x).all() and depth.max() == L - 1
    assert (path == path[x]).all()  # a path's vertices share its root
    assert np.bincount(path).tolist() == [L] * (n // L)
    p2, _ = synth.chain_forest(n, L)
    np.testing.assert_array_equal(parent, p2)
