"""The many-graph pool (batched form) against one oracle per graph."""
import numpy as np
import pytest
import torch

import oracle
import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def cc():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1602_05232_amd as ccgpu
    ccgpu.lib()
    return ccgpu


def dev(a):
    a = np.ascontiguousarray(np.asarray(a, dtype=np.int32))
    return torch.from_numpy(a).cuda()


def small_graphs(G, seed=5):
    """Graphs of the many-graph recipe, with sizes scaled down for the oracle."""
    ns = synth.multi_graph_sizes(G=G, mu=9.0, sigma=2.0, lo=1 << 4, hi=1 << 13, seed=seed)
    return [synth.multi_graph_stream(g, int(ns[g]), qbatch=200, rmat_from=G // 2, seed=seed) for g in range(G)]


@pytest.mark.parametrize("opts", [dict(), dict(hook=1), dict(items=1, block=64, grid_cap=5),
                                  dict(items=8, block=512, compress_linked=0, query_halving=0),
                                  dict(one_launch=1), dict(one_launch=1, hook=1, items=1, grid_cap=3),
                                  dict(hook=2), dict(hook=2, compress_linked=0, items=8, block=1024),
                                  dict(one_launch=1, hook=2, grid_cap=7),
                                  dict(filter=1), dict(filter=1, hook=2, compress_linked=0, items=8, block=512),
                                  dict(filter=1, hook=1, items=1, block=64, grid_cap=5),
                                  dict(filter=1, hook=0, items=4, query_halving=0),
                                  dict(filter=1, one_launch=1, hook=2, grid_cap=7)],
                         ids=lambda o: ",".join("%s=%s" % kv for kv in sorted(o.items())) or "default")
def test_pool_steps_match_oracle(cc, opts):
    G = 96
    streams = small_graphs(G)
    pool = cc.Pool(sum(s.n for s in streams) + 1000, G + 4, **opts)
    ids = [pool.add(s.n) for s in streams]
    refs = [oracle.UnionFind(s.n) for s in streams]
    E = [dev(s.edges) for s in streams]
    Q = [dev(s.queries) for s in streams]
    outs = [torch.empty(len(s.queries), dtype=torch.uint8, device="cuda") for s in streams]
    for step in range(4):
        ops = []
        for g, s in enumerate(streams):
            e0, e1 = int(s.eoff[step]), int(s.eoff[step + 1])
            q0, q1 = int(s.qoff[step]), int(s.qoff[step + 1])
            ops.append((ids[g], cc.UPDATE, E[g][e0:e1], None))
        for g, s in enumerate(streams):
            q0, q1 = int(s.qoff[step]), int(s.qoff[step + 1])
            ops.append((ids[g], cc.QUERY, Q[g][q0:q1], outs[g][q0:q1]))
        pool.run(ops)
    for g, s in enumerate(streams):
        want = []
        for k in range(4):
            refs[g].bulk_update(s.batch(k))
            want.append(refs[g].bulk_query(s.query(k)))
        np.testing.assert_array_equal(outs[g].cpu().numpy(), np.concatenate(want), err_msg="graph %d" % g)
        np.testing.assert_array_equal(pool.labels(ids[g]).cpu().numpy(), refs[g].labels(), err_msg="graph %d" % g)
        assert pool.num_components(ids[g]) == refs[g].num_components()
    assert pool.sync() == cc.cc.CC_OK
    pool.close()


@pytest.mark.parametrize("one_launch", [0, 1])
def test_pool_many_rounds_in_one_run(cc, one_launch):
    # several operations per graph in one run: rounds must keep list order
    G = 24
    streams = small_graphs(G, seed=9)
    pool = cc.Pool(sum(s.n for s in streams), G, one_launch=one_launch)
    ids = [pool.add(s.n) for s in streams]
    ops, outs, want = [], [], []
    for g, s in enumerate(streams):
        ref = oracle.UnionFind(s.n)
        for k in range(4):
            ops.append((ids[g], cc.UPDATE, dev(s.batch(k)), None))
            ref.bulk_update(s.batch(k))
            o = torch.empty(len(s.query(k)), dtype=torch.uint8, device="cuda")
            ops.append((ids[g], cc.QUERY, dev(s.query(k)), o))
            outs.append(o)
            want.append(ref.bulk_query(s.query(k)))
    # interleave graphs so that consecutive list entries belong to different graphs
    order = sorted(range(len(ops)), key=lambda i: (i % 8, i))
    per_graph = {}
    for i in order:
        per_graph.setdefault(ops[i][0], []).append(i)
    assert all(v == sorted(v) for v in per_graph.values())
    pool.run([ops[i] for i in order])
    for o, w in zip(outs, want):
        np.testing.assert_array_equal(o.cpu().numpy(), w)
    pool.close()


def test_pool_gaps_eviction_and_images(cc):
    pool = cc.Pool(10000, 8)
    a = pool.add(4000)
    b = pool.add(3000)
    c = pool.add(3000)
    assert pool.free_vertices() == 0
    with pytest.raises(cc.CCError) as ei:
        pool.add(1)
    assert ei.value.code == cc.cc.CC_ENOMEM
    s = synth.rmat_stream(scale=11, size_lo=6, size_hi=10, qbatch=64)  # n = 2048 <= 3000
    eb = synth.uniform_pairs(synth.key(3, 0, 1), 0, 5000, 3000)
    pool.run([(b, cc.UPDATE, dev(eb), None)])
    ref = oracle.UnionFind(3000)
    ref.bulk_update(eb)
    img = pool.save(b)  # evict b
    pool.remove(b)
    assert pool.largest_gap() == 3000
    d = pool.add(2048)  # another graph takes part of the gap
    pool.run([(d, cc.UPDATE, dev(s.edges), None)])
    with pytest.raises(cc.CCError):
        pool.add(3000)  # no room for b any more
    pool.remove(d)
    b2 = pool.add(3000)  # restore b elsewhere
    pool.load(b2, img)
    np.testing.assert_array_equal(pool.labels(b2).cpu().numpy(), ref.labels())
    assert pool.num_components(b2) == ref.num_components()
    # a corrupt image is refused on the device and the graph is left as it was
    bad = bytearray(img)
    par = np.frombuffer(bad, np.int32, offset=16)
    par[10] = 11  # points upward in id order
    with pytest.raises(cc.CCError) as ei:
        pool.load(b2, bad)
    assert ei.value.code == cc.cc.CC_ECORRUPT
    np.testing.assert_array_equal(pool.labels(b2).cpu().numpy(), ref.labels())
    # the image is a cc_save image: a standalone graph takes it as is
    g = cc.Graph(3000)
    g.load(img)
    np.testing.assert_array_equal(g.labels().cpu().numpy(), ref.labels())
    g.close()
    # invalid operations are rejected before anything runs
    with pytest.raises(cc.CCError) as ei:
        pool.run([(a, cc.UPDATE, dev(eb[:10]), None), (77, cc.UPDATE, dev(eb[:10]), None)])
    assert ei.value.code == cc.cc.CC_EINVAL
    assert pool.num_components(a) == 4000
    # out-of-range ids are skipped and reported
    pool.run([(c, cc.UPDATE, dev([[0, 1], [2, 3000], [5, 6]]), None)])
    assert pool.sync() == cc.cc.CC_ERANGE
    assert pool.num_components(c) == 3000 - 2
    pool.close()


def test_pool_rank_images_and_limits(cc):
    """Union by rank in a pool: a graph's image carries ranks in its roots'
    words; it round-trips through another slot and through a standalone
    graph, a cyclic image is refused, and rank needs graphs of at most 2^27
    vertices (the arena may be larger)."""
    pool = cc.Pool(9000, 4, hook=2)
    a = pool.add(3000)
    b = pool.add(3000)
    eb = synth.uniform_pairs(synth.key(13, 0, 1), 0, 4000, 3000)
    pool.run([(a, cc.UPDATE, dev(eb[:2000]), None), (b, cc.UPDATE, dev(eb[2000:]), None)])
    pool.run([(a, cc.UPDATE, dev(eb[2000:]), None)])
    ref = oracle.UnionFind(3000)
    ref.bulk_update(eb)
    np.testing.assert_array_equal(pool.labels(a).cpu().numpy(), ref.labels())
    img = pool.save(a)
    words = np.frombuffer(bytes(img), np.int32, offset=16)
    assert (words.view(np.uint32) >> 27).max() > 0, "no root carries a rank"
    c = pool.add(3000)
    pool.load(c, img)
    np.testing.assert_array_equal(pool.labels(c).cpu().numpy(), ref.labels())
    assert pool.num_components(c) == ref.num_components()
    q = synth.uniform_pairs(synth.key(13, 0, 2), 0, 3000, 3000)
    out = torch.empty(len(q), dtype=torch.uint8, device="cuda")
    pool.run([(c, cc.QUERY, dev(q), out)])
    np.testing.assert_array_equal(out.cpu().numpy(), ref.bulk_query(q))
    g = cc.Graph(3000, hook=2)
    g.load(img)
    np.testing.assert_array_equal(g.labels().cpu().numpy(), ref.labels())
    g.close()
    bad = bytearray(img)
    par = np.frombuffer(bad, np.int32, offset=16)
    x = int(np.flatnonzero((par & ((1 << 27) - 1)) != np.arange(3000))[0])
    par[x], par[int(par[x]) & ((1 << 27) - 1)] = int(par[x]) & ((1 << 27) - 1), x  # two-cycle
    with pytest.raises(cc.CCError) as ei:
        pool.load(c, bad)
    assert ei.value.code == cc.cc.CC_ECORRUPT
    np.testing.assert_array_equal(pool.labels(c).cpu().numpy(), ref.labels())
    assert pool.sync() == cc.cc.CC_OK
    pool.close()
    # the rank bits limit each graph to 2^27 vertices, not the arena
    big = cc.Pool((1 << 27) + 2, 2, hook=2)
    with pytest.raises(cc.CCError) as ei:
        big.add((1 << 27) + 1)
    assert ei.value.code == cc.cc.CC_EINVAL
    h = big.add(1 << 27)
    k = big.add(2)
    big.run([(k, cc.UPDATE, dev([[0, 1]]), None), (h, cc.UPDATE, dev([[0, (1 << 27) - 1], [5, 6]]), None)])
    assert big.num_components(k) == 1 and big.num_components(h) == (1 << 27) - 2
    lab = big.labels(h)
    assert int(lab[(1 << 27) - 1]) == 0 and int(lab[6]) == 5
    big.close()


def test_prepared_ops_rerun_with_new_contents(cc):
    """A prepared operation list is submitted twice; between the runs the
    pool is reset and the item tensors get new contents in place."""
    G, n, m, q = 6, 500, 700, 300
    pool = cc.Pool(G * n, G, hook=2)
    ids = [pool.add(n) for _ in range(G)]
    E = [torch.empty((m, 2), dtype=torch.int32, device="cuda") for _ in range(G)]
    Q = [torch.empty((q, 2), dtype=torch.int32, device="cuda") for _ in range(G)]
    O = [torch.empty(q, dtype=torch.uint8, device="cuda") for _ in range(G)]
    prep = pool.prepare([(ids[g], cc.UPDATE, E[g], None) for g in range(G)] +
                        [(ids[g], cc.QUERY, Q[g], O[g]) for g in range(G)])
    for run in range(2):
        pool.reset_all()
        refs = []
        for g in range(G):
            e = synth.uniform_pairs(synth.key(41, g, 2 * run), 0, m, n)
            qq = synth.uniform_pairs(synth.key(41, g, 2 * run + 1), 0, q, n)
            E[g].copy_(torch.from_numpy(e))
            Q[g].copy_(torch.from_numpy(qq))
            ref = oracle.UnionFind(n)
            ref.bulk_update(e)
            refs.append(ref.bulk_query(qq))
        pool.run(prep)
        for g in range(G):
            np.testing.assert_array_equal(O[g].cpu().numpy(), refs[g], err_msg="run %d graph %d" % (run, g))
    assert pool.sync() == cc.cc.CC_OK
    pool.close()


def test_overlapping_one_launch_runs_on_two_streams(cc):
    """Runs of the one-launch form issued back to back on two streams (as the
    serving executor does) each keep their own barrier and never run at the
    same time; every answer equals the oracle's."""
    G = 32
    streams = small_graphs(G, seed=13)
    half = G // 2
    sts = [torch.cuda.Stream(), torch.cuda.Stream()]
    pool = cc.Pool(sum(s.n for s in streams), G, one_launch=1, hook=2, compress_linked=0)
    ids = [pool.add(s.n) for s in streams]
    torch.cuda.synchronize()
    outs = [torch.zeros(len(s.queries), dtype=torch.uint8, device="cuda") for s in streams]
    E = [dev(s.edges) for s in streams]
    Q = [dev(s.queries) for s in streams]
    for k in range(4):
        for part in range(2):
            gs = range(part * half, (part + 1) * half)
            ops = [(ids[g], cc.UPDATE, E[g][int(streams[g].eoff[k]):int(streams[g].eoff[k + 1])], None) for g in gs]
            ops += [(ids[g], cc.QUERY, Q[g][int(streams[g].qoff[k]):int(streams[g].qoff[k + 1])],
                     outs[g][int(streams[g].qoff[k]):int(streams[g].qoff[k + 1])]) for g in gs]
            pool.set_stream(sts[part])
            pool.run(ops)
    torch.cuda.synchronize()
    pool.set_stream(torch.cuda.current_stream())  # labels below are read on the current stream
    for g, s in enumerate(streams):
        ref = oracle.UnionFind(s.n)
        want = []
        for k in range(4):
            ref.bulk_update(s.batch(k))
            want.append(ref.bulk_query(s.query(k)))
        np.testing.assert_array_equal(outs[g].cpu().numpy(), np.concatenate(want), err_msg="graph %d" % g)
        np.testing.assert_array_equal(pool.labels(ids[g]).cpu().numpy(), ref.labels(), err_msg="graph %d" % g)
    assert pool.sync() == cc.cc.CC_OK
    pool.close()


@pytest.mark.parametrize("hook", [0, 2])
def test_pool_filter_cleared_with_the_forest(cc, hook):
    """The pool's membership bits claim connectivity to an anchor; every
    operation that replaces a graph's forest (reset, reset_all, remove and
    add over the same range, load, turning the filter back on) must drop
    them, or a query would answer 1 for vertices the new forest keeps apart."""
    n = 4000
    pool = cc.Pool(2 * n + 100, 4, hook=hook, filter=1)
    a = pool.add(n)
    b = pool.add(n)
    ring = np.stack([np.arange(n), (np.arange(n) + 1) % n], axis=1).astype(np.int32)  # one component
    sparse = synth.uniform_pairs(synth.key(71, 0, 1), 0, n // 4, n)
    q = synth.uniform_pairs(synth.key(71, 0, 2), 0, 3000, n)
    out = torch.empty(len(q), dtype=torch.uint8, device="cuda")

    def ask(g):
        pool.run([(g, cc.QUERY, dev(q), out)])
        return out.cpu().numpy().copy()

    def fill(g):
        # twice, so that the second pass finds the tree joined and sets bits
        pool.run([(g, cc.UPDATE, dev(ring), None)])
        pool.run([(g, cc.UPDATE, dev(ring), None)])
        assert ask(g).all()

    ref = oracle.UnionFind(n)
    ref.bulk_update(sparse)
    want_sparse = ref.bulk_query(q)
    want_alone = (q[:, 0] == q[:, 1]).astype(np.uint8)
    pool.run([(b, cc.UPDATE, dev(sparse), None)])
    img = pool.save(b)
    # reset
    fill(a)
    pool.reset(a)
    np.testing.assert_array_equal(ask(a), want_alone)
    # reset_all
    fill(a)
    pool.reset_all()
    np.testing.assert_array_equal(ask(a), want_alone)
    # load over a filled graph
    fill(a)
    pool.load(a, img)
    np.testing.assert_array_equal(ask(a), want_sparse)
    pool.run([(a, cc.UPDATE, dev(sparse), None)])
    np.testing.assert_array_equal(ask(a), want_sparse)
    # remove, then a new graph over the same slots
    fill(a)
    pool.remove(a)
    c = pool.add(n)
    np.testing.assert_array_equal(ask(c), want_alone)
    # bits left from before the filter was turned off
    fill(c)
    pool.set_option("filter", 0)
    pool.reset(c)
    pool.set_option("filter", 1)
    np.testing.assert_array_equal(ask(c), want_alone)
    pool.run([(c, cc.UPDATE, dev(sparse), None)])
    np.testing.assert_array_equal(ask(c), want_sparse)
    assert pool.sync() == cc.cc.CC_OK
    with pytest.raises(cc.CCError) as ei:
        pool.set_option("filter", 2)
    assert ei.value.code == cc.cc.CC_EINVAL
    pool.close()


@pytest.mark.parametrize("items", [2, 4, 8])
def test_one_launch_full_grid_is_resident(cc, items):
    """The one-launch form over many more tiles than the grid holds, with the
    small register footprints of 2 and 4 items per thread: the cooperative
    grid must become resident at once (a grid sized to the occupancy
    calculator's 8 wavefronts per SIMD took seconds per launch), and every
    answer equals the oracle's."""
    import time
    G, n = 64, 1 << 14
    ks = [synth.key(83, g, 1) for g in range(G)]
    E = [synth.uniform_pairs(k, 0, 8 * n, n) for k in ks]
    Qh = [synth.uniform_pairs(k, 8 * n, 512, n) for k in ks]
    pool = cc.Pool(G * n, G, one_launch=1, hook=2, compress_linked=0, block=512, items=items)
    ids = [pool.add(n) for _ in range(G)]
    Ed = [dev(e) for e in E]
    Qd = [dev(q) for q in Qh]
    outs = [torch.zeros(len(q), dtype=torch.uint8, device="cuda") for q in Qh]
    ops = [(ids[g], cc.UPDATE, Ed[g][: 4 * n], None) for g in range(G)]
    ops += [(ids[g], cc.UPDATE, Ed[g][4 * n:], None) for g in range(G)]
    ops += [(ids[g], cc.QUERY, Qd[g], outs[g]) for g in range(G)]
    prep = pool.prepare(ops)
    pool.run(prep)  # first launch: module load and allocations
    torch.cuda.synchronize()
    pool.reset_all()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    pool.run(prep)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    print("items %d: one-launch run of %d edges in %.2f ms" % (items, G * 8 * n, dt * 1e3), flush=True)
    assert pool.sync() == cc.cc.CC_OK
    for g in range(G):
        ref = oracle.UnionFind(n)
        ref.bulk_update(E[g])
        np.testing.assert_array_equal(outs[g].cpu().numpy(), ref.bulk_query(Qh[g]), err_msg="graph %d" % g)
    assert dt < 1.0, "one-launch run took %.2f s: the cooperative grid was not resident at once" % dt
    pool.close()
