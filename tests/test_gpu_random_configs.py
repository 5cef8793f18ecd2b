"""Seeded sweep over option combinations and workload shapes: every answer,
label and count bit-exact against the oracle.  Each case prints its seed and
options before it runs."""
import numpy as np
import pytest
import torch

import oracle
import synth

pytestmark = pytest.mark.gpu

SCHEDULES = [dict(update_mode=0), dict(update_mode=1), dict(update_mode=2), dict(find=1), dict(find=2)]


def case_options(rng):
    o = dict(SCHEDULES[int(rng.integers(len(SCHEDULES)))])
    hooks = [0, 1] if o.get("update_mode", 0) != 0 else [0, 1, 2]
    o["hook"] = int(rng.choice(hooks))
    o["block"] = int(rng.choice([64, 128, 256, 512, 1024]))
    o["items"] = int(rng.choice([0, 1, 2, 4, 8]))
    o["grid_cap"] = int(rng.choice([1, 2, 7, 64, 4096]))
    o["query_halving"] = int(rng.integers(2))
    o["compress_linked"] = int(rng.integers(2))
    o["compress_every"] = int(rng.choice([0, 0, 1, 3]))
    return o


def filter_option(seed):
    """Drawn from its own generator so the other options of a seed stay as
    they were before the filter existed."""
    return int(np.random.default_rng(seed + 7919).integers(3))


def query_items_option(seed):
    """Likewise for the query's own items per thread."""
    return int(np.random.default_rng(seed + 104729).choice([0, 0, 1, 2, 4, 8]))


def case_stream(rng, seed):
    kind = int(rng.integers(5))
    if kind == 0:
        n = int(rng.choice([1, 2, 17, 1000, 1 << 12]))
        sizes = [int(x) for x in rng.integers(0, 3 * n + 2, size=int(rng.integers(1, 6)))]
        e = synth.uniform_pairs(synth.key(seed, 0, 1), 0, sum(sizes), n)
        q = synth.uniform_pairs(synth.key(seed, 0, 2), 0, 300 * len(sizes), n)
        return synth.Stream("uniform", n, e, synth._offsets(sizes), q, synth._offsets([300] * len(sizes)))
    if kind == 1:
        return synth.rmat_stream(scale=int(rng.integers(8, 15)), size_lo=6, size_hi=13, qbatch=512,
                                 seed=seed, probes=0)
    if kind == 2:
        W = int(rng.integers(2, 90))
        return synth.grid_stream_cfg(W=W, H=int(rng.integers(1, 90)), batch=int(rng.choice([16, 500, 4096])),
                                     qbatch=128, probes=0)
    if kind == 3:
        return synth.grid3d_stream_cfg(L=int(rng.integers(2, 20)), batch=int(rng.choice([64, 1000])), qbatch=128,
                                       probes=0)
    return synth.local_stream(n=int(rng.choice([100, 5000, 1 << 14])), degree=int(rng.choice([1, 5, 16])),
                              window=int(rng.choice([1, 64, 1 << 10])), batch=int(rng.choice([64, 4096])),
                              qbatch=256, probes=0)


@pytest.fixture(scope="module")
def cc():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1602_05232_amd as ccgpu
    ccgpu.lib()
    return ccgpu


@pytest.mark.parametrize("seed", range(200))
def test_random_config(cc, seed):
    rng = np.random.default_rng(1000 + seed)
    opts = case_options(rng)
    opts["filter"] = filter_option(seed)
    opts["query_items"] = query_items_option(seed)
    s = case_stream(rng, 7000 + seed)
    print("case %d: %s n=%d edges=%d batches=%d opts=%s" % (seed, s.name, s.n, len(s.edges), s.num_batches, opts),
          flush=True)
    ref = oracle.UnionFind(s.n)
    g = cc.Graph(s.n, **opts)
    for i in range(s.num_batches):
        b, q = s.batch(i), s.query(i)
        ref.bulk_update(b)
        g.bulk_update(torch.from_numpy(np.ascontiguousarray(b)).cuda())
        if len(q):
            got = g.bulk_query(torch.from_numpy(np.ascontiguousarray(q)).cuda()).cpu().numpy()
            np.testing.assert_array_equal(got, ref.bulk_query(q), err_msg="answers after minibatch %d" % i)
    np.testing.assert_array_equal(g.labels().cpu().numpy(), ref.labels())
    assert g.num_components() == ref.num_components() == g.count_roots()
    assert g.sync() == cc.cc.CC_OK
    g.close()


def pool_options(rng):
    return dict(hook=int(rng.integers(3)), block=int(rng.choice([64, 256, 1024])),
                items=int(rng.choice([0, 1, 2, 4, 8])), grid_cap=int(rng.choice([1, 3, 64, 4096])),
                query_halving=int(rng.integers(2)), compress_linked=int(rng.integers(2)),
                one_launch=int(rng.integers(2)))


@pytest.mark.parametrize("seed", list(range(60)) + [140])  # 140: rank links on a 3-vertex graph in one block
def test_random_pool_config(cc, seed):
    """Random graph mixes in one pool, several operations per graph in one
    run (so runs have several rounds), against one oracle per graph."""
    rng = np.random.default_rng(5000 + seed)
    opts = pool_options(rng)
    # the pool's membership filter, from a generator of its own so that the
    # other draws of a seed stay as they were before the option existed
    opts["filter"] = int(np.random.default_rng(seed + 15485863).integers(2))
    G = int(rng.integers(1, 40))
    ns = [int(x) for x in rng.integers(1, 3000, size=G)]
    print("pool case %d: G=%d sum_n=%d opts=%s" % (seed, G, sum(ns), opts), flush=True)
    pool = cc.Pool(sum(ns) + int(rng.integers(0, 100)), G, **opts)
    ids = [pool.add(n) for n in ns]
    refs = [oracle.UnionFind(n) for n in ns]
    for run in range(int(rng.integers(1, 4))):
        ops, checks = [], []
        for g in rng.permutation(G):
            g = int(g)
            for k in range(int(rng.integers(0, 4))):
                if rng.random() < 0.6:
                    e = synth.uniform_pairs(synth.key(9000 + seed, g, 10 * run + k), 0,
                                            int(rng.integers(0, 4 * ns[g] + 2)), ns[g])
                    refs[g].bulk_update(e)
                    ops.append((ids[g], cc.UPDATE, torch.from_numpy(e).cuda(), None))
                else:
                    q = synth.uniform_pairs(synth.key(9100 + seed, g, 10 * run + k), 0, int(rng.integers(0, 500)), ns[g])
                    out = torch.empty(len(q), dtype=torch.uint8, device="cuda")
                    ops.append((ids[g], cc.QUERY, torch.from_numpy(q).cuda(), out))
                    checks.append((out, refs[g].bulk_query(q), g))
        pool.run(ops)
        for out, want, g in checks:
            np.testing.assert_array_equal(out.cpu().numpy(), want, err_msg="graph %d, run %d" % (g, run))
    for g in range(G):
        np.testing.assert_array_equal(pool.labels(ids[g]).cpu().numpy(), refs[g].labels(), err_msg="graph %d" % g)
        assert pool.num_components(ids[g]) == refs[g].num_components()
    assert pool.sync() == cc.cc.CC_OK
    pool.close()


@pytest.mark.parametrize("n", [2, 3, 4, 5, 8])
def test_rank_links_contend_on_tiny_graphs(cc, n):
    """Union by rank with thousands of edges on a few vertices in one block
    (plain launches, the one-launch stream form, pools): a link retried after
    lost CAS races must not be taken for a cycle (its step bound counts links
    and rank increments, not only vertices)."""
    print("tiny rank contention: n=%d" % n, flush=True)
    g = cc.Graph(n, hook=2, block=1024, items=2, grid_cap=1, compress_linked=1)
    for rep in range(100):
        g.reset()
        e = synth.uniform_pairs(synth.key(321, n, rep), 0, 2048, n)
        ref = oracle.UnionFind(n)
        ref.bulk_update(e)
        g.bulk_update(torch.from_numpy(e).cuda())
        np.testing.assert_array_equal(g.labels().cpu().numpy(), ref.labels(), err_msg="rep %d" % rep)
        assert g.sync() == cc.cc.CC_OK, "rep %d" % rep
    # the one-launch stream form: four minibatches and their queries per launch
    for rep in range(20):
        g.reset()
        e = synth.uniform_pairs(synth.key(987, n, rep), 0, 4 * 1024, n)
        q = synth.uniform_pairs(synth.key(988, n, rep), 0, 4 * 64, n)
        eo = torch.arange(0, 4 * 1024 + 1, 1024, dtype=torch.int64, device="cuda")
        qo = torch.arange(0, 4 * 64 + 1, 64, dtype=torch.int64, device="cuda")
        out = torch.empty(len(q), dtype=torch.uint8, device="cuda")
        g.bulk_stream(torch.from_numpy(e).cuda(), eo, torch.from_numpy(q).cuda(), qo, out)
        ref = oracle.UnionFind(n)
        want = []
        for b in range(4):
            ref.bulk_update(e[1024 * b:1024 * (b + 1)])
            want.append(ref.bulk_query(q[64 * b:64 * (b + 1)]))
        np.testing.assert_array_equal(out.cpu().numpy(), np.concatenate(want), err_msg="stream rep %d" % rep)
        np.testing.assert_array_equal(g.labels().cpu().numpy(), ref.labels(), err_msg="stream rep %d" % rep)
        assert g.sync() == cc.cc.CC_OK, "stream rep %d" % rep
    g.close()
    for one_launch in (0, 1):
        pool = cc.Pool(64 * n, 64, hook=2, block=1024, items=2, grid_cap=1, one_launch=one_launch)
        ids = [pool.add(n) for _ in range(64)]
        for rep in range(20):
            pool.reset_all()
            ops, refs = [], []
            for k, gid in enumerate(ids):
                e = synth.uniform_pairs(synth.key(654, 64 * rep + k, n), 0, 256, n)
                ref = oracle.UnionFind(n)
                ref.bulk_update(e)
                refs.append(ref)
                ops.append((gid, cc.UPDATE, torch.from_numpy(e).cuda(), None))
            pool.run(ops)
            for gid, ref in zip(ids, refs):
                np.testing.assert_array_equal(pool.labels(gid).cpu().numpy(), ref.labels())
            assert pool.sync() == cc.cc.CC_OK, "one_launch %d rep %d" % (one_launch, rep)
        pool.close()
