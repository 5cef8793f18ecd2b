"""Parity of the HIP path (through the C ABI) with the CPU oracle.

Bit-exact on every query answer byte, every min-id label and the component
count, after every minibatch unless stated otherwise.  Inputs come from the
seeded generators; expected values only from the oracle.
"""
import numpy as np
import pytest
import torch

import oracle
import synth

pytestmark = pytest.mark.gpu

OPTION_SETS = [
    dict(update_mode=0, hook=0),
    dict(update_mode=1, hook=0),
    dict(update_mode=0, hook=1),
    dict(update_mode=1, hook=1),
    dict(update_mode=0, block=64, items=1, grid_cap=7, compress_linked=0),
    dict(update_mode=1, block=1024, items=8, grid_cap=3),
    dict(update_mode=0, query_halving=0, compress_every=3, items=2, compress_linked=0),
    dict(update_mode=0, hook=1, items=8, block=512, grid_cap=5),
    dict(update_mode=0, hook=2),
    dict(update_mode=0, hook=2, compress_linked=0, items=8, query_halving=0, compress_every=2),
    dict(update_mode=2),
    dict(update_mode=2, hook=1, grid_cap=3),
    dict(update_mode=2, query_halving=0, compress_every=2),
    dict(find=1, grid_cap=3),
    dict(find=1, hook=1, grid_cap=16),
    dict(find=1),
    dict(find=1, hook=2),
    dict(find=2),
    dict(find=2, hook=1, grid_cap=3),
    dict(find=2, hook=2, grid_cap=16),
    dict(update_mode=0, filter=2),
    dict(update_mode=0, hook=1, filter=1, items=8, grid_cap=5),
    dict(update_mode=0, hook=2, filter=1, compress_linked=0),
    dict(update_mode=0, hook=2, filter=2, block=64, items=1, query_halving=0, compress_every=2),
    dict(update_mode=1, filter=2),
    dict(update_mode=0, hook=2, filter=2, items=1, query_items=4, block=512, grid_cap=768, compress_linked=0),
    dict(update_mode=0, query_items=8, block=128),
    dict(update_mode=1, hook=2),
    dict(update_mode=1, hook=2, items=8, block=256, query_halving=0),
    dict(update_mode=0, split_below=100, hook=2),
    dict(update_mode=0, split_below=60, hook=0, compress_linked=0),
    dict(update_mode=0, split_below=100, hook=1, filter=2),
    dict(find=1, hook=2, filter=2),
    dict(find=1, hook=1, filter=1, grid_cap=5),
    dict(find=2, hook=2, filter=2, grid_cap=16),
    dict(find=2, hook=0, filter=2),
]


def opt_id(o):
    return ",".join("%s=%s" % kv for kv in sorted(o.items()))


@pytest.fixture(scope="module")
def cc():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1602_05232_amd as ccgpu  # raises if libcc.so is missing
    ccgpu.lib()
    return ccgpu


def dev(a):
    a = np.asarray(a)
    if a.dtype != np.int32:
        a = a.astype(np.int32)
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def run_parity(cc, s, opts, label_every=1, check_roots=True):
    """Stream s through the GPU graph and the oracle side by side."""
    print("parity: %s n=%d batches=%d opts=%s" % (s.name, s.n, s.num_batches, opts), flush=True)
    ref = oracle.UnionFind(s.n)
    g = cc.Graph(s.n, **opts)
    edges, queries = dev(s.edges), dev(s.queries)
    probes = dev(s.probes) if len(s.probes) else None
    out = torch.empty(len(s.queries), dtype=torch.uint8, device="cuda")
    want = np.empty(len(s.queries), np.uint8)
    prev = np.zeros(len(s.probes), np.uint8)
    nb = s.num_batches
    for i in range(nb):
        e0, e1 = int(s.eoff[i]), int(s.eoff[i + 1])
        q0, q1 = int(s.qoff[i]), int(s.qoff[i + 1])
        ref.bulk_update(s.edges[e0:e1])
        g.bulk_update(edges[e0:e1])
        want[q0:q1] = ref.bulk_query(s.queries[q0:q1])
        g.bulk_query(queries[q0:q1], out=out[q0:q1])
        if probes is not None:
            pa = g.bulk_query(probes).cpu().numpy()
            np.testing.assert_array_equal(pa, ref.bulk_query(s.probes))
            assert (pa >= prev).all()
            prev = pa
        if (label_every and i % label_every == 0) or i == nb - 1:
            lab = g.labels().cpu().numpy()
            np.testing.assert_array_equal(lab, ref.labels(), err_msg="labels after minibatch %d" % i)
            assert g.num_components() == ref.num_components()
            if check_roots:
                assert g.count_roots() == ref.num_components()
    np.testing.assert_array_equal(out.cpu().numpy(), want)
    assert g.sync() == cc.cc.CC_OK
    g.close()
    return ref


@pytest.mark.parametrize("opts", OPTION_SETS, ids=opt_id)
def test_er_tiny(cc, opts):
    run_parity(cc, synth.er_stream(), opts)


@pytest.mark.parametrize("opts", OPTION_SETS, ids=opt_id)
def test_rmat_small(cc, opts):
    run_parity(cc, synth.rmat_stream(scale=16, size_lo=8, size_hi=16, qbatch=1 << 12), opts)


@pytest.mark.parametrize("opts", OPTION_SETS[:4] + [dict(update_mode=2), dict(update_mode=2, hook=1)]
                         + OPTION_SETS[-2:], ids=opt_id)
def test_grid_small(cc, opts):
    s = synth.grid_stream_cfg(W=256, H=256, batch=1 << 12, qbatch=1 << 10)
    ref = run_parity(cc, s, opts, label_every=4)
    assert ref.num_components() >= 1


@pytest.mark.parametrize("which", ["grid3d", "local"])
@pytest.mark.parametrize("opts", [dict(), dict(hook=2), dict(update_mode=1), dict(update_mode=2)], ids=opt_id)
def test_more_workload_shapes(cc, which, opts):
    if which == "grid3d":
        s = synth.grid3d_stream_cfg(L=40, batch=1 << 13, qbatch=1 << 10)
    else:
        s = synth.local_stream(n=1 << 16, degree=5, window=1 << 10, batch=1 << 15, qbatch=1 << 10)
    run_parity(cc, s, opts, label_every=3)


@pytest.mark.parametrize("mode", [0, 1, 2])
def test_ragged_sizes(cc, mode):
    sizes = [1, 63, 64, 65, 255, 257, 1023, 1025, 4095, 4097, 0, 3, 12289]
    n = 5000
    m = sum(sizes)
    e = synth.uniform_pairs(synth.key(11, 0, 1), 0, m, n)
    q = synth.uniform_pairs(synth.key(11, 0, 2), 0, 997 * len(sizes), n)
    s = synth.Stream("ragged", n, e, synth._offsets(sizes), q, synth._offsets([997] * len(sizes)))
    run_parity(cc, s, dict(update_mode=mode, items=4, block=256))


@pytest.mark.parametrize("mode", [0, 1, 2])
def test_edge_cases(cc, mode):
    n = 1 << 12
    g = cc.Graph(n, update_mode=mode)
    ref = oracle.UnionFind(n)

    def both(e):
        e = np.asarray(e, np.int32).reshape(-1, 2)
        ref.bulk_update(e)
        g.bulk_update(dev(e))

    both(np.empty((0, 2)))  # empty minibatch
    both(np.stack([np.arange(n), np.arange(n)], 1))  # all self-loops
    assert g.num_components() == n
    both(np.tile([[5, 9]], (1 << 16, 1)))  # one edge repeated
    assert g.num_components() == n - 1
    star = [(100, 100 + k) for k in range(1, 8)]  # the Section 4.2 star
    both(star)
    lab = g.labels().cpu().numpy()
    np.testing.assert_array_equal(lab, ref.labels())
    assert (lab[100:108] == 100).all()
    assert g.sync() == cc.cc.CC_OK
    # (u, u) queries answer 1 even for isolated vertices
    a = g.bulk_query(dev([[7, 7], [4000, 4000], [5, 9], [9, 5], [5, 6]])).cpu().numpy()
    np.testing.assert_array_equal(a, [1, 1, 1, 1, 0])
    g.close()


@pytest.mark.parametrize("opts", [dict(update_mode=0), dict(update_mode=1), dict(update_mode=0, hook=1),
                                  dict(update_mode=0, hook=2), dict(update_mode=2), dict(update_mode=2, hook=1),
                                  dict(find=1), dict(find=1, hook=2), dict(find=2), dict(find=2, hook=2)],
                         ids=opt_id)
def test_deep_chain(cc, opts):
    # reversed path in one minibatch, then in single-edge minibatches
    n = 1 << 20
    i = np.arange(n - 2, -1, -1, dtype=np.int32)
    g = cc.Graph(n, **opts)
    g.bulk_update(dev(np.stack([i, i + 1], 1)))
    assert g.num_components() == 1
    assert (g.labels().cpu().numpy() == 0).all()
    g.close()
    n = 1 << 12
    g = cc.Graph(n, **opts)
    i = np.arange(n - 2, -1, -1, dtype=np.int32)
    e = dev(np.stack([i + 1, i], 1))
    for k in range(n - 1):
        g.bulk_update(e[k:k + 1])
    assert g.num_components() == 1
    q = dev(np.stack([np.zeros(n, np.int32), np.arange(n, dtype=np.int32)], 1))
    assert g.bulk_query(q).cpu().numpy().all()
    assert g.sync() == cc.cc.CC_OK
    g.close()


@pytest.mark.parametrize("mode", [0, 1, 2])
def test_invalid_ids(cc, mode):
    n = 10
    g = cc.Graph(n, update_mode=mode)
    ref = oracle.UnionFind(n)
    e = np.array([(0, 1), (-1, 2), (2, 10), (3, 4), (11, -5), (4, 5)], np.int32)
    ref.bulk_update(e)
    g.bulk_update(dev(e))
    assert g.sync() == cc.cc.CC_ERANGE
    assert g.sync() == cc.cc.CC_OK  # reported once
    assert g.num_components() == ref.num_components() == n - 3
    p = np.array([(0, 1), (3, 5), (0, 10), (-1, -1), (7, 7), (1, 3)], np.int32)
    np.testing.assert_array_equal(g.bulk_query(dev(p)).cpu().numpy(), ref.bulk_query(p))
    assert g.sync() == cc.cc.CC_ERANGE
    np.testing.assert_array_equal(g.labels().cpu().numpy(), ref.labels())
    g.close()


def test_argument_errors(cc):
    g = cc.Graph(16)
    L = cc.lib()
    assert L.cc_set_option(g.handle, 6, 3) == cc.cc.CC_EINVAL
    g2 = cc.Graph(16, hook=2, update_mode=2)  # rank linking does not run with the contracting schedule
    assert L.cc_bulk_update(g2.handle, g2.handle, 0) == cc.cc.CC_OK
    with pytest.raises(cc.CCError):
        g2.bulk_update(dev([[1, 2]]))
    assert g2.num_components() == 16
    g2.close()
    assert L.cc_set_option(g.handle, 14, 101) == cc.cc.CC_EINVAL  # compaction threshold is a percentage
    assert L.cc_set_option(g.handle, 14, -1) == cc.cc.CC_EINVAL
    assert L.cc_set_option(g.handle, 1, 3) == cc.cc.CC_EINVAL
    assert L.cc_bulk_update(g.handle, None, 3) == cc.cc.CC_EINVAL
    assert L.cc_bulk_update(g.handle, None, -1) == cc.cc.CC_EINVAL
    assert L.cc_bulk_query(g.handle, None, 2, None) == cc.cc.CC_EINVAL
    assert L.cc_set_option(g.handle, 2, 100) == cc.cc.CC_EINVAL
    assert L.cc_set_option(g.handle, 99, 1) == cc.cc.CC_EINVAL
    assert g.sync() == cc.cc.CC_OK
    g.close()


def test_misaligned_item_arrays_are_rejected(cc):
    """Edge and pair arrays are read one 8-byte pair per load: an array that
    does not start on an 8-byte boundary is an argument error at every entry
    point, and nothing runs."""
    import ctypes
    from paper_1602_05232_amd import cc as ccmod
    L = cc.lib()
    g = cc.Graph(16)
    buf = torch.arange(10, dtype=torch.int32, device="cuda")
    bad = ctypes.c_void_p(buf.data_ptr() + 4)
    good = ctypes.c_void_p(buf.data_ptr())
    out = torch.zeros(8, dtype=torch.uint8, device="cuda")
    eo = torch.tensor([0, 4], dtype=torch.int64, device="cuda")
    assert L.cc_bulk_update(g.handle, bad, 4) == cc.cc.CC_EINVAL
    assert L.cc_bulk_query(g.handle, bad, 4, out.data_ptr()) == cc.cc.CC_EINVAL
    assert L.cc_bulk_stream(g.handle, 1, bad, eo.data_ptr(), good, eo.data_ptr(), out.data_ptr(), 4) == \
        cc.cc.CC_EINVAL
    assert L.cc_bulk_stream(g.handle, 1, good, eo.data_ptr(), bad, eo.data_ptr(), out.data_ptr(), 4) == \
        cc.cc.CC_EINVAL
    with pytest.raises(ValueError):
        g.bulk_update(buf[1:9].view(4, 2))
    assert g.num_components() == 16
    assert g.sync() == cc.cc.CC_OK
    g.close()
    pool = cc.Pool(32, 2)
    gid = pool.add(16)
    ops = (ccmod.CcOp * 1)()
    ops[0].graph, ops[0].kind, ops[0].count, ops[0].items, ops[0].out = gid, 0, 4, bad.value, None
    assert L.cc_pool_run(pool._h, ops, 1) == cc.cc.CC_EINVAL
    with pytest.raises(ValueError):
        pool.run([(gid, cc.UPDATE, buf[1:9].view(4, 2), None)])
    assert pool.num_components(gid) == 16
    assert pool.sync() == cc.cc.CC_OK
    pool.close()


def test_linking_order_is_fixed_until_reset(cc):
    """Rank bits live in root words and the label passes assume one order, so
    the order may change only on a fresh forest; a rejected update leaves the
    graph fresh."""
    s = synth.rmat_stream(scale=12, size_lo=6, size_hi=11, qbatch=256)
    g = cc.Graph(s.n, hook=2, update_mode=2)
    with pytest.raises(cc.CCError):
        g.bulk_update(dev(s.batch(0)))  # rank does not run with the contracting schedule: nothing runs
    g.set_option("hook", 1)  # still fresh
    g.set_option("update_mode", 0)
    ref = oracle.UnionFind(s.n)
    ref.bulk_update(s.batch(0))
    g.bulk_update(dev(s.batch(0)))
    for h in (0, 2):
        with pytest.raises(cc.CCError) as ei:
            g.set_option("hook", h)
        assert ei.value.code == cc.cc.CC_EINVAL
    g.set_option("hook", 1)  # the same order is not a change
    np.testing.assert_array_equal(g.labels().cpu().numpy(), ref.labels())
    img = g.save()
    g.reset()
    g.set_option("hook", 2)
    ref = oracle.UnionFind(s.n)
    for i in range(s.num_batches):
        ref.bulk_update(s.batch(i))
        g.bulk_update(dev(s.batch(i)))
    np.testing.assert_array_equal(g.labels().cpu().numpy(), ref.labels())
    g.reset()
    g.set_option("hook", 1)
    g.load(img)  # checked against the hashed order, then fixed
    with pytest.raises(cc.CCError):
        g.set_option("hook", 0)
    g.close()


@pytest.mark.parametrize("hook", [0, 1, 2])
def test_save_load_resume(cc, hook):
    s = synth.rmat_stream(scale=14, size_lo=8, size_hi=13, qbatch=256)
    half = s.num_batches // 2
    a = cc.Graph(s.n, hook=hook)
    for i in range(half):
        a.bulk_update(dev(s.batch(i)))
    img = a.save()
    b = cc.Graph(s.n, hook=hook, update_mode=1 if hook != 2 else 0)
    b.load(img)
    assert b.num_components() == a.num_components()
    for i in range(half, s.num_batches):
        a.bulk_update(dev(s.batch(i)))
        b.bulk_update(dev(s.batch(i)))
    np.testing.assert_array_equal(a.labels().cpu().numpy(), b.labels().cpu().numpy())
    ref = oracle.UnionFind(s.n)
    ref.bulk_update(s.edges)
    np.testing.assert_array_equal(b.labels().cpu().numpy(), ref.labels())
    # a cycle in the image is rejected and leaves the graph unchanged
    bad = bytearray(img)
    par = np.frombuffer(bad, np.int32, offset=16)
    par[3], par[4] = 4, 3
    before = b.labels().cpu().numpy()
    with pytest.raises(cc.CCError) as ei:
        b.load(bad)
    assert ei.value.code == cc.cc.CC_ECORRUPT
    np.testing.assert_array_equal(b.labels().cpu().numpy(), before)
    a.close()
    b.close()


def test_order_independence_and_reset(cc):
    s = synth.rmat_stream(scale=15, size_lo=10, size_hi=15, qbatch=16)
    rng = np.random.default_rng(3)
    g = cc.Graph(s.n)
    g.bulk_update(dev(s.edges))
    want = g.labels().cpu().numpy()
    for mode in (0, 1, 2):
        g.set_option("update_mode", mode)
        g.reset()
        assert g.num_components() == s.n
        e = s.edges[rng.permutation(len(s.edges))][:, ::-1]
        for b in np.array_split(e, 5):
            g.bulk_update(dev(b))
        np.testing.assert_array_equal(g.labels().cpu().numpy(), want)
    g.close()


@pytest.mark.parametrize("find", [1, 2], ids=["jumping", "response-distributor"])
def test_bulk_find_worked_example(cc, find):
    """Section 5's example: a tree rooted at 19 in which the finds of 1 and 7
    meet at 4 (1 -> 2 -> 4 and 7 -> 8 -> 9 -> 4) and the find of 3 joins 1's
    flow at 2.  After Bulk-Find of {1, 3, 4, 7} every traversed vertex points
    straight at the root (Phase II).  The figure's full tree is not in the
    text; the fragment given there is used, with 4 -> 19.  Loaded as a rank
    forest image, which accepts any acyclic parent array."""
    n = 24
    par = np.arange(n, dtype=np.int32)
    for c, p in ((1, 2), (3, 2), (2, 4), (7, 8), (8, 9), (9, 4), (4, 19)):
        par[c] = p
    img = bytearray(np.array([n, 7], np.int64).tobytes() + par.tobytes())
    g = cc.Graph(n, hook=2, find=find)
    g.load(img)
    ans = g.bulk_query(dev([[1, 3], [4, 7], [1, 19], [5, 19]])).cpu().numpy()
    np.testing.assert_array_equal(ans, [1, 1, 1, 0])
    after = np.frombuffer(bytes(g.save()), np.int32, offset=16) & ((1 << 27) - 1)
    for v in (1, 2, 3, 4, 7, 8, 9):
        assert after[v] == 19, (v, after[v])
    assert after[5] == 5 and after[19] == 19
    assert g.sync() == cc.cc.CC_OK
    g.close()


@pytest.mark.parametrize("opts", [dict(find=1), dict(find=1, grid_cap=5), dict(find=1, hook=2, grid_cap=64),
                                  dict(find=2), dict(find=2, grid_cap=5), dict(find=2, hook=2, grid_cap=64)],
                         ids=opt_id)
def test_bulk_find_wide_levels(cc, opts):
    """Minibatches large enough that Bulk-Find's levels are appended in
    per-block chunks (more than blockDim.x entries per block), on forests
    deep enough to need several levels: a long path split over the batches
    plus uniform random edges."""
    n = 1 << 20
    rng = np.random.default_rng(7)
    path = np.stack([np.arange(n - 1), np.arange(1, n)], 1).astype(np.int32)[rng.permutation(n - 1)]
    rand = synth.uniform_pairs(synth.key(29, 0, 1), 0, 1 << 20, n)
    edges = np.concatenate([path[: n // 2], rand, path[n // 2:]])
    sizes = [1 << 18, 1 << 19, 1 << 20, len(edges) - (1 << 18) - (1 << 19) - (1 << 20)]
    q = synth.uniform_pairs(synth.key(29, 0, 2), 0, (1 << 19) * len(sizes), n)
    s = synth.Stream("wide", n, edges, synth._offsets(sizes), q, synth._offsets([1 << 19] * len(sizes)))
    run_parity(cc, s, opts)


@pytest.mark.parametrize("opts", [dict(find=2), dict(find=2, grid_cap=1), dict(find=2, grid_cap=3),
                                  dict(find=2, hook=2), dict(find=1, grid_cap=3)], ids=opt_id)
def test_bulk_find_hubs(cc, opts):
    """Stars of very different sizes (2^18 leaves down to a few) linked in
    one minibatch, then queried from their leaves while a chain grows under
    the leaves: the response distributor's hub buckets (served by the grid),
    each block's hot parent (counted and placed through shared memory), the
    other buckets of the same blocks, and root entries appended in chunks
    all meet in one call.  Compared with the oracle answer by answer."""
    n = 1 << 20
    rng = np.random.default_rng(11)
    centres = [0, 1, 2, 3, 4]
    sizes = [1 << 18, 1 << 16, 1 << 12, 300, 7]
    leaves = rng.permutation(np.arange(5, n, dtype=np.int32))
    star, at = [], 0
    for c, k in zip(centres, sizes):
        star.append(np.stack([np.full(k, c, np.int32), leaves[at:at + k]], 1))
        at += k
    star = np.concatenate(star)[rng.permutation(sum(sizes))]
    # chains hanging off leaves of every star, and a few random edges
    tail = leaves[at:at + (1 << 16)]
    heads = star[rng.integers(0, len(star), 1 << 16), 1]
    chain = np.stack([heads, tail], 1).astype(np.int32)
    rand = synth.uniform_pairs(synth.key(31, 0, 1), 0, 1 << 14, n)
    edges = np.concatenate([star, chain, rand])
    bsizes = [len(star), len(chain), len(rand)]
    picks = np.concatenate([star[:, 1], tail])
    q = picks[rng.integers(0, len(picks), (3 << 18, 2))].astype(np.int32)
    s = synth.Stream("hubs", n, edges, synth._offsets(bsizes), q, synth._offsets([1 << 18] * 3))
    run_parity(cc, s, opts)


@pytest.mark.parametrize("find", [1, 2], ids=["jumping", "response-distributor"])
def test_bulk_find_compresses_every_endpoint(cc, find):
    s = synth.rmat_stream(scale=15, size_lo=10, size_hi=14, qbatch=1 << 12)
    g = cc.Graph(s.n, find=find, hook=2)
    ref = oracle.UnionFind(s.n)
    for i in range(s.num_batches):
        g.bulk_update(dev(s.batch(i)))
        ref.bulk_update(s.batch(i))
        q = s.query(i)
        np.testing.assert_array_equal(g.bulk_query(dev(q)).cpu().numpy(), ref.bulk_query(q))
        par = np.frombuffer(bytes(g.save()), np.int32, offset=16) & ((1 << 27) - 1)
        ends = np.unique(q)
        assert (par[par[ends]] == par[ends]).all(), "a queried vertex does not point at its root"
    np.testing.assert_array_equal(g.labels().cpu().numpy(), ref.labels())
    g.close()


@pytest.mark.parametrize("opts", [dict(update_mode=0), dict(update_mode=1), dict(update_mode=0, compress_linked=0),
                                  dict(update_mode=2)], ids=opt_id)
def test_id_order_forest_invariants(cc, opts):
    """Under id-order linking every parent pointer goes to a smaller id, so
    each root is its tree's minimum; the number of roots equals n minus the
    successful links; checked on the device state after every minibatch."""
    s = synth.rmat_stream(scale=15, size_lo=9, size_hi=14, qbatch=16)
    g = cc.Graph(s.n, **opts)
    for i in range(s.num_batches):
        g.bulk_update(dev(s.batch(i)))
        par = np.frombuffer(bytes(g.save()), np.int32, offset=16)
        assert (par <= np.arange(s.n)).all()
        roots = int((par == np.arange(s.n)).sum())
        assert roots == g.num_components() == g.count_roots()
    g.close()


@pytest.mark.parametrize("L", [16, 4096])
@pytest.mark.parametrize("opts", [dict(find=0, query_halving=1), dict(find=0, query_halving=0), dict(find=1),
                                  dict(find=2), dict(find=1, grid_cap=3)],
                         ids=["halving", "no-halving", "find1", "find2", "find1-small-grid"])
def test_queries_on_loaded_path_forest(cc, L, opts):
    """Long uncompressed paths that many query ends share (the case of
    Section 5's work bound), loaded as a state image: every answer and every
    label against the oracle fed the same forest as edges."""
    n = 1 << 16
    parent, path = synth.chain_forest(n, L)
    v = np.arange(n, dtype=np.int32)
    kids = parent != v
    ref = oracle.UnionFind(n)
    ref.bulk_update(np.stack([parent[kids], v[kids]], 1))
    k = synth.key(synth.BASE_SEED + 9, 1, synth.P_QUERIES)
    pairs = synth.uniform_pairs(k, 0, 1 << 14, n)
    same = np.argsort(path, kind="stable").astype(np.int32)  # path by path
    pairs = np.concatenate([pairs, np.stack([same[:-1], same[1:]], 1)])  # mostly within one path
    want = ref.bulk_query(pairs)
    assert want.sum() > len(pairs) // 2  # the second half is mostly connected pairs
    g = cc.Graph(n, hook=0, compress_linked=0, **opts)
    img = np.array([n, n - n // L], np.int64).tobytes() + parent.tobytes()
    g.load(img)
    got = g.bulk_query(dev(pairs)).cpu().numpy()
    np.testing.assert_array_equal(got, want)
    np.testing.assert_array_equal(g.labels().cpu().numpy(), ref.labels())
    assert g.num_components() == ref.num_components() == n // L
    assert g.sync() == cc.cc.CC_OK
    g.close()


@pytest.mark.parametrize("opts", [dict(find=1), dict(find=2, hook=2), dict(find=1, hook=2, filter=2)],
                         ids=["find1", "find2-rank", "find1-rank-filter"])
def test_bulk_find_wide_call(cc, opts):
    """One Bulk-Update and one Bulk-Query of 2^20 items each, so that level 0
    runs 2048 blocks and every block of the 256-block cooperative launch
    reads several level-0 segments: every answer and label is the oracle's."""
    n = 1 << 20
    k = synth.key(synth.BASE_SEED + 11, 0, synth.P_EDGES)
    first = synth.rmat_edges(k, 0, 1 << 18, 20, n)
    edges = synth.rmat_edges(k, 1 << 18, 1 << 20, 20, n)
    pairs = synth.uniform_pairs(synth.key(synth.BASE_SEED + 11, 0, synth.P_QUERIES), 0, 1 << 20, n)
    ref = oracle.UnionFind(n)
    g = cc.Graph(n, **opts)
    for e in (first, edges):  # a first call, so that the filter has an anchor for the wide one
        ref.bulk_update(e)
        g.bulk_update(dev(e))
    np.testing.assert_array_equal(g.bulk_query(dev(pairs)).cpu().numpy(), ref.bulk_query(pairs))
    np.testing.assert_array_equal(g.labels().cpu().numpy(), ref.labels())
    assert g.num_components() == ref.num_components()
    assert g.sync() == cc.cc.CC_OK
    g.close()
