"""Membership filter of the largest component (CC_OPT_FILTER).

Answers, labels and counts stay bit-exact against the oracle, and every bit
the filter holds is a vertex that the oracle finds connected to the filter's
anchor, after every minibatch (the bits are proofs, never guesses)."""
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
    return torch.from_numpy(np.ascontiguousarray(np.asarray(a, np.int32))).cuda()


def members(bits, n):
    v = np.unpackbits(bits.view(np.uint8), bitorder="little")[:n]
    return np.flatnonzero(v)


def check_bits(g, ref, where):
    """Every member is connected to the anchor; while the touched bitmap is
    complete, every vertex that is not alone has its touched bit (members
    included: queries read the touched words alone to prove a vertex alone)."""
    anchor, complete, bits, touched = g.filter_state()
    got = members(bits, g.n)
    lab = ref.labels()
    if anchor < 0:
        assert len(got) == 0, where
    else:
        bad = got[lab[got] != lab[anchor]]
        assert len(bad) == 0, "%s: %d member bits outside the anchor's component, e.g. %s" % (where, len(bad), bad[:8])
    if complete:
        known = np.zeros(g.n, bool)
        known[members(touched, g.n)] = True
        size = np.bincount(lab, minlength=g.n)[lab]
        bad = np.flatnonzero(~known & (size > 1))
        assert len(bad) == 0, "%s: %d vertices with edges outside the touched bitmap, e.g. %s" % (
            where, len(bad), bad[:8])
    return anchor, got


def run(cc, s, opts, check_every=1):
    print("filter: %s n=%d batches=%d opts=%s" % (s.name, s.n, s.num_batches, opts), flush=True)
    g = cc.Graph(s.n, **opts)
    ref = oracle.UnionFind(s.n)
    for i in range(s.num_batches):
        b, q = s.batch(i), s.query(i)
        ref.bulk_update(b)
        g.bulk_update(dev(b))
        if len(q):
            np.testing.assert_array_equal(g.bulk_query(dev(q)).cpu().numpy(), ref.bulk_query(q),
                                          err_msg="answers after minibatch %d" % i)
        if i % check_every == 0 or i == s.num_batches - 1:
            check_bits(g, ref, "after minibatch %d" % i)
    np.testing.assert_array_equal(g.labels().cpu().numpy(), ref.labels())
    assert g.num_components() == ref.num_components() == g.count_roots()
    assert g.sync() == cc.cc.CC_OK
    return g, ref


@pytest.mark.parametrize("opts", [dict(hook=0, filter=2), dict(hook=1, filter=1), dict(hook=1, filter=2),
                                  dict(hook=2, filter=1, compress_linked=0),
                                  dict(hook=2, filter=2, query_halving=0, items=1, block=64)],
                         ids=lambda o: ",".join("%s=%s" % kv for kv in sorted(o.items())))
def test_rmat_bits_are_proofs_and_the_anchor_is_the_giant(cc, opts):
    s = synth.rmat_stream(scale=16, size_lo=8, size_hi=16, qbatch=1 << 12)
    g, ref = run(cc, s, opts)
    anchor, got = check_bits(g, ref, "at the end")
    lab = ref.labels()
    sizes = np.bincount(lab, minlength=s.n)
    assert anchor >= 0 and sizes[lab[anchor]] == sizes.max()
    # the filter engaged: most of the giant component is known to it
    assert len(got) > sizes.max() // 2
    g.close()


@pytest.mark.parametrize("opts", [dict(find=1, hook=2, filter=2), dict(find=2, hook=1, filter=2),
                                  dict(find=1, hook=0, filter=1, grid_cap=7)],
                         ids=lambda o: ",".join("%s=%s" % kv for kv in sorted(o.items())))
def test_bulk_find_with_the_filter_keeps_both_bitmaps(cc, opts):
    """Bulk-Find under the filter: the membership bits it settles items with
    stay proofs, its updates keep the touched bitmap complete (queries then
    settle pairs with an end that never had an edge), and every answer and
    label is the oracle's."""
    s = synth.rmat_stream(scale=15, size_lo=8, size_hi=15, qbatch=1 << 11)
    g, ref = run(cc, s, opts)
    anchor, got = check_bits(g, ref, "at the end")
    assert g.filter_state()[1], "touched bitmap no longer complete"
    lab = ref.labels()
    sizes = np.bincount(lab, minlength=s.n)
    assert anchor >= 0 and len(got) > sizes.max() // 2, "the refills did not engage"
    g.close()


def test_anchor_moves_to_the_larger_component_and_the_bitmap_is_refilled(cc):
    n = 1 << 15
    rng = np.random.default_rng(5)
    path = np.stack([np.arange(0, 1999), np.arange(1, 2000)], 1)          # component A: [0, 2000)
    again = rng.integers(0, 2000, size=(4096, 2))                         # more edges inside A
    big = [rng.integers(2000, n, size=(8192, 2)) for _ in range(10)]      # component B grows on the rest
    batches = [path, again] + big
    edges = np.concatenate(batches).astype(np.int32)
    queries = rng.integers(0, n, size=(len(batches) * 512, 2)).astype(np.int32)
    s = synth.tiny_stream(n, edges, [len(b) for b in batches])
    s = synth.Stream("two-parts", n, s.edges, s.eoff, queries, np.arange(0, len(queries) + 1, 512), s.probes)
    g = cc.Graph(n, filter=2, hook=2)
    ref = oracle.UnionFind(n)
    anchors = []
    for i in range(s.num_batches):
        ref.bulk_update(s.batch(i))
        g.bulk_update(dev(s.batch(i)))
        np.testing.assert_array_equal(g.bulk_query(dev(s.query(i))).cpu().numpy(), ref.bulk_query(s.query(i)))
        a, _ = check_bits(g, ref, "after minibatch %d" % i)
        anchors.append(a)
    lab = ref.labels()
    assert 0 <= anchors[1] < 2000, anchors         # first anchor: in A (the only structure then)
    assert anchors[-1] >= 2000 and lab[anchors[-1]] != lab[0], anchors  # moved to B
    np.testing.assert_array_equal(g.labels().cpu().numpy(), lab)
    g.close()


def test_reset_load_and_tiny_ragged_sizes(cc):
    s = synth.rmat_stream(scale=12, size_lo=6, size_hi=11, qbatch=256)
    g, ref = run(cc, s, dict(filter=2, hook=2))
    a, got = check_bits(g, ref, "end")
    assert a >= 0 and len(got) > 0
    assert g.filter_state()[1]
    img = g.save()
    g.reset()
    a, complete, got, touched = g.filter_state()
    assert a == -1 and complete and not got.any() and not touched.any()
    g.load(img)
    a, complete, got, touched = g.filter_state()
    assert a == -1 and not complete and not got.any() and not touched.any()
    np.testing.assert_array_equal(g.labels().cpu().numpy(), ref.labels())
    g.close()
    # n not a multiple of 32, single-edge minibatches, self-loops, ids out of range
    for n in (1, 2, 33, 95):
        g = cc.Graph(n, filter=2)
        ref = oracle.UnionFind(n)
        rng = np.random.default_rng(n)
        for i in range(12):
            b = rng.integers(0, n, size=(int(rng.integers(1, 6)), 2)).astype(np.int32)
            ref.bulk_update(b)
            g.bulk_update(dev(b))
            q = rng.integers(0, n, size=(7, 2)).astype(np.int32)
            np.testing.assert_array_equal(g.bulk_query(dev(q)).cpu().numpy(), ref.bulk_query(q))
            check_bits(g, ref, "n=%d minibatch %d" % (n, i))
        g.bulk_update(dev([[0, n], [n - 1, 0]]))
        ref.bulk_update(np.array([[0, n], [n - 1, 0]], np.int32))
        assert g.sync() == cc.cc.CC_ERANGE
        np.testing.assert_array_equal(g.labels().cpu().numpy(), ref.labels())
        g.close()


def test_filter_with_other_schedules_keeps_bits_sound(cc):
    """Switching schedule mid-stream: the split and contracting schedules
    leave the bitmaps alone, Bulk-Find refills the membership bits and keeps
    the touched ones, and what the bitmaps hold stays true."""
    s = synth.rmat_stream(scale=14, size_lo=8, size_hi=13, qbatch=1 << 10)
    g = cc.Graph(s.n, filter=2)
    ref = oracle.UnionFind(s.n)
    modes = [dict(update_mode=0, find=0), dict(update_mode=1), dict(update_mode=2), dict(update_mode=0, find=1)]
    for i in range(s.num_batches):
        for k, v in modes[i % len(modes)].items():
            g.set_option(k, v)
        ref.bulk_update(s.batch(i))
        g.bulk_update(dev(s.batch(i)))
        np.testing.assert_array_equal(g.bulk_query(dev(s.query(i))).cpu().numpy(), ref.bulk_query(s.query(i)))
        check_bits(g, ref, "after minibatch %d" % i)
        assert g.filter_state()[1] == (i == 0), "touched bitmap complete only before the first other schedule"
    np.testing.assert_array_equal(g.labels().cpu().numpy(), ref.labels())
    g.close()


def test_filter_enabled_mid_stream_does_not_trust_the_touched_bitmap(cc):
    s = synth.rmat_stream(scale=12, size_lo=6, size_hi=11, qbatch=256)
    g = cc.Graph(s.n, hook=2)
    ref = oracle.UnionFind(s.n)
    for i in range(s.num_batches):
        if i == 3:
            g.set_option("filter", 2)
        ref.bulk_update(s.batch(i))
        g.bulk_update(dev(s.batch(i)))
        np.testing.assert_array_equal(g.bulk_query(dev(s.query(i))).cpu().numpy(), ref.bulk_query(s.query(i)))
        if i >= 3:
            assert not g.filter_state()[1]
            check_bits(g, ref, "after minibatch %d" % i)
    g.reset()
    assert g.filter_state()[1]
    ref = oracle.UnionFind(s.n)
    for i in range(s.num_batches):
        ref.bulk_update(s.batch(i))
        g.bulk_update(dev(s.batch(i)))
        np.testing.assert_array_equal(g.bulk_query(dev(s.query(i))).cpu().numpy(), ref.bulk_query(s.query(i)))
        assert g.filter_state()[1]
        check_bits(g, ref, "second pass, minibatch %d" % i)
    g.close()


def test_stream_of_isolated_vertices_and_a_giant(cc):
    """Most query pairs have an endpoint that never had an edge: the touched
    bitmap answers them 0; pairs inside the giant answer 1 from the
    membership bitmap; everything else takes finds."""
    n = 1 << 16
    rng = np.random.default_rng(11)
    half = rng.permutation(n)[: n // 2]
    batches = [np.stack([rng.choice(half, 20000), rng.choice(half, 20000)], 1) for _ in range(8)]
    batches.append(np.array([[5, 5], [7, 7]]))  # self-loops only: nothing joined, nobody touched
    edges = np.concatenate(batches).astype(np.int32)
    q = np.concatenate([rng.integers(0, n, size=(4000, 2)), np.stack([half[:1000], half[1000:2000]], 1),
                        np.array([[5, 5], [5, 7]])]).astype(np.int32)
    queries = np.concatenate([q] * len(batches))
    base = synth.tiny_stream(n, edges, [len(b) for b in batches])
    s = synth.Stream("isolated-and-giant", n, base.edges, base.eoff, queries,
                     np.arange(0, len(queries) + 1, len(q)), base.probes)
    for opts in (dict(filter=2, hook=2), dict(filter=2, hook=0), dict(filter=2, hook=1, items=8, block=128)):
        g, ref = run(cc, s, opts)
        assert g.filter_state()[1]
        g.close()



def test_replays_and_other_schedules_keep_queries_exact(cc):
    """A replay can reset the graph behind the host's back: an update by
    another schedule after it must still mark the touched bitmap incomplete."""
    s = synth.rmat_stream(scale=12, size_lo=6, size_hi=11, qbatch=512)
    half = s.num_batches // 2
    E = dev(s.edges)
    st = torch.cuda.Stream()
    with torch.cuda.stream(st):
        g = cc.Graph(s.n, stream=st, filter=2)
        g.reserve(int(np.diff(s.eoff).max()))
        with g.capture() as cap:
            g.reset()
            for i in range(half):
                g.bulk_update(E[int(s.eoff[i]):int(s.eoff[i + 1])])
        rec = cap.recording
        for rep in range(2):
            rec.launch()
            ref = oracle.UnionFind(s.n)
            for i in range(half):
                ref.bulk_update(s.batch(i))
            assert g.filter_state()[1]
            other = False  # an update by another schedule since the replay
            for i in range(half, s.num_batches):
                mode = 1 if i % 2 == 0 else 0
                other = other or mode == 1
                g.set_option("update_mode", mode)
                ref.bulk_update(s.batch(i))
                g.bulk_update(E[int(s.eoff[i]):int(s.eoff[i + 1])])
                got = g.bulk_query(dev(s.query(i))).cpu().numpy()
                np.testing.assert_array_equal(got, ref.bulk_query(s.query(i)), err_msg="replay %d minibatch %d" % (rep, i))
                assert g.filter_state()[1] == (not other)
                check_bits(g, ref, "replay %d minibatch %d" % (rep, i))
            g.set_option("update_mode", 0)
        np.testing.assert_array_equal(g.labels().cpu().numpy(), ref.labels())
        rec.close()
        g.close()


def test_stream_kernel_after_filtered_updates_keeps_answers_exact(cc):
    """cc_bulk_stream applies minibatches without the bitmaps: afterwards the
    touched bitmap is no longer trusted, and every answer stays exact."""
    s = synth.rmat_stream(scale=13, size_lo=7, size_hi=12, qbatch=512)
    half = s.num_batches // 2
    g = cc.Graph(s.n, filter=2, hook=2)
    ref = oracle.UnionFind(s.n)
    for i in range(half):
        ref.bulk_update(s.batch(i))
        g.bulk_update(dev(s.batch(i)))
        np.testing.assert_array_equal(g.bulk_query(dev(s.query(i))).cpu().numpy(), ref.bulk_query(s.query(i)))
    assert g.filter_state()[1]
    rest = range(half, s.num_batches)
    edges = np.concatenate([s.batch(i) for i in rest])
    pairs = np.concatenate([s.query(i) for i in rest])
    eoff = torch.tensor(np.concatenate([[0], np.cumsum([len(s.batch(i)) for i in rest])]), dtype=torch.int64).cuda()
    qoff = torch.tensor(np.concatenate([[0], np.cumsum([len(s.query(i)) for i in rest])]), dtype=torch.int64).cuda()
    out = torch.empty(len(pairs), dtype=torch.uint8, device="cuda")
    g.bulk_stream(dev(edges), eoff, dev(pairs), qoff, out)
    want = np.concatenate([(ref.bulk_update(s.batch(i)), ref.bulk_query(s.query(i)))[1] for i in rest])
    np.testing.assert_array_equal(out.cpu().numpy(), want)
    assert not g.filter_state()[1]
    check_bits(g, ref, "after the stream kernel")
    q = np.random.default_rng(2).integers(0, s.n, size=(4096, 2)).astype(np.int32)
    np.testing.assert_array_equal(g.bulk_query(dev(q)).cpu().numpy(), ref.bulk_query(q))
    np.testing.assert_array_equal(g.labels().cpu().numpy(), ref.labels())
    assert g.sync() == cc.cc.CC_OK
    g.close()
