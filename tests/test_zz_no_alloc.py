"""cc_bulk_update_noalloc, called through the C ABI, against cc_bulk_update
and the oracle: two calls in a row (the second smaller), every linking
order, answers, labels and counts equal; sizes beyond the limit refused with
nothing enqueued; and the calls captured into a HIP graph and replayed."""
import ctypes

import numpy as np
import pytest
import torch

import oracle
import synth

pytestmark = pytest.mark.gpu

LIMIT = 1 << 22


@pytest.fixture(scope="module")
def cc():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1602_05232_amd as ccgpu
    ccgpu.lib()
    return ccgpu


def ptr(t):
    return ctypes.c_void_p(t.data_ptr())


@pytest.mark.parametrize("opts", [dict(), dict(hook=1), dict(hook=2, compress_linked=0),
                                  dict(hook=2, filter=2, compress_linked=0, block=512, items=1, grid_cap=768)],
                         ids=lambda o: ",".join("%s=%s" % kv for kv in sorted(o.items())) or "default")
def test_noalloc_matches_bulk_update(cc, opts):
    L = cc.lib()
    n = 1 << 20
    k = synth.key(synth.BASE_SEED + 11, 0, synth.P_EDGES)
    big = synth.rmat_edges(k, 0, 3 << 20, 20, n, synth.permutation(synth.key(synth.BASE_SEED + 11, 0, synth.P_PERM), n))
    small = synth.uniform_pairs(synth.key(synth.BASE_SEED + 11, 1, synth.P_EDGES), 0, 100_003, n)
    pairs = synth.uniform_pairs(synth.key(synth.BASE_SEED + 11, 0, synth.P_QUERIES), 0, 1 << 18, n)
    B, S, P = (torch.from_numpy(a).cuda() for a in (big, small, pairs))
    g_ref = cc.Graph(n, **opts)
    g_new = cc.Graph(n, **opts)
    ref = oracle.UnionFind(n)
    for step, E in enumerate((B, S)):
        assert L.cc_bulk_update(ctypes.c_void_p(g_ref.handle), ptr(E), E.shape[0]) == cc.cc.CC_OK
        assert L.cc_bulk_update_noalloc(ctypes.c_void_p(g_new.handle), ptr(E), E.shape[0]) == cc.cc.CC_OK
        ref.bulk_update(E.cpu().numpy())
        want = ref.bulk_query(pairs)
        for g in (g_ref, g_new):
            np.testing.assert_array_equal(g.bulk_query(P).cpu().numpy(), want, err_msg="call %d" % step)
            np.testing.assert_array_equal(g.labels().cpu().numpy(), ref.labels(), err_msg="call %d" % step)
            assert g.num_components() == ref.num_components()
            assert g.count_roots() == ref.num_components()
    # beyond the limit: refused, nothing enqueued, the graph unchanged
    over = torch.zeros((LIMIT + 1, 2), dtype=torch.int32, device="cuda")
    assert L.cc_bulk_update_noalloc(ctypes.c_void_p(g_new.handle), ptr(over), LIMIT + 1) == cc.cc.CC_EINVAL
    assert g_new.num_components() == ref.num_components()
    for g in (g_ref, g_new):
        assert g.sync() == cc.cc.CC_OK
        g.close()


def test_noalloc_under_capture(cc):
    """The entry point's work records into a HIP graph (no allocation, no
    memset node); replays with eager work between them give the eager result."""
    n = 1 << 16
    s = synth.er_stream(n=n, batches=4, batch=1 << 14, qbatch=1 << 14, probes=0)
    st = torch.cuda.Stream()
    with torch.cuda.stream(st):
        E = torch.from_numpy(s.edges).cuda()
        Q = torch.from_numpy(s.queries).cuda()
        out = torch.zeros(len(s.queries), dtype=torch.uint8, device="cuda")
        g = cc.Graph(n, stream=st, hook=2, compress_linked=0)
        with g.capture() as cap:
            g.reset()
            for i in range(s.num_batches):
                g.bulk_update_noalloc(E[s.eoff[i]:s.eoff[i + 1]])
                g.bulk_query(Q[s.qoff[i]:s.qoff[i + 1]], out=out[s.qoff[i]:s.qoff[i + 1]])
        rec = cap.recording
        ref = oracle.UnionFind(n)
        want = np.concatenate([(ref.bulk_update(s.batch(i)), ref.bulk_query(s.query(i)))[1]
                               for i in range(s.num_batches)])
        other = cc.Graph(1000, stream=st)
        for rep in range(3):
            out.fill_(7)
            other.bulk_update_noalloc(torch.randint(0, 1000, (5000, 2), dtype=torch.int32, device="cuda"))
            st.synchronize()
            rec.launch()
            st.synchronize()
            np.testing.assert_array_equal(out.cpu().numpy(), want, err_msg="replay %d" % rep)
            np.testing.assert_array_equal(g.labels().cpu().numpy(), ref.labels(), err_msg="replay %d" % rep)
            assert g.num_components() == ref.num_components()
        assert g.sync() == cc.cc.CC_OK and other.sync() == cc.cc.CC_OK
        rec.close()
        other.close()
        g.close()
