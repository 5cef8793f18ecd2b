"""Captured (HIP graph) update/query sequences replay to the eager results.

Each replay is checked against the eager run, with other eager work and
host synchronisations between replays."""
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


@pytest.mark.parametrize("opts", [dict(), dict(update_mode=1), dict(hook=1), dict(hook=2),
                                  dict(compress_linked=0, items=1), dict(filter=1),
                                  dict(filter=2, hook=2, compress_linked=0)],
                         ids=lambda o: ",".join("%s=%s" % kv for kv in sorted(o.items())) or "default")
def test_capture_replays_match_eager(cc, opts):
    s = synth.grid_stream_cfg(W=128, H=128, batch=1 << 10, qbatch=1 << 8)
    st = torch.cuda.Stream()
    with torch.cuda.stream(st):
        E = torch.from_numpy(s.edges).cuda()
        Q = torch.from_numpy(s.queries).cuda()
        out_e = torch.empty(len(s.queries), dtype=torch.uint8, device="cuda")
        out_g = torch.empty_like(out_e)
        lab_e = torch.empty(s.n, dtype=torch.int32, device="cuda")
        lab_g = torch.empty_like(lab_e)
        g = cc.Graph(s.n, stream=st, **opts)
        g.reserve(int(np.diff(s.eoff).max()))

        def sequence(out, lab):
            g.reset()
            for i in range(s.num_batches):
                g.bulk_update(E[s.eoff[i]:s.eoff[i + 1]])
                g.bulk_query(Q[s.qoff[i]:s.qoff[i + 1]], out=out[s.qoff[i]:s.qoff[i + 1]])
            g.labels(out=lab)

        sequence(out_e, lab_e)
        st.synchronize()
        comps = g.num_components()
        with g.capture() as cap:
            sequence(out_g, lab_g)
        rec = cap.recording
        ref = oracle.UnionFind(s.n)
        want = np.concatenate([(ref.bulk_update(s.batch(i)), ref.bulk_query(s.query(i)))[1]
                               for i in range(s.num_batches)])
        np.testing.assert_array_equal(out_e.cpu().numpy(), want)
        np.testing.assert_array_equal(lab_e.cpu().numpy(), ref.labels())
        other = cc.Graph(1000, stream=st)
        for rep in range(3):
            out_g.fill_(7)
            lab_g.fill_(-1)
            other.bulk_update(torch.randint(0, 1000, (500, 2), dtype=torch.int32, device="cuda"))
            st.synchronize()
            rec.launch()
            st.synchronize()
            np.testing.assert_array_equal(out_g.cpu().numpy(), out_e.cpu().numpy(), err_msg="replay %d" % rep)
            np.testing.assert_array_equal(lab_g.cpu().numpy(), lab_e.cpu().numpy(), err_msg="replay %d" % rep)
            assert g.num_components() == comps
            assert g.sync() == cc.cc.CC_OK
        rec.close()
        other.close()
        g.close()


def test_capture_rejects_waiting_calls(cc):
    st = torch.cuda.Stream()
    g = cc.Graph(100, stream=st)
    L = cc.lib()
    import ctypes
    e = torch.zeros((4, 2), dtype=torch.int32, device="cuda")
    torch.cuda.synchronize()
    assert L.cc_capture_begin(g.handle) == 0
    v = ctypes.c_int64()
    assert L.cc_num_components(g.handle, ctypes.byref(v)) == cc.cc.CC_EINVAL
    assert L.cc_sync(g.handle) == cc.cc.CC_EINVAL
    assert L.cc_capture_begin(g.handle) == cc.cc.CC_EINVAL
    assert L.cc_set_option(g.handle, 1, 2) == 0  # the contracting update is one cooperative launch
    assert L.cc_bulk_update(g.handle, ctypes.c_void_p(e.data_ptr()), 4) == cc.cc.CC_EINVAL
    assert L.cc_set_option(g.handle, 1, 0) == 0
    x = ctypes.c_void_p()
    assert L.cc_capture_end(g.handle, ctypes.byref(x)) == 0
    assert L.cc_exec_destroy(x.value) == 0
    g0 = cc.Graph(10, stream=torch.cuda.default_stream())
    if g0.stream.cuda_stream == 0:
        assert L.cc_capture_begin(g0.handle) == cc.cc.CC_EINVAL
    g0.close()
    g.close()


@pytest.mark.parametrize("filt", [0, 2])
def test_replay_after_eager_reset_keeps_forest_state(cc, filt):
    """A recording that resets and updates, replayed after an eager reset,
    leaves a forest with links: the linking order can no longer change, the
    filter's bitmaps stay proofs, and answers and labels are the oracle's."""
    import ctypes
    s = synth.er_stream(n=1 << 12, batches=4, batch=1 << 11, qbatch=1 << 11, probes=0)
    st = torch.cuda.Stream()
    L = cc.lib()
    with torch.cuda.stream(st):
        E = torch.from_numpy(s.edges).cuda()
        Q = torch.from_numpy(s.queries).cuda()
        out = torch.zeros(len(s.queries), dtype=torch.uint8, device="cuda")
        g = cc.Graph(s.n, stream=st, hook=2, compress_linked=0, filter=filt)
        g.reserve(int(np.diff(s.eoff).max()))
        with g.capture() as cap:
            g.reset()
            for i in range(2):
                g.bulk_update(E[s.eoff[i]:s.eoff[i + 1]])
        rec = cap.recording
        g.reset()  # eager: the forest is pristine again
        assert L.cc_set_option(g.handle, 6, 2) == 0  # same order: allowed
        rec.launch()
        st.synchronize()
        # the replay linked vertices: another linking order is refused now
        assert L.cc_set_option(g.handle, 6, 0) == cc.cc.CC_EINVAL
        ref = oracle.UnionFind(s.n)
        for i in range(2):
            ref.bulk_update(s.batch(i))
        for i in range(2, 4):
            g.bulk_update(E[s.eoff[i]:s.eoff[i + 1]])
            ref.bulk_update(s.batch(i))
        got = g.bulk_query(Q[:4096], out=out[:4096])
        st.synchronize()
        np.testing.assert_array_equal(got.cpu().numpy(), ref.bulk_query(s.queries[:4096]))
        np.testing.assert_array_equal(g.labels().cpu().numpy(), ref.labels())
        assert g.num_components() == ref.num_components()
        # after an eager reset the order may change, but this recording was
        # made under union by rank and is refused under another order
        g.reset()
        assert L.cc_set_option(g.handle, 6, 0) == 0
        assert L.cc_exec_launch(ctypes.c_void_p(rec._h)) == cc.cc.CC_EINVAL
        assert g.sync() == cc.cc.CC_OK
        rec.close()
        g.close()


def test_replay_of_recording_made_before_filter_bitmaps(cc):
    """A recording made while the graph had no filter bitmaps resets and
    updates the forest; bitmaps allocated later must not claim proofs about
    the forest the replay leaves."""
    s = synth.er_stream(n=1 << 12, batches=3, batch=1 << 11, qbatch=1 << 11, probes=0)
    st = torch.cuda.Stream()
    with torch.cuda.stream(st):
        E = torch.from_numpy(s.edges).cuda()
        Q = torch.from_numpy(s.queries).cuda()
        g = cc.Graph(s.n, stream=st, hook=2, compress_linked=0)
        with g.capture() as cap:
            g.reset()
            g.bulk_update(E[s.eoff[0]:s.eoff[1]])
        rec = cap.recording
        # build filter state on another forest, then replay the old recording
        g.set_option("filter", 2)
        g.bulk_update(E[s.eoff[1]:s.eoff[3]])
        g.bulk_query(Q[:1024])
        rec.launch()
        ref = oracle.UnionFind(s.n)
        ref.bulk_update(s.batch(0))
        got = g.bulk_query(Q)
        st.synchronize()
        np.testing.assert_array_equal(got.cpu().numpy(), ref.bulk_query(s.queries))
        np.testing.assert_array_equal(g.labels().cpu().numpy(), ref.labels())
        g.bulk_update(E[s.eoff[1]:s.eoff[2]])
        ref.bulk_update(s.batch(1))
        got = g.bulk_query(Q)
        st.synchronize()
        np.testing.assert_array_equal(got.cpu().numpy(), ref.bulk_query(s.queries))
        assert g.sync() == cc.cc.CC_OK
        rec.close()
        g.close()
