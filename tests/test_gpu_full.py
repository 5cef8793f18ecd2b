"""Full-size parity on the two single-graph workloads, in the launch
configurations the benchmark times, against the oracle:

* the R-MAT scale-24 stream (77 minibatches of log-uniform size, 2^20 query
  pairs after each): every query answer, and the labels and the component
  count after EVERY minibatch;
* the 4096^2 mesh stream (8272 minibatches of 2^12 edges, 2^10 pairs after
  each) in all three forms the benchmark compares:
    - plain launches: every answer, the component count and a fixed probe set
      after every minibatch, the labels every 256th minibatch and at the end;
    - one HIP-graph replay of the whole sequence (replayed twice), and
      recordings of 256 minibatches each replayed in turn with the labels and
      count checked after each;
    - the one-launch stream kernel over the whole stream, and over chunks of
      256 minibatches with the labels and count checked after each.
"""
import numpy as np
import pytest
import torch

import oracle
import synth

pytestmark = [pytest.mark.gpu, pytest.mark.slow]

CHUNK = 256  # minibatches between label checks on the mesh stream


@pytest.fixture(scope="module")
def cc():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1602_05232_amd as ccgpu
    ccgpu.lib()
    return ccgpu


def labels_equal(got: torch.Tensor, want: np.ndarray, what: str):
    g = got.cpu().numpy()
    bad = np.flatnonzero(g != want)
    assert bad.size == 0, "%s: %d labels differ, first at vertex %d (%d vs %d)" % (
        what, bad.size, bad[0], g[bad[0]], want[bad[0]])


def answers_equal(got: np.ndarray, want: np.ndarray, what: str):
    bad = np.flatnonzero(got != want)
    assert bad.size == 0, "%s: %d answers differ, first at pair %d" % (what, bad.size, bad[0])


@pytest.mark.timeout(900)
def test_rmat24_labels_after_every_minibatch(cc):
    from paper_1602_05232_amd import tuning
    s = synth.rmat_stream(scale=24)
    opts = tuning.plain_options(s.n, "rmat")
    print("rmat24 full parity: n=%d edges=%d minibatches=%d opts=%s" % (s.n, len(s.edges), s.num_batches, opts),
          flush=True)
    ref = oracle.UnionFind(s.n)
    g = cc.Graph(s.n, **opts)
    g.reserve(int(np.diff(s.eoff).max()))
    E = torch.from_numpy(s.edges).cuda()
    Q = torch.from_numpy(s.queries).cuda()
    out = torch.empty(len(s.queries), dtype=torch.uint8, device="cuda")
    lab = torch.empty(s.n, dtype=torch.int32, device="cuda")
    for i in range(s.num_batches):
        e0, e1, q0, q1 = int(s.eoff[i]), int(s.eoff[i + 1]), int(s.qoff[i]), int(s.qoff[i + 1])
        g.bulk_update(E[e0:e1])
        g.bulk_query(Q[q0:q1], out=out[q0:q1])
        g.labels(out=lab)
        ref.bulk_update(s.edges[e0:e1])
        answers_equal(out[q0:q1].cpu().numpy(), ref.bulk_query(s.queries[q0:q1]), "minibatch %d" % i)
        labels_equal(lab, ref.labels(), "labels after minibatch %d" % i)
        assert g.num_components() == ref.num_components(), "components after minibatch %d" % i
        if i % 8 == 0 or i == s.num_batches - 1:
            print("  minibatch %d/%d: answers and labels equal, components=%d"
                  % (i + 1, s.num_batches, ref.num_components()), flush=True)
    assert g.count_roots() == ref.num_components()
    assert g.sync() == cc.cc.CC_OK
    g.close()


class GridExpect:
    """The oracle's results on the mesh stream: every query answer, the probe
    answers and component count after every minibatch, and the labels after
    every CHUNK-th minibatch and the last one."""

    def __init__(self, s):
        ref = oracle.UnionFind(s.n)
        nb = s.num_batches
        self.answers = np.empty(len(s.queries), np.uint8)
        self.probes = np.empty((nb, len(s.probes)), np.uint8)
        self.counts = np.empty(nb, np.int64)
        self.labels = {}
        for i in range(nb):
            ref.bulk_update(s.batch(i))
            self.answers[int(s.qoff[i]):int(s.qoff[i + 1])] = ref.bulk_query(s.query(i))
            self.probes[i] = ref.bulk_query(s.probes)
            self.counts[i] = ref.num_components()
            if (i + 1) % CHUNK == 0 or i == nb - 1:
                self.labels[i] = ref.labels()


@pytest.fixture(scope="module")
def grid():
    s = synth.grid_stream_cfg()
    print("mesh stream: n=%d edges=%d minibatches=%d" % (s.n, len(s.edges), s.num_batches), flush=True)
    return s, GridExpect(s)


def grid_setup(cc, s, st):
    from paper_1602_05232_amd import tuning
    opts = tuning.plain_options(s.n, "grid")
    with torch.cuda.stream(st):
        g = cc.Graph(s.n, stream=st, **opts)
        g.reserve(int(np.diff(s.eoff).max()))
        E = torch.from_numpy(s.edges).cuda()
        Q = torch.from_numpy(s.queries).cuda()
        out = torch.zeros(len(s.queries), dtype=torch.uint8, device="cuda")
        lab = torch.empty(s.n, dtype=torch.int32, device="cuda")
    st.synchronize()
    return g, E, Q, out, lab, opts


@pytest.mark.timeout(900)
def test_grid4096_plain_every_minibatch(cc, grid):
    s, want = grid
    st = torch.cuda.Stream()
    g, E, Q, out, lab, opts = grid_setup(cc, s, st)
    print("mesh, plain launches, opts=%s" % opts, flush=True)
    P = torch.from_numpy(s.probes).cuda()
    pout = torch.empty((s.num_batches, len(s.probes)), dtype=torch.uint8, device="cuda")
    with torch.cuda.stream(st):
        for i in range(s.num_batches):
            e0, e1, q0, q1 = int(s.eoff[i]), int(s.eoff[i + 1]), int(s.qoff[i]), int(s.qoff[i + 1])
            g.bulk_update(E[e0:e1])
            g.bulk_query(Q[q0:q1], out=out[q0:q1])
            g.bulk_query(P, out=pout[i])
            assert g.num_components() == want.counts[i], "components after minibatch %d" % i
            if i in want.labels:
                g.labels(out=lab)
                labels_equal(lab, want.labels[i], "labels after minibatch %d" % i)
                answers_equal(pout[:i + 1].cpu().numpy(), want.probes[:i + 1], "probes up to minibatch %d" % i)
                print("  minibatch %d/%d: counts, probes and labels equal" % (i + 1, s.num_batches), flush=True)
    st.synchronize()
    answers_equal(out.cpu().numpy(), want.answers, "mesh stream, plain launches")
    assert g.sync() == cc.cc.CC_OK
    g.close()


@pytest.mark.timeout(900)
def test_grid4096_hipgraph_replay(cc, grid):
    s, want = grid
    st = torch.cuda.Stream()
    g, E, Q, out, lab, opts = grid_setup(cc, s, st)
    nb = s.num_batches
    eoff, qoff = [int(x) for x in s.eoff], [int(x) for x in s.qoff]
    last = nb - 1
    with torch.cuda.stream(st):
        # the benchmark's form: reset, the whole stream and the label pass in one recording
        with g.capture() as cap:
            g.reset()
            for i in range(nb):
                g.bulk_update(E[eoff[i]:eoff[i + 1]])
                g.bulk_query(Q[qoff[i]:qoff[i + 1]], out=out[qoff[i]:qoff[i + 1]])
            g.labels(out=lab)
        rec = cap.recording
        for rep in range(2):
            out.zero_()
            rec.launch()
            st.synchronize()
            answers_equal(out.cpu().numpy(), want.answers, "whole-stream replay %d" % rep)
            labels_equal(lab, want.labels[last], "labels after whole-stream replay %d" % rep)
            assert g.num_components() == want.counts[last]
            print("  whole-stream replay %d: every answer and the labels equal" % rep, flush=True)
        rec.close()
        # recordings of CHUNK minibatches, replayed in turn
        g.reset()
        out.zero_()
        for j0 in range(0, nb, CHUNK):
            j1 = min(nb, j0 + CHUNK)
            with g.capture() as cap:
                for i in range(j0, j1):
                    g.bulk_update(E[eoff[i]:eoff[i + 1]])
                    g.bulk_query(Q[qoff[i]:qoff[i + 1]], out=out[qoff[i]:qoff[i + 1]])
            cap.recording.launch()
            cap.recording.close()
            assert g.num_components() == want.counts[j1 - 1], "components after minibatch %d" % (j1 - 1)
            g.labels(out=lab)
            labels_equal(lab, want.labels[j1 - 1], "labels after minibatch %d (chunked replay)" % (j1 - 1))
            answers_equal(out[qoff[j0]:qoff[j1]].cpu().numpy(), want.answers[qoff[j0]:qoff[j1]],
                          "chunked replay, minibatches %d..%d" % (j0, j1 - 1))
    print("  chunked replays: labels and counts equal after every %d minibatches" % CHUNK, flush=True)
    assert g.sync() == cc.cc.CC_OK
    g.close()


@pytest.mark.timeout(900)
def test_grid4096_stream_kernel(cc, grid):
    s, want = grid
    st = torch.cuda.Stream()
    g, E, Q, out, lab, opts = grid_setup(cc, s, st)
    nb = s.num_batches
    last = nb - 1
    mx = int(max(np.diff(s.eoff).max(), np.diff(s.qoff).max()))
    from paper_1602_05232_amd import tuning
    for k, v in tuning.lookup("stream", "grid", s.n).items():  # the benchmark's launch shape
        g.set_option(k, v)
    with torch.cuda.stream(st):
        eo = torch.from_numpy(s.eoff.astype(np.int64)).cuda()
        qo = torch.from_numpy(s.qoff.astype(np.int64)).cuda()
        # the benchmark's form: the whole stream in one launch
        for rep in range(2):
            g.reset()
            out.zero_()
            g.bulk_stream(E, eo, Q, qo, out, max_items=mx)
            g.labels(out=lab)
            st.synchronize()
            assert g.sync() == cc.cc.CC_OK
            answers_equal(out.cpu().numpy(), want.answers, "one launch over the stream, run %d" % rep)
            labels_equal(lab, want.labels[last], "labels after the one-launch stream, run %d" % rep)
            assert g.num_components() == want.counts[last]
            print("  one launch over %d minibatches (run %d): every answer and the labels equal" % (nb, rep),
                  flush=True)
        # chunks of CHUNK minibatches, one launch each
        g.reset()
        out.zero_()
        for j0 in range(0, nb, CHUNK):
            j1 = min(nb, j0 + CHUNK)
            g.bulk_stream(E, eo[j0:j1 + 1], Q, qo[j0:j1 + 1], out, max_items=mx)
            assert g.num_components() == want.counts[j1 - 1], "components after minibatch %d" % (j1 - 1)
            g.labels(out=lab)
            labels_equal(lab, want.labels[j1 - 1], "labels after minibatch %d (chunked stream kernel)" % (j1 - 1))
    st.synchronize()
    answers_equal(out.cpu().numpy(), want.answers, "chunked stream kernel")
    print("  chunked launches: labels and counts equal after every %d minibatches" % CHUNK, flush=True)
    assert g.sync() == cc.cc.CC_OK
    g.close()
