"""Full-size parity: the benchmark workload and the high-diameter mesh, in the
launch configuration the benchmark uses, every query answer compared with the
oracle and the labels at checkpoints and at the end."""
import numpy as np
import pytest
import torch

import oracle
import synth

pytestmark = [pytest.mark.gpu, pytest.mark.slow]


@pytest.fixture(scope="module")
def cc():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1602_05232_amd as ccgpu
    ccgpu.lib()
    return ccgpu


def stream_parity(cc, s, opts, checkpoints):
    print("full parity: %s n=%d edges=%d batches=%d opts=%s" % (s.name, s.n, len(s.edges), s.num_batches, opts),
          flush=True)
    ref = oracle.UnionFind(s.n)
    g = cc.Graph(s.n, **opts)
    g.reserve(int(np.diff(s.eoff).max()))
    E = torch.from_numpy(s.edges).cuda()
    Q = torch.from_numpy(s.queries).cuda()
    out = torch.empty(len(s.queries), dtype=torch.uint8, device="cuda")
    want = np.empty(len(s.queries), np.uint8)
    for i in range(s.num_batches):
        e0, e1, q0, q1 = int(s.eoff[i]), int(s.eoff[i + 1]), int(s.qoff[i]), int(s.qoff[i + 1])
        g.bulk_update(E[e0:e1])
        g.bulk_query(Q[q0:q1], out=out[q0:q1])
        ref.bulk_update(s.edges[e0:e1])
        want[q0:q1] = ref.bulk_query(s.queries[q0:q1])
        if i in checkpoints or i == s.num_batches - 1:
            np.testing.assert_array_equal(g.labels().cpu().numpy(), ref.labels(),
                                          err_msg="labels after minibatch %d" % i)
            assert g.num_components() == ref.num_components()
            print("  minibatch %d/%d: labels equal, components=%d" % (i, s.num_batches, ref.num_components()),
                  flush=True)
    got = out.cpu().numpy()
    bad = np.flatnonzero(got != want)
    assert bad.size == 0, "%d answers differ, first at %d" % (bad.size, bad[0])
    assert g.count_roots() == ref.num_components()
    assert g.sync() == cc.cc.CC_OK
    g.close()


@pytest.mark.timeout(600)
def test_rmat24_benchmark_stream(cc):
    from paper_1602_05232_amd import tuning
    s = synth.rmat_stream(scale=24)
    stream_parity(cc, s, tuning.plain_options(s.n, "rmat"), checkpoints={0, 1, s.num_batches // 2})


@pytest.mark.timeout(600)
def test_grid4096_stream(cc):
    from paper_1602_05232_amd import tuning
    s = synth.grid_stream_cfg()
    stream_parity(cc, s, tuning.plain_options(s.n, "grid"), checkpoints={s.num_batches // 2})
