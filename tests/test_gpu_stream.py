"""cc_bulk_stream (a whole update/query sequence in one cooperative launch)
against the oracle, and its bounded barrier wait."""
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


def run_stream(cc, s, opts, max_items=None):
    print("stream kernel: %s n=%d batches=%d %s" % (s.name, s.n, s.num_batches, opts), flush=True)
    g = cc.Graph(s.n, **opts)
    E = torch.from_numpy(s.edges).cuda()
    Q = torch.from_numpy(s.queries).cuda()
    eo = torch.from_numpy(s.eoff.astype(np.int64)).cuda()
    qo = torch.from_numpy(s.qoff.astype(np.int64)).cuda()
    out = torch.full((len(s.queries),), 7, dtype=torch.uint8, device="cuda")
    g.bulk_stream(E, eo, Q, qo, out, max_items=max_items)
    try:
        rc = g.sync()
    except cc.CCError as e:  # a device error (the barrier timeout) raises
        rc = e.code
    return g, out.cpu().numpy(), rc


@pytest.mark.parametrize("which", ["grid", "er", "rmat"])
@pytest.mark.parametrize("opts", [dict(), dict(hook=1), dict(hook=2), dict(block=64, grid_cap=3),
                                  dict(block=1024, grid_cap=1, hook=2), dict(block=128, hook=1)],
                         ids=["id", "hash", "rank", "b64-g3", "b1024-g1-rank", "b128-hash"])
def test_stream_kernel_matches_oracle(cc, which, opts):
    if which == "grid":
        s = synth.grid_stream_cfg(W=256, H=256, batch=1 << 12, qbatch=1 << 10)
    elif which == "er":
        s = synth.er_stream()
    else:
        s = synth.rmat_stream(scale=16, size_lo=6, size_hi=14, qbatch=1 << 11)
    g, got, rc = run_stream(cc, s, opts)
    assert rc == cc.cc.CC_OK
    ref = oracle.UnionFind(s.n)
    want = np.concatenate([(ref.bulk_update(s.batch(i)), ref.bulk_query(s.query(i)))[1]
                           for i in range(s.num_batches)])
    np.testing.assert_array_equal(got, want)
    np.testing.assert_array_equal(g.labels().cpu().numpy(), ref.labels())
    assert g.num_components() == ref.num_components()
    g.close()


def test_stream_kernel_small_grid_and_ragged(cc):
    # a grid smaller than one operation (grid-stride inside phases), empty batches
    sizes = [0, 5, 1000, 0, 3000, 1]
    n = 700
    e = synth.uniform_pairs(synth.key(17, 0, 1), 0, sum(sizes), n)
    q = synth.uniform_pairs(synth.key(17, 0, 2), 0, 333 * len(sizes), n)
    s = synth.Stream("ragged", n, e, synth._offsets(sizes), q, synth._offsets([333] * len(sizes)))
    g, got, rc = run_stream(cc, s, {}, max_items=64)
    assert rc == cc.cc.CC_OK
    ref = oracle.UnionFind(n)
    want = np.concatenate([(ref.bulk_update(s.batch(i)), ref.bulk_query(s.query(i)))[1]
                           for i in range(s.num_batches)])
    np.testing.assert_array_equal(got, want)
    g.close()


def test_stream_barrier_timeout_is_reported(cc):
    # forced from the host: a spin limit of 0 makes the first block that has
    # to wait give up; every block then leaves the kernel at its next barrier
    s = synth.er_stream(n=1 << 14, batches=8, batch=1 << 13, qbatch=1 << 12)
    g, got, rc = run_stream(cc, s, dict(spin_limit=0), max_items=1 << 20)
    assert rc == cc.cc.CC_EDEVICE
    assert g.sync() == cc.cc.CC_OK  # reported once
    g.close()
