"""The largest graphs the boundary accepts: n = 2^31 - 1 (int32 ids) and, for
union by rank, n = 2^27 (rank bits above the id).  Edges concentrate on both
ends of the id range, so the extreme ids are linked, queried and labelled.
Answers and counts are compared with the oracle; labels at sampled vertices
with the smallest id of each component, computed directly from the edges."""
import numpy as np
import pytest
import torch

import oracle

pytestmark = [pytest.mark.gpu, pytest.mark.slow]


@pytest.fixture(scope="module")
def cc():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1602_05232_amd as ccgpu
    ccgpu.lib()
    return ccgpu


def end_heavy_edges(n, m, seed):
    rng = np.random.default_rng(seed)
    span = 1 << 12
    ids = np.concatenate([np.arange(span), np.arange(n - span, n)]).astype(np.int64)
    e = ids[rng.integers(0, len(ids), size=(m, 2))]
    e[:4] = [[0, n - 1], [n - 1, n - 2], [1, n - 2], [n - 1, n - 1]]
    return e.astype(np.int32)


def min_labels(edges, vertices):
    """Smallest id of each vertex's component, by a dictionary union-find over
    the edges (every vertex no edge touches is alone)."""
    par = {}

    def find(x):
        par.setdefault(x, x)
        while par[x] != x:
            par[x] = par[par[x]]
            x = par[x]
        return x

    for u, v in edges.tolist():
        a, b = find(u), find(v)
        if a != b:
            par[max(a, b)] = min(a, b)  # the smaller id stays the root
    return np.array([find(int(x)) for x in vertices], dtype=np.int64)


@pytest.mark.timeout(600)
@pytest.mark.parametrize("n,opts", [((1 << 31) - 1, dict()), ((1 << 31) - 1, dict(update_mode=2)),
                                    ((1 << 31) - 1, dict(filter=2)),
                                    (1 << 27, dict(hook=2)), (1 << 27, dict(hook=2, find=1)),
                                    (1 << 27, dict(hook=2, filter=2))],
                         ids=["2^31-1-fused", "2^31-1-contract", "2^31-1-filter", "2^27-rank", "2^27-rank-bulkfind",
                              "2^27-rank-filter"])
def test_maximum_vertex_count(cc, n, opts):
    print("max size: n=%d opts=%s" % (n, opts), flush=True)
    edges = end_heavy_edges(n, 30000, seed=n % 1000)
    rng = np.random.default_rng(3)
    probe = np.concatenate([np.arange(16), n - 1 - np.arange(16), rng.integers(0, n, 64)]).astype(np.int64)
    pairs = probe[rng.integers(0, len(probe), size=(4096, 2))].astype(np.int32)
    ref = oracle.UnionFind(n)
    g = cc.Graph(n, **opts)
    for b in np.array_split(edges, 3):
        ref.bulk_update(b)
        g.bulk_update(torch.from_numpy(np.ascontiguousarray(b)).cuda())
        np.testing.assert_array_equal(g.bulk_query(torch.from_numpy(pairs).cuda()).cpu().numpy(),
                                      ref.bulk_query(pairs))
    assert g.num_components() == ref.num_components() == g.count_roots()
    if opts.get("filter"):
        anchor, complete, _, _ = g.filter_state()
        assert anchor >= 0 and complete  # the bitmaps took part
    lab = g.labels()
    got = lab[torch.from_numpy(probe).cuda()].cpu().numpy()
    np.testing.assert_array_equal(got, min_labels(edges, probe))
    del lab
    assert g.sync() == cc.cc.CC_OK
    g.close()
    torch.cuda.empty_cache()


def test_size_limits(cc):
    L = cc.lib()
    assert not L.cc_create(1 << 31)  # ids are int32
    assert not L.cc_create(0)
    g = cc.Graph((1 << 27) + 1)
    with pytest.raises(cc.CCError) as ei:
        g.set_option("hook", 2)  # rank bits need ids below 2^27
    assert ei.value.code == cc.cc.CC_EINVAL
    g.close()
