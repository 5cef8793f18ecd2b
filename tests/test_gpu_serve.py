"""The serving loop on the GPU pool: every query answer equals the oracle's
for its stream, alone and in the mix, with and without evictions."""
import numpy as np
import pytest
import torch

from test_serve import expected_answers, make_trace

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def serve():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1602_05232_amd.serve as serve
    import paper_1602_05232_amd as ccgpu
    ccgpu.lib()
    return serve


def to_gpu(serve, reqs):
    out = []
    for r in reqs:
        items = torch.from_numpy(np.ascontiguousarray(r.items)).cuda()
        o = torch.zeros(r.size, dtype=torch.uint8, device="cuda") if r.kind == serve.QUERY else None
        out.append(serve.Request(r.rid, r.stream, r.kind, r.arrival, items, o, r.size))
    torch.cuda.synchronize()
    return out


@pytest.mark.parametrize("opts", [dict(), dict(hook=2, compress_linked=0, filter=1)],
                         ids=["default", "rank+filter"])
@pytest.mark.parametrize("budget_graphs", [None, 3])
def test_gpu_serving_matches_oracle(serve, budget_graphs, opts):
    # rank+filter: the pool's membership bits across two run streams,
    # evictions (save, remove) and readmissions (add, load)
    ns, reqs = make_trace(S=12, R=300, rate=5e4, seed=21, nmax=1 << 12)
    want, _ = expected_answers(ns, reqs)
    budget = sum(ns) if budget_graphs is None else max(ns) * budget_graphs
    ex = serve.GpuExecutor(budget, len(ns) + 1, **opts)
    sch = serve.Scheduler(ex, ns, max_inflight=2)
    done = sch.run(to_gpu(serve, reqs))
    torch.cuda.synchronize()
    for r in done:
        if r.kind == serve.QUERY:
            np.testing.assert_array_equal(r.out.cpu().numpy(), want[r.rid], err_msg="request %d" % r.rid)
    if budget_graphs is not None:
        assert sch.evictions > 0
    assert ex.pool.sync() == 0
    ex.close()
    # one stream alone
    s0 = [r for r in reqs if r.stream == 0]
    ex = serve.GpuExecutor(ns[0], 2, **opts)
    done = serve.Scheduler(ex, ns, max_inflight=2).run(to_gpu(serve, s0))
    torch.cuda.synchronize()
    for r in done:
        if r.kind == serve.QUERY:
            np.testing.assert_array_equal(r.out.cpu().numpy(), want[r.rid])
    ex.close()


@pytest.mark.parametrize("opts", [dict(), dict(hook=2, compress_linked=0, filter=1)],
                         ids=["default", "rank+filter"])
def test_gpu_serving_checkpoint_resume(serve, opts):
    """Serve the first half of a trace, checkpoint every stream, drop the
    executor, resume the second half on a fresh one: the answers are those of
    the uninterrupted run (the oracle's)."""
    ns, reqs = make_trace(S=10, R=240, rate=5e4, seed=33, nmax=1 << 12)
    want, _ = expected_answers(ns, reqs)
    first, second = reqs[:120], reqs[120:]
    ex = serve.GpuExecutor(max(ns) * 4, len(ns) + 1, **opts)
    done = serve.Scheduler(ex, ns, max_inflight=2).run(to_gpu(serve, first))
    images = ex.checkpoint()
    ex.close()
    t0 = min(r.arrival for r in second)
    for r in second:
        r.arrival -= t0
    ex2 = serve.GpuExecutor(max(ns) * 4, len(ns) + 1, **opts)
    ex2.restore(images)
    done += serve.Scheduler(ex2, ns, max_inflight=2).run(to_gpu(serve, second))
    torch.cuda.synchronize()
    for r in done:
        if r.kind == serve.QUERY:
            np.testing.assert_array_equal(r.out.cpu().numpy(), want[r.rid], err_msg="request %d" % r.rid)
    ex2.close()
