"""The serving scheduler (continuous batching, per-stream order, memory-budget
admission and eviction) driven by the CPU oracle executor."""
import numpy as np

import oracle
import synth
from mock_executor import OracleExecutor
from paper_1602_05232_amd.serve import QUERY, UPDATE, Request, Scheduler, serial_scheduler


def make_trace(S=12, R=300, rate=2e5, seed=4, nmax=1 << 10, upd_frac=0.7):
    rng = np.random.default_rng(seed)
    ns = [int(rng.integers(nmax // 4, nmax)) for _ in range(S)]
    arrivals = np.cumsum(rng.exponential(1.0 / rate, size=R))
    reqs = []
    for i in range(R):
        s = int(rng.integers(0, S))
        kind = UPDATE if rng.random() < upd_frac else QUERY
        size = int(2 ** rng.uniform(2, 9))
        items = rng.integers(0, ns[s], size=(size, 2)).astype(np.int32)
        out = np.zeros(size, np.uint8) if kind == QUERY else None
        reqs.append(Request(i, s, kind, float(arrivals[i]), items, out, size))
    return ns, reqs


def expected_answers(ns, reqs):
    """Each stream's requests applied in arrival order to its own oracle."""
    refs = [oracle.UnionFind(n) for n in ns]
    want = {}
    for r in sorted(reqs, key=lambda r: r.arrival):
        if r.kind == UPDATE:
            refs[r.stream].bulk_update(r.items)
        else:
            want[r.rid] = refs[r.stream].bulk_query(r.items)
    return want, refs


def fresh(reqs):
    return [Request(r.rid, r.stream, r.kind, r.arrival, r.items,
                    None if r.out is None else np.zeros_like(r.out), r.size) for r in reqs]


def test_served_answers_equal_oracle_alone_and_in_mix(built_libs):
    ns, reqs = make_trace()
    want, _ = expected_answers(ns, reqs)
    ex = OracleExecutor(budget=sum(ns))
    done = Scheduler(ex, ns, max_inflight=2).run(fresh(reqs))
    got = {r.rid: r.out for r in done if r.kind == QUERY}
    assert set(got) == set(want)
    for rid in want:
        np.testing.assert_array_equal(got[rid], want[rid])
    # each stream alone gives the same answers
    for s in range(len(ns)):
        alone = [r for r in fresh(reqs) if r.stream == s]
        out = Scheduler(OracleExecutor(budget=ns[s]), ns, max_inflight=2).run(alone)
        for r in out:
            if r.kind == QUERY:
                np.testing.assert_array_equal(r.out, want[r.rid])


def test_continuous_batching_overlaps_and_keeps_stream_order(built_libs):
    ns, reqs = make_trace(rate=2e6)  # arrivals faster than service: queues build up
    ex = OracleExecutor(budget=sum(ns), launch_cost=20e-6)
    sch = Scheduler(ex, ns, max_inflight=2)
    done = sch.run(fresh(reqs))
    assert max(sch.round_sizes) > 1, "no round packed more than one request"
    assert ex.max_concurrent == 2, "rounds never overlapped"
    # per stream: launched and completed in arrival order
    for s in range(len(ns)):
        mine = [r for r in done if r.stream == s]
        starts = [t for (st, k, t) in ex.log if st == s]
        assert starts == sorted(starts)
        fin = [r.done_at for r in sorted(mine, key=lambda r: r.arrival)]
        assert fin == sorted(fin)
    assert all(r.latency >= 0 for r in done)


def test_budget_forces_eviction_without_changing_answers(built_libs):
    ns, reqs = make_trace(S=16, R=400, seed=8)
    want, refs = expected_answers(ns, reqs)
    budget = sorted(ns)[-1] * 3  # room for about three graphs
    ex = OracleExecutor(budget=budget)
    sch = Scheduler(ex, ns, max_inflight=2)
    done = sch.run(fresh(reqs))
    assert sch.evictions > 0 and ex.used <= budget
    for r in done:
        if r.kind == QUERY:
            np.testing.assert_array_equal(r.out, want[r.rid])
    # the kept state of every stream equals the oracle's
    for s in range(len(ns)):
        uf = ex.state.get(s) or ex.evicted.get(s)
        if uf is not None:
            np.testing.assert_array_equal(uf.labels(), refs[s].labels())


def test_serial_baseline_is_fifo(built_libs):
    ns, reqs = make_trace(R=120, rate=5e6)
    ex = OracleExecutor(budget=sum(ns))
    sch = serial_scheduler(ex, ns)
    done = sch.run(fresh(reqs))
    assert max(sch.round_sizes) == 1 and ex.max_concurrent == 1
    order = [s for (s, k, t) in ex.log]
    assert order == [r.stream for r in sorted(done, key=lambda r: r.arrival)]


def test_crash_mid_trace_and_replay_from_checkpoint(built_libs):
    """The executor is lost half way through a trace (the scheduler and every
    resident state with it).  A new executor takes the last checkpoint's
    images, the requests after the checkpoint are replayed, and every answer
    equals that of the uninterrupted run, under a budget that evicts."""
    ns, reqs = make_trace(S=10, R=400, seed=19, nmax=1 << 9)
    want, _ = expected_answers(ns, reqs)
    cut = 200
    budget = max(ns) * 3
    ex = OracleExecutor(budget)
    done = Scheduler(ex, ns, max_inflight=2).run(fresh(reqs[:cut]))
    images = ex.checkpoint()
    # requests after the checkpoint that the lost executor had started are
    # simply replayed; nothing of its state survives but the images
    Scheduler(ex, ns, max_inflight=2).run(fresh(reqs[cut:cut + 50]))
    del ex
    ex2 = OracleExecutor(budget)
    ex2.restore(images)
    t0 = min(r.arrival for r in reqs[cut:])
    rest = fresh(reqs[cut:])
    for r in rest:
        r.arrival -= t0
    done += Scheduler(ex2, ns, max_inflight=2).run(rest)
    got = {r.rid: r.out for r in done if r.kind == QUERY}
    assert set(got) == set(want)
    for rid, w in want.items():
        np.testing.assert_array_equal(got[rid], w, err_msg="request %d" % rid)
