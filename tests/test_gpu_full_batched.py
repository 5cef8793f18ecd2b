"""Full-size parity of the batched and served forms, in the configurations the
benchmark times, against one oracle per graph:

* the many-graph workload: 1024 graphs (log-normal sizes, 8n edges each in 4
  uneven minibatches, 2^12 query pairs per step), in the pool's per-round
  form and its one-launch form, with the benchmark's options: every answer,
  and every graph's labels and component count after each of the 4 steps;
* the serving workload: 1024 requests over 64 R-MAT scale-22 graphs through
  the continuous-batching scheduler (all requests at once, Poisson arrivals
  under a 256 MiB budget that forces evictions, and the serial form), every
  answer against the oracle of its stream, and all 64 streams re-run alone.
"""
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


def answers_equal(got: np.ndarray, want: np.ndarray, what: str):
    bad = np.flatnonzero(got != want)
    assert bad.size == 0, "%s: %d answers differ, first at pair %d" % (what, bad.size, bad[0])


class ManyGraphs:
    """The 1024-graph workload and the oracle's results after each step: all
    answers in one array laid out like the queries, every graph's labels in
    one array laid out like the graphs, and the component counts."""

    def __init__(self, G=1024, steps=4):
        self.ns = synth.multi_graph_sizes(G=G)
        self.streams = [synth.multi_graph_stream(g, int(self.ns[g])) for g in range(G)]
        self.G, self.steps = G, steps
        self.ebase = np.cumsum([0] + [len(s.edges) for s in self.streams])
        self.qbase = np.cumsum([0] + [len(s.queries) for s in self.streams])
        self.vbase = np.cumsum([0] + [s.n for s in self.streams])
        self.answers = np.empty(int(self.qbase[-1]), np.uint8)
        self.labels = [np.empty(int(self.vbase[-1]), np.int32) for _ in range(steps)]
        self.counts = np.empty((steps, G), np.int64)
        for g, s in enumerate(self.streams):
            ref = oracle.UnionFind(s.n)
            for k in range(steps):
                ref.bulk_update(s.batch(k))
                q0 = int(self.qbase[g] + s.qoff[k])
                self.answers[q0:q0 + len(s.query(k))] = ref.bulk_query(s.query(k))
                self.labels[k][int(self.vbase[g]):int(self.vbase[g + 1])] = ref.labels()
                self.counts[k, g] = ref.num_components()


@pytest.fixture(scope="module")
def many():
    m = ManyGraphs()
    print("many graphs: %d graphs, sum n=%d, %d edges, %d queries" % (
        m.G, int(m.vbase[-1]), int(m.ebase[-1]), int(m.qbase[-1])), flush=True)
    return m


@pytest.mark.timeout(900)
@pytest.mark.parametrize("one_launch", [0, 1], ids=["per-round", "one-launch"])
def test_batched1024_pool_full(cc, many, one_launch):
    from paper_1602_05232_amd import tuning
    m = many
    popts = tuning.lookup("pool", "mixed", int(np.median(m.ns))) or {}
    popts = {k: v for k, v in popts.items() if k not in ("update_mode", "compress_every")}
    popts["one_launch"] = one_launch
    print("pool form, options %s" % popts, flush=True)
    Eall = torch.from_numpy(np.concatenate([s.edges for s in m.streams])).cuda()
    Qall = torch.from_numpy(np.concatenate([s.queries for s in m.streams])).cuda()
    out = torch.zeros(len(m.answers), dtype=torch.uint8, device="cuda")
    lab = torch.empty(int(m.vbase[-1]), dtype=torch.int32, device="cuda")
    pool = cc.Pool(int(m.vbase[-1]), m.G, **popts)
    ids = [pool.add(s.n) for s in m.streams]
    for k in range(m.steps):
        ops = []
        for g, s in enumerate(m.streams):
            e0 = int(m.ebase[g] + s.eoff[k])
            ops.append((ids[g], cc.UPDATE, Eall[e0:e0 + len(s.batch(k))], None))
        for g, s in enumerate(m.streams):
            q0 = int(m.qbase[g] + s.qoff[k])
            q1 = q0 + len(s.query(k))
            ops.append((ids[g], cc.QUERY, Qall[q0:q1], out[q0:q1]))
        pool.run(ops)
        for g in range(m.G):
            pool.labels(ids[g], out=lab[int(m.vbase[g]):int(m.vbase[g + 1])])
        got = lab.cpu().numpy()
        bad = np.flatnonzero(got != m.labels[k])
        if bad.size:
            gbad = int(np.searchsorted(m.vbase, bad[0], side="right") - 1)
            raise AssertionError("step %d: %d labels differ, first in graph %d" % (k, bad.size, gbad))
        counts = [pool.num_components(ids[g]) for g in range(m.G)]
        assert counts == list(m.counts[k]), "component counts differ after step %d" % k
        print("  step %d: labels and counts of all %d graphs equal" % (k, m.G), flush=True)
    answers_equal(out.cpu().numpy(), m.answers, "pool answers")
    assert pool.sync() == cc.cc.CC_OK
    pool.close()


# ---------------------------------------------------------------------------
# serving

S, SCALE, R = 64, 22, 1024


@pytest.fixture(scope="module")
def trace():
    t = synth.serving_trace(S=S, scale=SCALE, R=R)
    n = 1 << SCALE
    want = {}
    for st in range(S):
        ref = oracle.UnionFind(n)
        for r in t:
            if r.stream != st:
                continue
            if r.kind == 0:
                ref.bulk_update(r.items)
            else:
                want[r.rid] = ref.bulk_query(r.items)
    dev = [torch.from_numpy(r.items).cuda() for r in t]
    print("serving trace: %d requests, %d update edges, %d query pairs" % (
        len(t), sum(r.size for r in t if r.kind == 0), sum(r.size for r in t if r.kind == 1)), flush=True)
    return t, dev, want


def serve_run(serve, popts, t, dev, want, arrivals, budget, form="served", only=None):
    n = 1 << SCALE
    reqs = []
    for r, items, a in zip(t, dev, arrivals):
        if only is not None and r.stream != only:
            continue
        o = torch.zeros(r.size, dtype=torch.uint8, device="cuda") if r.kind == 1 else None
        reqs.append(serve.Request(r.rid, r.stream, serve.UPDATE if r.kind == 0 else serve.QUERY, float(a), items,
                                  o, r.size))
    ex = serve.GpuExecutor(budget, S + 1, **popts)
    sch = serve.serial_scheduler(ex, [n] * S) if form == "serial" else serve.Scheduler(ex, [n] * S, 2)
    done = sch.run(reqs)
    torch.cuda.synchronize()
    for r in done:
        if r.kind == serve.QUERY:
            answers_equal(r.out.cpu().numpy(), want[r.rid], "%s form, request %d (stream %d)" % (form, r.rid, r.stream))
    assert ex.pool.sync() == 0
    ex.close()
    return sch


@pytest.mark.timeout(900)
def test_serve64_trace_full(cc, trace):
    from paper_1602_05232_amd import serve, tuning
    t, dev, want = trace
    n = 1 << SCALE
    popts = tuning.lookup("serve", "rmat", n) or tuning.lookup("pool", "mixed", n) or {}
    popts = {k: v for k, v in popts.items() if k not in ("update_mode", "compress_every")}
    popts["compress_linked"] = 0
    print("serving, options %s" % popts, flush=True)
    zeros = np.zeros(len(t))
    sch = serve_run(serve, popts, t, dev, want, zeros, S * n)
    print("  served, all at once: %d rounds, every answer equal" % sch.rounds, flush=True)
    serve_run(serve, popts, t, dev, want, zeros, S * n, form="serial")
    print("  serial: every answer equal", flush=True)
    arr = synth.poisson_arrivals(synth.key(synth.BASE_SEED + 5, 0, synth.P_ARRIVALS), len(t), 2.0e4)
    sch = serve_run(serve, popts, t, dev, want, arr, (256 << 20) // 4)
    assert sch.evictions > 0
    print("  served, Poisson arrivals, 256 MiB budget: %d evictions, every answer equal" % sch.evictions, flush=True)
    for st in range(S):
        serve_run(serve, popts, t, dev, want, zeros, n, only=st)
    print("  each of the %d streams alone: every answer equal" % S, flush=True)
