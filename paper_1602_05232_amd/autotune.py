"""Autotuner for the launch options of the connectivity kernels.

For a workload it times every candidate option set over full passes of the
workload's stream (median of `reps` passes after one warm-up) and stores the
fastest in tuned.json (see tuning.py) under the key the benchmark and the
tests look up for that workload.  No option changes any result; the tuner
still checks that every candidate ends with the same component count.

The plain forms are tuned in two stages: launch shape, linking order,
compression and filter first, then the compaction threshold
(CC_OPT_SPLIT_BELOW: the live-edge fraction below which an update compacts
its live edges before linking, Algorithm 2's relabel and filter, instead of
linking in place) on top of the stage-one winner.

  python -m paper_1602_05232_amd.autotune --workload rmat24
  python -m paper_1602_05232_amd.autotune --workload rmat24-unfiltered
  python -m paper_1602_05232_amd.autotune --workload er16
  python -m paper_1602_05232_amd.autotune --workload er16-stream
  python -m paper_1602_05232_amd.autotune --workload grid4096
  python -m paper_1602_05232_amd.autotune --workload grid4096-stream
  python -m paper_1602_05232_amd.autotune --workload batched1024
  python -m paper_1602_05232_amd.autotune --workload serve64

--log writes every candidate's time to a file (the sweep behind the entry).
"""
from __future__ import annotations

import argparse
import itertools
import json
import os
import sys
import time

import numpy as np
import torch

from . import tuning
from .cc import QUERY, UPDATE, Graph, Pool

SPLIT_THRESHOLDS = (5, 20, 50, 100)


def _median_pass(fn, reps):
    fn()  # warm-up
    torch.cuda.synchronize()
    ts = []
    for _ in range(reps):
        t0 = time.perf_counter()
        fn()
        torch.cuda.synchronize()
        ts.append(time.perf_counter() - t0)
    return float(np.median(ts))


def plain_candidates(quick=False, filtered=True):
    out = []
    for block, items, cl, hook in itertools.product((256, 512, 1024), (0, 4, 8), (0, 1), (0, 1, 2)):
        out.append(dict(update_mode=0, block=block, items=items, compress_linked=cl, hook=hook))
    out += [dict(update_mode=1, block=b, items=0, hook=h) for b in (256, 1024) for h in (0, 2)]
    if filtered:
        # the membership filter's form settles open edges per block, so it
        # prefers fewer, longer-lived blocks
        for block, gc, f, hook, qi in itertools.product((256, 512), (512, 768, 1024, 1280), (1, 2), (0, 1, 2),
                                                        (0, 2, 4)):
            out.append(dict(update_mode=0, block=block, items=1, grid_cap=gc, compress_linked=0, hook=hook,
                            filter=f, query_items=qi))
    if quick:
        out = out[::5]
    return out


def tune_plain(stream, workload, reps=3, quick=False, filtered=True, log=print):
    E = torch.from_numpy(stream.edges).cuda()
    Q = torch.from_numpy(stream.queries).cuda()
    out = torch.empty(len(stream.queries), dtype=torch.uint8, device="cuda")
    eoff = [int(x) for x in stream.eoff]
    qoff = [int(x) for x in stream.qoff]
    comps = [None]

    def measure(opts):
        full = dict(tuning.DEFAULTS)
        full.update(opts)
        g = Graph(stream.n, **full)
        g.reserve(max(eoff[i + 1] - eoff[i] for i in range(stream.num_batches)))

        def run():
            g.reset()
            for i in range(stream.num_batches):
                g.bulk_update(E[eoff[i]:eoff[i + 1]])
                g.bulk_query(Q[qoff[i]:qoff[i + 1]], out=out[qoff[i]:qoff[i + 1]])

        t = _median_pass(run, reps)
        c = g.num_components()
        assert comps[0] is None or c == comps[0], "component count depends on options"
        comps[0] = c
        g.close()
        log("  %-110s %.3f ms" % (opts, t * 1e3))
        return t, full

    best = None
    for opts in plain_candidates(quick, filtered):
        r = measure(opts)
        if best is None or r[0] < best[0]:
            best = r
    log("stage 1 best for %s: %s (%.3f ms)" % (workload, best[1], best[0] * 1e3))
    # stage 2: the compaction threshold on top of the stage-one winner (the
    # fused schedule only; the split schedule compacts every minibatch)
    if best[1].get("update_mode", 0) == 0:
        for th in SPLIT_THRESHOLDS:
            r = measure({**best[1], "split_below": th})
            if r[0] < best[0]:
                best = r
    log("best for %s: %s (%.3f ms)" % (workload, best[1], best[0] * 1e3))
    return best


def tune_stream(stream, reps=3, log=print):
    """The one-launch form (cc_bulk_stream): launch shape and linking order."""
    E = torch.from_numpy(stream.edges).cuda()
    Q = torch.from_numpy(stream.queries).cuda()
    eo = torch.from_numpy(stream.eoff.astype(np.int64)).cuda()
    qo = torch.from_numpy(stream.qoff.astype(np.int64)).cuda()
    out = torch.empty(len(stream.queries), dtype=torch.uint8, device="cuda")
    mx = int(max(np.diff(stream.eoff).max(), np.diff(stream.qoff).max()))
    best, comps = None, None
    for block, hook in itertools.product((64, 128, 256, 512), (0, 1, 2)):
        opts = dict(block=block, hook=hook)
        g = Graph(stream.n, **opts)

        def run():
            g.reset()
            g.bulk_stream(E, eo, Q, qo, out, max_items=mx)

        t = _median_pass(run, reps)
        c = g.num_components()
        assert comps is None or c == comps
        comps = c
        assert g.sync() == 0
        g.close()
        log("  %-40s %.3f ms" % (opts, t * 1e3))
        if best is None or t < best[0]:
            best = (t, opts)
    log("best for the one-launch form: %s (%.3f ms)" % (best[1], best[0] * 1e3))
    return best


def pool_candidates(quick=False):
    out = [dict(block=b, items=i, hook=h, compress_linked=c)
           for b, i, h, c in itertools.product((256, 512, 1024), (0, 4, 8), (0, 1, 2), (0, 1))]
    # launch width (blocks that stride over the tiles) for the family that
    # wins above: union by rank without linked-root compression
    out += [dict(block=b, items=i, hook=2, compress_linked=0, grid_cap=g)
            for b, i, g in itertools.product((256, 512, 1024), (0, 4), (1024, 2048, 8192))]
    # the membership filter (bits refreshed before each update round) on the
    # same family, and under hashed priority
    out += [dict(block=b, items=i, hook=2, compress_linked=0, filter=1)
            for b, i in itertools.product((256, 512, 1024), (0, 4, 8))]
    out += [dict(block=b, items=0, hook=1, compress_linked=0, filter=1) for b in (256, 512, 1024)]
    out += [dict(block=b, items=0, hook=2, compress_linked=0, filter=1, grid_cap=g)
            for b, g in itertools.product((256, 512), (1024, 2048, 8192))]
    return out[::5] if quick else out


def tune_pool(streams, reps=3, quick=False, log=print):
    G = len(streams)
    Eall = torch.from_numpy(np.concatenate([s.edges for s in streams])).cuda()
    Qall = torch.from_numpy(np.concatenate([s.queries for s in streams])).cuda()
    out = torch.empty(len(Qall), dtype=torch.uint8, device="cuda")
    eb = np.cumsum([0] + [len(s.edges) for s in streams])
    qb = np.cumsum([0] + [len(s.queries) for s in streams])
    total = sum(s.n for s in streams)
    best, comps = None, None
    for opts in pool_candidates(quick):
        pool = Pool(total, G, **opts)
        ids = [pool.add(s.n) for s in streams]
        steps = []
        for k in range(4):
            ops = [(ids[g], UPDATE, Eall[int(eb[g] + s.eoff[k]):int(eb[g] + s.eoff[k + 1])], None)
                   for g, s in enumerate(streams)]
            ops += [(ids[g], QUERY, Qall[int(qb[g] + s.qoff[k]):int(qb[g] + s.qoff[k + 1])],
                     out[int(qb[g] + s.qoff[k]):int(qb[g] + s.qoff[k + 1])]) for g, s in enumerate(streams)]
            steps.append(pool.prepare(ops))

        def run():
            pool.reset_all()
            for ops in steps:
                pool.run(ops)

        t = _median_pass(run, reps)
        c = sum(pool.num_components(i) for i in ids)
        assert comps is None or c == comps
        comps = c
        pool.close()
        log("  %-70s %.3f ms" % (opts, t * 1e3))
        if best is None or t < best[0]:
            best = (t, opts)
    log("best for the pool: %s (%.3f ms)" % (best[1], best[0] * 1e3))
    return best


def tune_serve(trace, n, reps=3, quick=False, log=print):
    """The served form: pool options of the executor, timed as the
    saturation run (every request at once) of the serving trace."""
    from . import serve
    S = 1 + max(r.stream for r in trace)
    items = [torch.from_numpy(r.items).cuda() for r in trace]
    best = None
    for opts in pool_candidates(quick):
        if opts["compress_linked"]:
            continue  # rounds overlap on two streams
        walls = []
        for _ in range(reps + 1):
            reqs = [serve.Request(r.rid, r.stream, serve.UPDATE if r.kind == 0 else serve.QUERY, 0.0, it,
                                  None if r.kind == 0 else torch.zeros(r.size, dtype=torch.uint8, device="cuda"),
                                  r.size) for r, it in zip(trace, items)]
            ex = serve.GpuExecutor(S * n, S + 1, **opts)
            sch = serve.Scheduler(ex, [n] * S, 2)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            sch.run(reqs)
            torch.cuda.synchronize()
            walls.append(time.perf_counter() - t0)
            assert ex.pool.sync() == 0
            ex.close()
        t = float(np.median(walls[1:]))
        log("  %-70s %.3f ms" % (opts, t * 1e3))
        if best is None or t < best[0]:
            best = (t, opts)
    log("best for the served form: %s (%.3f ms)" % (best[1], best[0] * 1e3))
    return best


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--workload", default="rmat24",
                    choices=["rmat24", "rmat24-unfiltered", "er16", "er16-stream", "grid4096", "grid4096-stream",
                             "batched1024", "serve64"])
    ap.add_argument("--reps", type=int, default=3)
    ap.add_argument("--quick", action="store_true")
    ap.add_argument("--log", default="", help="also write every candidate's time to this file")
    ap.add_argument("--copy-to", default="", help="also write the resulting table here")
    args = ap.parse_args()
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    sys.path.insert(0, root)
    import synth

    lines = []

    def log(*a):
        text = " ".join(str(x) for x in a)
        lines.append(text)
        print(text, flush=True)

    w = args.workload
    if w in ("rmat24", "rmat24-unfiltered"):
        s = synth.rmat_stream(scale=24)
        t, opts = tune_plain(s, w, args.reps, args.quick, filtered=w == "rmat24", log=log)
        tuning.store("plain", "rmat" if w == "rmat24" else "rmat-unfiltered", s.n, opts)
    elif w == "er16":
        s = synth.er_stream()
        t, opts = tune_plain(s, "er", args.reps, args.quick, log=log)
        tuning.store("plain", "er", s.n, opts)
    elif w == "er16-stream":
        s = synth.er_stream()
        t, opts = tune_stream(s, args.reps, log=log)
        tuning.store("stream", "er", s.n, opts)
    elif w == "grid4096":
        s = synth.grid_stream_cfg()
        t, opts = tune_plain(s, "grid", args.reps, args.quick, filtered=False, log=log)
        tuning.store("plain", "grid", s.n, opts)
    elif w == "grid4096-stream":
        s = synth.grid_stream_cfg()
        t, opts = tune_stream(s, args.reps, log=log)
        tuning.store("stream", "grid", s.n, opts)
    elif w == "batched1024":
        ns = synth.multi_graph_sizes(G=1024)
        streams = [synth.multi_graph_stream(g, int(ns[g])) for g in range(1024)]
        t, opts = tune_pool(streams, args.reps, args.quick, log)
        tuning.store("pool", "mixed", int(np.median(ns)), opts)
    else:
        trace = synth.serving_trace()
        t, opts = tune_serve(trace, 1 << 22, args.reps, args.quick, log)
        tuning.store("serve", "rmat", 1 << 22, opts)
    if args.copy_to:
        with open(tuning.CACHE) as f, open(args.copy_to, "w") as g:
            g.write(f.read())
    log(json.dumps({"workload": w, "best_ms": t * 1e3, "options": opts}))
    if args.log:
        with open(args.log, "w") as f:
            f.write("\n".join(lines) + "\n")


if __name__ == "__main__":
    main()
