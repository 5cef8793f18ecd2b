"""Autotuner for the launch options of the connectivity kernels.

For a workload it times every candidate option set over full passes of the
workload's stream (median of `reps` passes after one warm-up) and stores the
fastest in tuned.json (see tuning.py).  No option changes any result; the
tuner still checks that every candidate ends with the same component count.

  python -m paper_1602_05232_amd.autotune --workload rmat24
  python -m paper_1602_05232_amd.autotune --workload grid4096
  python -m paper_1602_05232_amd.autotune --workload batched1024
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


def plain_candidates(quick=False):
    out = []
    for block, items, cl, hook in itertools.product((256, 512, 1024), (0, 4, 8), (0, 1), (0, 1, 2)):
        out.append(dict(update_mode=0, block=block, items=items, compress_linked=cl, hook=hook))
    out += [dict(update_mode=1, block=b, items=0) for b in (256, 1024)]
    # the membership filter's form settles open edges per block, so it
    # prefers fewer, longer-lived blocks
    for block, gc, f, hook, qi in itertools.product((256, 512), (512, 768, 1024, 1280), (1, 2), (0, 1, 2), (0, 2, 4)):
        out.append(dict(update_mode=0, block=block, items=1, grid_cap=gc, compress_linked=0, hook=hook, filter=f,
                        query_items=qi))
    if quick:
        out = out[::5]
    return out


def tune_plain(stream, workload, reps=3, quick=False, log=print):
    E = torch.from_numpy(stream.edges).cuda()
    Q = torch.from_numpy(stream.queries).cuda()
    out = torch.empty(len(stream.queries), dtype=torch.uint8, device="cuda")
    eoff = [int(x) for x in stream.eoff]
    qoff = [int(x) for x in stream.qoff]
    best = None
    comps = None
    for opts in plain_candidates(quick):
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
        assert comps is None or c == comps, "component count depends on options"
        comps = c
        g.close()
        log("  %-90s %.3f ms" % (opts, t * 1e3))
        if best is None or t < best[0]:
            best = (t, full)
    log("best for %s: %s (%.3f ms)" % (workload, best[1], best[0] * 1e3))
    return best


def pool_candidates(quick=False):
    out = [dict(block=b, items=i, hook=h, compress_linked=c)
           for b, i, h, c in itertools.product((256, 512, 1024), (0, 4, 8), (0, 1, 2), (0, 1))]
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
            steps.append(ops)

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


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--workload", default="rmat24", choices=["rmat24", "grid4096", "batched1024"])
    ap.add_argument("--reps", type=int, default=3)
    ap.add_argument("--quick", action="store_true")
    ap.add_argument("--copy-to", default="", help="also write the resulting table here")
    args = ap.parse_args()
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    sys.path.insert(0, root)
    import synth

    def log(*a):
        print(*a, flush=True)

    if args.workload == "rmat24":
        s = synth.rmat_stream(scale=24)
        t, opts = tune_plain(s, "rmat", args.reps, args.quick, log)
        tuning.store("plain", "rmat", s.n, opts)
    elif args.workload == "grid4096":
        s = synth.grid_stream_cfg()
        t, opts = tune_plain(s, "grid", args.reps, args.quick, log)
        tuning.store("plain", "grid", s.n, opts)
    else:
        ns = synth.multi_graph_sizes(G=1024)
        streams = [synth.multi_graph_stream(g, int(ns[g])) for g in range(1024)]
        t, opts = tune_pool(streams, args.reps, args.quick, log)
        tuning.store("pool", "mixed", int(np.median(ns)), opts)
    if args.copy_to:
        with open(tuning.CACHE) as f, open(args.copy_to, "w") as g:
            g.write(f.read())
    log(json.dumps({"workload": args.workload, "best_ms": t * 1e3, "options": opts}))


if __name__ == "__main__":
    main()
