#!/usr/bin/env python3
"""Throughput benchmark of the bulk incremental connectivity hot path.

Default workload (`--workload rmat24`, the headline configuration): one step
is one pass of the whole path over the R-MAT scale-24 stream (n = 2^24
vertices, 2^28 edges with a=.57 b=.19 c=.19 d=.05 and randomly permuted ids,
streamed as minibatches of log-uniform size in [2^16, 2^24], each followed by
a Bulk-Query of 2^20 uniform random pairs): reset the forest, every
Bulk-Update and Bulk-Query in stream order, then the min-id label pass and the
component count.  Inputs are generated on the host and resident in HBM before
timing starts.

Other workloads compare the forms of the path on their own configurations:
  grid4096     4096^2 mesh + 1% long-range edges, 2^12-edge minibatches each
               followed by 2^10 queries: plain launches vs one HIP-graph replay
  batched1024  1024 independent graphs (log-normal sizes): one launch per
               graph and operation vs the pool's one launch per round
  serve64      request loop over 64 R-MAT scale-22 graphs, Poisson arrivals of
               70% updates / 30% queries: continuous batching vs serial plain,
               saturation throughput and p50/p99 latency
  bigbatch     the R-MAT scale-24 and an Erdos-Renyi (n = 2^24, 5n edges) edge
               set in 1, 8 and 64 equal minibatches: Bulk-Update throughput of
               the fused (CAS) schedule under each linking order against the
               contracting schedule (Algorithm 2 with rounds on A'')
  components   number of components along each workload shape's stream

Prints ONE JSON line.  `value` is (update edges + query pairs) per second of
wall clock over the timed steps.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "Bulk-Update edges/s + Bulk-Query queries/s, batched vs plain; p50/p99 latency"
HBM_PEAK_GBS = 8000.0
# algorithmic bytes per update edge: 8 B of ids streamed + two random 4-B parent reads
UPDATE_BYTES_PER_EDGE = 16
EV_STEPS = 3  # timed steps of the R-MAT stream that record kernel intervals
PAPER_CONTEXT = {"value": 167.68e6, "unit": "edges/s",
                 "what": "Bulk-Update, rMat16 (2^27 vertices, 1.6e9 edges), b=10M, 20-core Xeon (Table 3)"}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


# sources of the update kernel: a change to any voids stored counter readings
KERNEL_SOURCES = ("uf_device.hpp", "cc_kernels.hpp", "cc_member_kernels.hpp", "cc_grid.hpp")


def source_digest() -> str:
    h = hashlib.sha256()
    d = os.path.join(ROOT, "paper_1602_05232_amd", "csrc")
    for f in KERNEL_SOURCES:
        with open(os.path.join(d, f), "rb") as fh:
            h.update(f.encode() + b"\0" + fh.read())
    return h.hexdigest()[:16]


def load_counter(file_tag: str, key: str):
    """A figure from a committed counter summary (profiles/pmc_<tag>.txt), if
    the counters were taken on the current kernel sources."""
    p = os.path.join(ROOT, "profiles", "pmc_%s.txt" % file_tag)
    if not os.path.exists(p):
        return None
    kv = {}
    for line in open(p):
        if ":" in line and not line.startswith(" "):
            k, v = line.split(":", 1)
            kv[k.strip()] = v.strip()
    if kv.get("source_digest") != source_digest():
        return None
    try:
        return float(kv[key])
    except (KeyError, ValueError):
        return None


def load_traffic(kernel_tag: str):
    """HBM traffic per launch (FETCH_SIZE + WRITE_SIZE, calibrated)."""
    return load_counter(kernel_tag, "traffic_bytes_per_launch")


def pct(xs, p):
    xs = sorted(xs)
    if not xs:
        return None
    k = min(len(xs) - 1, max(0, int(round(p / 100.0 * (len(xs) - 1)))))
    return xs[k]


def host_info() -> dict:
    """The host the CPU baseline ran on: model name, clock, logical CPUs."""
    info = {"nproc": os.cpu_count()}
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                k, _, v = line.partition(":")
                k = k.strip()
                if k == "model name" and "model" not in info:
                    info["model"] = v.strip()
                elif k == "cpu MHz" and "mhz" not in info:
                    info["mhz"] = float(v)
    except OSError:
        pass
    return info


def cpu_baseline(streams, budget_s: float):
    """The oracle, as it is, on a prefix of the same work (one thread)."""
    import oracle
    edges = queries = 0
    t0 = time.perf_counter()
    done = []
    for s in streams:
        uf = oracle.UnionFind(s.n)
        nb = 0
        for i in range(s.num_batches):
            uf.bulk_update(s.batch(i))
            uf.bulk_query(s.query(i))
            edges += int(s.eoff[i + 1] - s.eoff[i])
            queries += int(s.qoff[i + 1] - s.qoff[i])
            nb = i + 1
            if time.perf_counter() - t0 > budget_s:
                break
        done.append((s.name, nb, s.num_batches))
        if time.perf_counter() - t0 > budget_s:
            break
    dt = time.perf_counter() - t0
    what = "; ".join("%s: %d of %d minibatches" % d for d in done[:3])
    if len(done) > 3:
        what += "; ... %d streams in all" % len(done)
    return {"value": (edges + queries) / dt, "unit": "edges+queries/s", "cores": 1, "kind": "oracle",
            "sample": "%s, each with its query batches (%d edges, %d queries, %.1f s)" % (what, edges, queries, dt),
            "update_edges": edges, "queries": queries, "seconds": dt, "host": host_info()}


def parse_options(text: str) -> dict:
    """Option overrides: a JSON object, or key=value pairs separated by commas
    (integer values), e.g. find=1,hook=2."""
    text = text.strip()
    if not text:
        return {}
    if text.startswith("{"):
        return json.loads(text)
    out = {}
    for part in text.split(","):
        k, v = part.split("=", 1)
        out[k.strip()] = int(v)
    return out


def result(value, steps, warmup, wall, config, dtype="int32"):
    return {"metric": METRIC, "value": value, "unit": "edges+queries/s", "n_gpus": 1, "steps": steps,
            "warmup": warmup, "ms_per_step": wall / max(1, steps) * 1e3, "higher_is_better": True,
            "scaling": "weak", "vs_baseline": None, "dtype": dtype, "data": "synthetic", "config": config}


# ---------------------------------------------------------------------------

def run_rmat(args):
    import torch

    import synth
    import paper_1602_05232_amd as ccgpu
    from paper_1602_05232_amd import roofline, tuning

    t = time.perf_counter()
    s = synth.rmat_stream(scale=args.scale)
    log("generated %s: n=%d edges=%d minibatches=%d queries=%d in %.1fs"
        % (s.name, s.n, len(s.edges), s.num_batches, len(s.queries), time.perf_counter() - t))
    M, Qn, nb = len(s.edges), len(s.queries), s.num_batches
    opts = tuning.plain_options(s.n, workload="rmat")
    if args.options:
        opts.update(parse_options(args.options))
    E = torch.from_numpy(s.edges).cuda()
    Q = torch.from_numpy(s.queries).cuda()
    out = torch.empty(Qn, dtype=torch.uint8, device="cuda")
    lab = torch.empty(s.n, dtype=torch.int32, device="cuda")
    eoff = [int(x) for x in s.eoff]
    qoff = [int(x) for x in s.qoff]
    g = ccgpu.Graph(s.n, **opts)
    g.reserve(max(eoff[i + 1] - eoff[i] for i in range(nb)))
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    # ev[2i] .. ev[2i+1]: update i; ev[2i+1] .. ev[2i+2]: query i.  Timing-only
    # events: a default event's cache writeback per record costs ~3.6 us of
    # GPU time, 0.8 ms per step at three records per minibatch.  Each
    # recording step records into its own set, read after the timed region,
    # so that reading 2 * nb intervals on the host is not counted as step
    # time.  Only the first EV_STEPS timed steps record: the 2 * nb + 1
    # records still cost about 0.17 ms of a 5.7 ms step, which the other
    # steps do not pay.
    nev = max(1, min(args.steps, EV_STEPS))
    ev_sets = [[roofline.TimingEvent() for _ in range(2 * nb + 1)] for _ in range(nev)]
    Es = [E[eoff[i]:eoff[i + 1]] for i in range(nb)]
    Qs = [Q[qoff[i]:qoff[i + 1]] for i in range(nb)]
    Os = [out[qoff[i]:qoff[i + 1]] for i in range(nb)]

    def step(ev):
        g.reset()
        for i in range(nb):
            if ev:
                ev[2 * i].record(stream)
            g.bulk_update(Es[i])
            if ev:
                ev[2 * i + 1].record(stream)
            g.bulk_query(Qs[i], out=Os[i])
        if ev:
            ev[2 * nb].record(stream)
        g.labels(out=lab)
        return g.num_components()  # waits for the stream

    for k in range(args.warmup):
        c = step(ev_sets[0])
        log("warmup step %d done: components=%d" % (k, c))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        c = step(ev_sets[k] if k < nev else None)
        log("step %d done: components=%d" % (k, c))
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    upd_t, qry_t, upd_lat = [], [], []
    for k in range(min(args.steps, nev)):
        ev = ev_sets[k]
        tu = [ev[2 * i].elapsed_time(ev[2 * i + 1]) / 1e3 for i in range(nb)]
        tq = [ev[2 * i + 1].elapsed_time(ev[2 * i + 2]) / 1e3 for i in range(nb)]
        upd_t.append(sum(tu))
        qry_t.append(sum(tq))
        upd_lat.extend(x * 1e3 for x in tu)
        log("step %d: update %.4fs query %.4fs" % (k, upd_t[-1], qry_t[-1]))
    rc = g.sync()
    if rc != 0:
        raise SystemExit("device reported status %d" % rc)
    for ev in ev_sets:  # released here, not at interpreter shutdown
        for e in ev:
            e.close()
    steps = max(1, args.steps)
    esteps = len(upd_t)  # steps whose kernel intervals were recorded
    upd_rate = esteps * M / sum(upd_t)
    qry_rate = esteps * Qn / sum(qry_t)
    res = result(steps * (M + Qn) / wall, args.steps, args.warmup, wall, {
        "workload": "rmat%d-plain" % args.scale, "n": s.n, "edges": M, "minibatches": nb,
        "minibatch_sizes": "log-uniform in [2^16, 2^24]", "queries_per_minibatch": qoff[1] - qoff[0],
        "rmat_abcd": [0.57, 0.19, 0.19, 0.05], "form": "plain", "options": opts})
    res.update({"update_edges_per_s": upd_rate, "queries_per_s": qry_rate,
                "update_op_ms": {"p50": pct(upd_lat, 50), "p99": pct(upd_lat, 99)},
                "components": c, "paper_context": PAPER_CONTEXT})
    if not args.no_roofline:
        fused = opts.get("update_mode", 0) == 0
        tag = ("update_fused_rmat%d" if fused else "update_split_rmat%d") % args.scale
        achieved = UPDATE_BYTES_PER_EDGE * upd_rate / 1e9
        traffic = load_traffic(tag)
        res["roofline"] = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                           "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                           "traffic_rate_GBs": None if traffic is None else
                           traffic * nb * esteps / sum(upd_t) / 1e9,
                           "l2_hit_rate": load_counter("l2_" + tag, "l2_hit_rate"),
                           "kernel": "k_update_fused" if fused else "k_filter+k_link_live+k_compress_live",
                           "bytes_per_edge": UPDATE_BYTES_PER_EDGE,
                           "avg_update_ms": sum(upd_t) / (esteps * nb) * 1e3,
                           "event_steps": esteps,
                           "bytes_per_update": UPDATE_BYTES_PER_EDGE * M / nb}
        del E, Q, Es, Qs, Os
        torch.cuda.empty_cache()
        G = roofline.gather_rate(s.n)
        Gbig = roofline.gather_rate(1 << 30, count=1 << 27)
        Gsmall = {"2^16": roofline.gather_rate(1 << 16), "2^22": roofline.gather_rate(1 << 22)}
        Bs = roofline.stream_bandwidth()
        C = roofline.cas_rate(s.n)
        Eroof = roofline.edge_roofline(G, Bs)
        links = s.n - c
        res["gather_roofline"] = {
            "G_gathers_per_s_table_n": G, "G_gathers_per_s_table_2^30": Gbig,
            "G_gathers_per_s_table_2^16": Gsmall["2^16"], "G_gathers_per_s_table_2^22": Gsmall["2^22"],
            "C_cas_per_s_table_n": C, "links_per_step": links,
            "links_per_s_in_update": links * esteps / sum(upd_t),
            "stream_read_GBs": Bs / 1e9,
            "E_roof_edges_per_s": Eroof, "frac": upd_rate / Eroof,
            "E_roof_beyond_cache_edges_per_s": roofline.edge_roofline(Gbig, Bs),
            "query_roof_per_s": G / 2.0, "query_frac": qry_rate / (G / 2.0),
            "note": "E_roof = 1/(2/G + 8/B_s): two random parent reads and 8 streamed bytes per edge"}
        log("gather roofline: G(n)=%.3g/s G(2^30)=%.3g/s B_s=%.1f GB/s E_roof=%.3g e/s frac=%.3f"
            % (G, Gbig, Bs / 1e9, Eroof, upd_rate / Eroof))
        if opts.get("filter", 0):
            # ceilings of the membership filter's fast paths: an edge settled
            # by its two membership words, and a query pair priced the same
            # (its first touched word alone settles a pair whose first end
            # never had an edge; two touched ends take up to four words), each
            # plus its 8 streamed bytes
            words = (s.n + 31) // 32
            Gb = roofline.gather_rate(words)
            Ef = 1.0 / (2.0 / Gb + 8.0 / Bs)
            Qf = Ef
            res["gather_roofline"]["filter"] = {
                "bitmap_words": words, "G_gathers_per_s_table_bitmap": Gb,
                "E_filter_roof_edges_per_s": Ef, "update_frac_of_filter_roof": upd_rate / Ef,
                "Q_filter_roof_per_s": Qf, "query_frac_of_filter_roof": qry_rate / Qf,
                "note": "ceiling if every edge (query pair) were settled by two bitmap words: "
                        "1/(2/G_b + 8/B_s) per item, G_b = gathers/s from a table of the bitmap's size; "
                        "a query pair reads one to four words"}
            log("filter roofline: G(bitmap)=%.3g/s E_f=%.3g e/s (frac %.3f) Q_f=%.3g q/s (frac %.3f)"
                % (Gb, Ef, upd_rate / Ef, Qf, qry_rate / Qf))
        # which measured ceiling binds this path: a fraction above 1 means the
        # path does not do the work that denominator prices (the filter turns
        # parent gathers into bitmap hits), so that ceiling does not bind it
        gr = res["gather_roofline"]
        cands = {"E_roof (two parent gathers from a table of n + 8 streamed bytes per edge)":
                 (gr["E_roof_edges_per_s"], gr["frac"], gr["query_roof_per_s"], gr["query_frac"])}
        if "filter" in gr:
            f = gr["filter"]
            cands["E_f (two bitmap gathers + 8 streamed bytes per item)"] = (
                f["E_filter_roof_edges_per_s"], f["update_frac_of_filter_roof"], f["Q_filter_roof_per_s"],
                f["query_frac_of_filter_roof"])
        binding = {k: v for k, v in cands.items() if v[1] <= 1.0 and v[3] <= 1.0}
        name = min(binding, key=lambda k: binding[k][0]) if binding else None
        res["roofline"]["binding_ceiling"] = None if name is None else {
            "name": name, "update_edges_per_s": binding[name][0], "update_frac": binding[name][1],
            "query_pairs_per_s": binding[name][2], "query_frac": binding[name][3]}
        res["roofline"]["non_binding"] = {k: {"update_frac": v[1], "query_frac": v[3]}
                                          for k, v in cands.items() if k != name}
    g.close()
    if not args.no_forms:
        res["hipgraph"] = rmat_hipgraph(s, opts, max(5, min(args.steps, 20)))
        log("hipgraph: %.3f ms per pass against %.3f ms for plain launches (%.3fx)" % (
            res["hipgraph"]["ms_per_step"], res["hipgraph"]["plain_ms_per_step"],
            res["hipgraph"]["speedup_vs_plain"]))
    if opts.get("filter", 0) and not args.no_forms:
        res["unfiltered"] = rmat_unfiltered(s, opts, max(2, min(args.steps, 5)))
        log("unfiltered: update %.3g edges/s, query %.3g pairs/s" % (
            res["unfiltered"]["update_edges_per_s"], res["unfiltered"]["queries_per_s"]))
    if not args.no_cpu_baseline:
        res["cpu_baseline"] = cpu_baseline([s], args.cpu_budget)
        log("cpu baseline: %s" % res["cpu_baseline"]["sample"])
    return res


def rmat_hipgraph(s, opts, steps):
    """The same pass (reset, every update and query, labels, count) captured
    once and replayed as one HIP graph, against the same plain launches
    without timing events, both on one stream of their own; every replay's
    answers and count must equal the plain pass's."""
    import torch

    import paper_1602_05232_amd as ccgpu

    st = torch.cuda.Stream()  # capture needs a stream of its own
    torch.cuda.set_stream(st)
    nb = s.num_batches
    E = torch.from_numpy(s.edges).cuda()
    Q = torch.from_numpy(s.queries).cuda()
    out = torch.empty(len(s.queries), dtype=torch.uint8, device="cuda")
    lab = torch.empty(s.n, dtype=torch.int32, device="cuda")
    eoff = [int(x) for x in s.eoff]
    qoff = [int(x) for x in s.qoff]
    Es = [E[eoff[i]:eoff[i + 1]] for i in range(nb)]
    Qs = [Q[qoff[i]:qoff[i + 1]] for i in range(nb)]
    Os = [out[qoff[i]:qoff[i + 1]] for i in range(nb)]
    g = ccgpu.Graph(s.n, stream=st, **opts)
    g.reserve(max(eoff[i + 1] - eoff[i] for i in range(nb)))

    def calls():
        g.reset()
        for i in range(nb):
            g.bulk_update(Es[i])
            g.bulk_query(Qs[i], out=Os[i])
        g.labels(out=lab)

    def plain():
        calls()
        return g.num_components()  # waits for the stream

    def timed(fn):
        c = fn()
        ts = []
        for _ in range(steps):
            st.synchronize()
            t0 = time.perf_counter()
            c = fn()
            ts.append(time.perf_counter() - t0)
        return sorted(ts)[len(ts) // 2], c

    t_plain, c = timed(plain)
    want = out.clone()
    with g.capture() as cap:
        calls()
    rec = cap.recording

    def replay():
        rec.launch()
        return g.num_components()

    out.zero_()
    t_graph, c2 = timed(replay)
    assert c2 == c and torch.equal(out, want), "HIP-graph replay differs from plain launches"
    rec.close()
    assert g.sync() == 0
    g.close()
    torch.cuda.set_stream(torch.cuda.default_stream())
    items = len(s.edges) + len(s.queries)
    return {"value": items / t_graph, "ms_per_step": t_graph * 1e3, "plain_ms_per_step": t_plain * 1e3,
            "speedup_vs_plain": t_plain / t_graph, "steps": steps,
            "what": "the pass captured once (cc_capture_*) and replayed as one HIP graph; plain_ms_per_step is the "
                    "same calls launched one by one on the same stream, without timing events (medians)"}


def rmat_unfiltered(s, opts, steps):
    """The same stream without the membership filter (union by rank, the
    unfiltered path's own launch shape): every edge and pair takes its two
    parent gathers, the work E_roof prices."""
    import torch

    import paper_1602_05232_amd as ccgpu
    from paper_1602_05232_amd import roofline, tuning

    uo = dict(opts)
    uo.update(tuning.lookup("plain", "rmat-unfiltered", s.n) or dict(filter=0, block=1024, items=0, grid_cap=4096))
    uo["filter"] = 0
    E = torch.from_numpy(s.edges).cuda()
    Q = torch.from_numpy(s.queries).cuda()
    out = torch.empty(len(s.queries), dtype=torch.uint8, device="cuda")
    nb = s.num_batches
    Es = [E[int(s.eoff[i]):int(s.eoff[i + 1])] for i in range(nb)]
    Qs = [Q[int(s.qoff[i]):int(s.qoff[i + 1])] for i in range(nb)]
    Os = [out[int(s.qoff[i]):int(s.qoff[i + 1])] for i in range(nb)]
    g = ccgpu.Graph(s.n, **uo)
    stream = torch.cuda.current_stream()
    ev = [roofline.TimingEvent() for _ in range(2 * nb + 1)]
    tu, tq = [], []
    for k in range(steps + 1):
        g.reset()
        for i in range(nb):
            ev[2 * i].record(stream)
            g.bulk_update(Es[i])
            ev[2 * i + 1].record(stream)
            g.bulk_query(Qs[i], out=Os[i])
        ev[2 * nb].record(stream)
        torch.cuda.synchronize()
        if k > 0:  # the first pass warms up
            tu.append(sum(ev[2 * i].elapsed_time(ev[2 * i + 1]) for i in range(nb)) / 1e3)
            tq.append(sum(ev[2 * i + 1].elapsed_time(ev[2 * i + 2]) for i in range(nb)) / 1e3)
    assert g.sync() == 0
    g.close()
    for e in ev:
        e.close()
    M, Qn = len(s.edges), len(s.queries)
    return {"update_edges_per_s": M * len(tu) / sum(tu), "queries_per_s": Qn * len(tq) / sum(tq),
            "update_ms_per_pass": sum(tu) / len(tu) * 1e3, "query_ms_per_pass": sum(tq) / len(tq) * 1e3,
            "options": uo, "steps": len(tu)}


def run_er(args):
    """The tiny uniform stream: n = 2^16, 16 minibatches of 2^14 uniform edges
    (self-loops and repeats kept), each followed by 2^14 uniform query pairs.
    Launch-latency bound: a pass is 32 operations of 2^14 items.  The value
    is the plain form's; the pass replayed as one HIP graph and run as one
    cooperative launch (cc_bulk_stream) are reported beside it, each checked
    answer for answer against the plain launches."""
    import torch

    import synth
    import paper_1602_05232_amd as ccgpu
    from paper_1602_05232_amd import tuning

    s = synth.er_stream()
    M, Qn, nb = len(s.edges), len(s.queries), s.num_batches
    opts = tuning.plain_options(s.n, workload="er")
    if args.options:
        opts.update(parse_options(args.options))
    st = torch.cuda.Stream()  # capture needs a stream of its own
    torch.cuda.set_stream(st)
    E = torch.from_numpy(s.edges).cuda()
    Q = torch.from_numpy(s.queries).cuda()
    out = torch.empty(Qn, dtype=torch.uint8, device="cuda")
    lab = torch.empty(s.n, dtype=torch.int32, device="cuda")
    g = ccgpu.Graph(s.n, stream=st, **opts)
    g.reserve(int(s.eoff[1] - s.eoff[0]))
    Es = [E[int(s.eoff[i]):int(s.eoff[i + 1])] for i in range(nb)]
    Qs = [Q[int(s.qoff[i]):int(s.qoff[i + 1])] for i in range(nb)]
    Os = [out[int(s.qoff[i]):int(s.qoff[i + 1])] for i in range(nb)]

    def step():
        g.reset()
        for i in range(nb):
            g.bulk_update(Es[i])
            g.bulk_query(Qs[i], out=Os[i])
        g.labels(out=lab)
        return g.num_components()

    def run(fn):
        for _ in range(max(1, args.warmup)):
            c = fn()
        times = []
        for _ in range(max(5, args.steps)):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            c = fn()
            times.append(time.perf_counter() - t0)
        return sorted(times)[len(times) // 2], times, c

    steps = max(5, args.steps)
    med, times, c = run(step)
    want = out.clone()
    # the same pass replayed as one HIP graph, and as one cooperative launch
    with g.capture() as cap:
        g.reset()
        for i in range(nb):
            g.bulk_update(Es[i])
            g.bulk_query(Qs[i], out=Os[i])
        g.labels(out=lab)
    rec = cap.recording

    def replay():
        rec.launch()
        return g.num_components()

    out.zero_()
    med_graph, _, c2 = run(replay)
    assert c2 == c and torch.equal(out, want), "replay differs from plain launches"
    rec.close()
    eo = torch.from_numpy(s.eoff.astype("int64")).cuda()
    qo = torch.from_numpy(s.qoff.astype("int64")).cuda()
    mx = int(max((s.eoff[1:] - s.eoff[:-1]).max(), (s.qoff[1:] - s.qoff[:-1]).max()))
    stream_opts = tuning.lookup("stream", "er", s.n) or tuning.lookup("stream", "grid", 1 << 24) or {}
    g.reset()
    for k, v in stream_opts.items():
        g.set_option(k, v)

    def one_launch():
        g.reset()
        g.bulk_stream(E, eo, Q, qo, out, max_items=mx)
        g.labels(out=lab)
        return g.num_components()

    out.zero_()
    med_stream, _, c3 = run(one_launch)
    assert c3 == c and torch.equal(out, want), "stream kernel differs from plain launches"
    assert g.sync() == 0
    g.close()
    torch.cuda.set_stream(torch.cuda.default_stream())
    res = result((M + Qn) / med, steps, args.warmup, sum(times), {
        "workload": "er16-plain", "n": s.n, "edges": M, "minibatches": nb, "minibatch": 1 << 14,
        "queries_per_minibatch": 1 << 14, "form": "plain", "options": opts})
    forms = {"plain": med, "hipgraph": med_graph, "stream_kernel": med_stream}
    res.update({"median_ms_per_pass": med * 1e3, "components": c,
                "forms": {k: {"value": (M + Qn) / v, "median_ms_per_pass": v * 1e3,
                              "speedup_vs_plain": med / v} for k, v in forms.items()},
                "stream_kernel_options": stream_opts})
    return res


def run_grid(args):
    import numpy as np
    import torch

    import synth
    import paper_1602_05232_amd as ccgpu
    from paper_1602_05232_amd import tuning

    t = time.perf_counter()
    s = synth.grid_stream_cfg()
    log("generated %s: n=%d edges=%d minibatches=%d in %.1fs" % (s.name, s.n, len(s.edges), s.num_batches,
                                                                  time.perf_counter() - t))
    M, Qn, nb = len(s.edges), len(s.queries), s.num_batches
    opts = tuning.plain_options(s.n, workload="grid")
    if args.options:
        opts.update(parse_options(args.options))
    st = torch.cuda.Stream()
    with torch.cuda.stream(st):
        E = torch.from_numpy(s.edges).cuda()
        Q = torch.from_numpy(s.queries).cuda()
        out = torch.empty(Qn, dtype=torch.uint8, device="cuda")
        lab = torch.empty(s.n, dtype=torch.int32, device="cuda")
        g = ccgpu.Graph(s.n, stream=st, **opts)
        g.reserve(int(np.diff(s.eoff).max()))
        eoff = [int(x) for x in s.eoff]
        qoff = [int(x) for x in s.qoff]

        def sequence():
            g.reset()
            for i in range(nb):
                g.bulk_update(E[eoff[i]:eoff[i + 1]])
                g.bulk_query(Q[qoff[i]:qoff[i + 1]], out=out[qoff[i]:qoff[i + 1]])
            g.labels(out=lab)

        def timed(fn, steps, warmup, name):
            for _ in range(warmup):
                fn()
                c = g.num_components()
            st.synchronize()
            t0 = time.perf_counter()
            for k in range(steps):
                fn()
                c = g.num_components()
                log("%s step %d done: components=%d" % (name, k, c))
            st.synchronize()
            return time.perf_counter() - t0, c

        wall_plain, c1 = timed(sequence, args.steps, args.warmup, "plain")
        want = out.clone()
        t = time.perf_counter()
        with g.capture() as cap:
            sequence()
        rec = cap.recording
        log("captured %d minibatches in %.2fs" % (nb, time.perf_counter() - t))
        wall_graph, c2 = timed(rec.launch, args.steps, args.warmup, "graph")
        assert c1 == c2 and torch.equal(out, want), "replay differs from plain launches"
        rec.close()
        eo = torch.from_numpy(s.eoff.astype(np.int64)).cuda()
        qo = torch.from_numpy(s.qoff.astype(np.int64)).cuda()
        mx = int(max(np.diff(s.eoff).max(), np.diff(s.qoff).max()))

        def one_launch():
            g.reset()
            g.bulk_stream(E, eo, Q, qo, out, max_items=mx)
            g.labels(out=lab)

        # the one-launch form takes its own launch shape (its grid is sized
        # from the block and the largest minibatch)
        stream_opts = tuning.lookup("stream", "grid", s.n)
        g.reset()  # a fresh forest may change its linking order
        for k, v in stream_opts.items():
            g.set_option(k, v)
        out.zero_()
        wall_stream, c3 = timed(one_launch, args.steps, args.warmup, "stream-kernel")
        assert c1 == c3 and torch.equal(out, want), "stream kernel differs from plain launches"
        assert g.sync() == 0
        g.close()
    steps = max(1, args.steps)
    forms = {"plain": wall_plain, "hipgraph": wall_graph, "stream_kernel": wall_stream}
    best = min(forms, key=forms.get)
    res = result(steps * (M + Qn) / forms[best], args.steps, args.warmup, forms[best], {
        "workload": "grid4096-" + best, "n": s.n, "edges": M, "minibatches": nb, "minibatch": 1 << 12,
        "queries_per_minibatch": 1 << 10, "long_range_edges": s.meta["extra"], "form": best,
        "options": opts, "stream_kernel_options": stream_opts})
    res.update({"forms": {k: {"value": steps * (M + Qn) / v, "ms_per_step": v / steps * 1e3}
                          for k, v in forms.items()},
                "speedup_vs_plain": wall_plain / forms[best], "components": c3})
    if not args.no_cpu_baseline:
        res["cpu_baseline"] = cpu_baseline([s], args.cpu_budget)
    return res


def run_batched(args):
    import numpy as np
    import torch

    import synth
    import paper_1602_05232_amd as ccgpu
    from paper_1602_05232_amd import tuning

    t = time.perf_counter()
    ns = synth.multi_graph_sizes(G=args.graphs)
    streams = [synth.multi_graph_stream(g, int(ns[g])) for g in range(args.graphs)]
    M = sum(len(s.edges) for s in streams)
    Qn = sum(len(s.queries) for s in streams)
    log("generated %d graphs: sum n=%d edges=%d queries=%d in %.1fs"
        % (len(streams), int(ns.sum()), M, Qn, time.perf_counter() - t))
    # all inputs in two device buffers
    Eall = torch.from_numpy(np.concatenate([s.edges for s in streams])).cuda()
    Qall = torch.from_numpy(np.concatenate([s.queries for s in streams])).cuda()
    out = torch.empty(Qn, dtype=torch.uint8, device="cuda")
    ebase = np.cumsum([0] + [len(s.edges) for s in streams])
    qbase = np.cumsum([0] + [len(s.queries) for s in streams])
    G = len(streams)

    def eslice(g, k):
        s = streams[g]
        return Eall[int(ebase[g] + s.eoff[k]):int(ebase[g] + s.eoff[k + 1])]

    def qslice(g, k, buf):
        s = streams[g]
        return buf[int(qbase[g] + s.qoff[k]):int(qbase[g] + s.qoff[k + 1])]

    popts = tuning.lookup("pool", "mixed", int(np.median(ns))) or {}
    popts = {k: v for k, v in popts.items() if k not in ("update_mode", "compress_every")}
    if args.options:
        popts.update(parse_options(args.options))
    pool = ccgpu.Pool(int(ns.sum()), G, **popts)
    ids = [pool.add(s.n) for s in streams]
    ops_per_step = []
    for k in range(4):
        ops = [(ids[g], ccgpu.UPDATE, eslice(g, k), None) for g in range(G)]
        ops += [(ids[g], ccgpu.QUERY, qslice(g, k, Qall), qslice(g, k, out)) for g in range(G)]
        ops_per_step.append(ops)

    prepared = [pool.prepare(ops) for ops in ops_per_step]  # marshalled once, submitted every step

    def pool_step():
        pool.reset_all()
        for ops in prepared:
            pool.run(ops)
        return pool.sync()

    # The per-graph baseline runs with its own best options: a short trial of
    # each candidate set (one step each), then the fastest is timed.
    candidates = [dict(), dict(hook=2, compress_linked=0), dict(hook=1, compress_linked=0),
                  dict(hook=2, compress_linked=0, block=1024), dict(hook=2, compress_linked=0, filter=2)]
    graphs = [] if args.no_plain else [ccgpu.Graph(s.n) for s in streams]
    out_plain = torch.empty_like(out)

    def set_plain_options(o):
        for gr in graphs:
            gr.reset()  # the linking order may change only on a fresh forest
            for k, v in {**dict(hook=0, compress_linked=1, block=256, filter=0), **o}.items():
                gr.set_option(k, v)

    # views made once, as the pool's operation lists are marshalled once
    pe = [[eslice(g, k) for g in range(G)] for k in range(4)]
    pq = [[(qslice(g, k, Qall), qslice(g, k, out_plain)) for g in range(G)] for k in range(4)]

    def plain_step():
        for gr in graphs:
            gr.reset()
        for k in range(4):
            for g in range(G):
                graphs[g].bulk_update(pe[k][g])
            for g in range(G):
                graphs[g].bulk_query(pq[k][g][0], out=pq[k][g][1])
        torch.cuda.synchronize()

    def timed(fn, name):
        for _ in range(args.warmup):
            fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for k in range(args.steps):
            fn()
            log("%s step %d done" % (name, k))
        torch.cuda.synchronize()
        return time.perf_counter() - t0

    if args.no_plain:  # the pool forms only (for profiling runs)
        candidates = []
    trial = []
    for o in candidates:
        set_plain_options(o)
        plain_step()
        t0 = time.perf_counter()
        plain_step()
        trial.append((time.perf_counter() - t0, o))
        log("per-graph trial %s: %.1f ms" % (o, trial[-1][0] * 1e3))
    wall_pool = timed(pool_step, "pool")
    if args.no_plain:
        plain_opts, wall_plain = None, float("nan")
        out_plain.copy_(out)
    else:
        plain_opts = min(trial, key=lambda x: x[0])[1]
        set_plain_options(plain_opts)
        wall_plain = timed(plain_step, "per-graph")
        assert torch.equal(out, out_plain), "pool answers differ from per-graph answers"
    # the same run with all rounds of a step in one cooperative launch
    ops_all = pool.prepare([op for ops in ops_per_step for op in ops])
    pool.set_option("one_launch", 1)

    def pool_one_launch():
        pool.reset_all()
        pool.run(ops_all)
        return pool.sync()

    out.zero_()
    wall_one = timed(pool_one_launch, "pool-one-launch")
    assert torch.equal(out, out_plain), "one-launch pool answers differ from per-graph answers"
    pool.set_option("one_launch", 0)
    comps = sum(pool.num_components(i) for i in ids)
    assert args.no_plain or comps == sum(gr.num_components() for gr in graphs)
    for gr in graphs:
        gr.close()
    pool.close()
    steps = max(1, args.steps)
    res = result(steps * (M + Qn) / wall_pool, args.steps, args.warmup, wall_pool, {
        "workload": "batched%d-pool" % G, "graphs": G, "sum_n": int(ns.sum()), "median_n": int(np.median(ns)),
        "edges": M, "queries": Qn, "steps_per_graph": 4, "queries_per_step": 1 << 12,
        "n_distribution": "clip(round(2^X), 2^10, 2^20), X ~ N(14, 2)", "form": "pool", "options": popts})
    res.update({"plain_value": steps * (M + Qn) / wall_plain, "plain_ms_per_step": wall_plain / steps * 1e3,
                "plain_options": plain_opts,
                "plain_trials_ms": [{"options": o, "ms": t * 1e3} for t, o in trial],
                "speedup_vs_plain": wall_plain / wall_pool, "components": comps,
                "one_launch": {"value": steps * (M + Qn) / wall_one, "ms_per_step": wall_one / steps * 1e3,
                               "speedup_vs_plain": wall_plain / wall_one,
                               "what": "all 8 rounds of a step in one cooperative launch"}})
    if not args.no_cpu_baseline:
        res["cpu_baseline"] = cpu_baseline(streams, args.cpu_budget)
    return res


def run_serve(args):
    import numpy as np
    import torch

    import synth
    from paper_1602_05232_amd import serve, tuning

    S, scale, R = 64, args.serve_scale, args.requests
    n = 1 << scale
    seed = synth.BASE_SEED + 5
    t = time.perf_counter()
    reqs = []
    tot_e = tot_q = 0
    for r in synth.serving_trace(S=S, scale=scale, R=R, seed=seed):
        items = torch.from_numpy(r.items).cuda()
        if r.kind == 0:
            reqs.append(serve.Request(r.rid, r.stream, serve.UPDATE, 0.0, items, None, r.size))
            tot_e += r.size
        else:
            reqs.append(serve.Request(r.rid, r.stream, serve.QUERY, 0.0, items,
                                      torch.zeros(r.size, dtype=torch.uint8, device="cuda"), r.size))
            tot_q += r.size
    torch.cuda.synchronize()
    log("serving trace: %d requests over %d streams of n=2^%d, %d update edges, %d query pairs (%.1fs)"
        % (R, S, scale, tot_e, tot_q, time.perf_counter() - t))
    popts = tuning.lookup("serve", "rmat", n) or tuning.lookup("pool", "mixed", n) or {}
    popts = {k: v for k, v in popts.items() if k not in ("update_mode", "compress_every")}
    if args.options:
        popts.update(parse_options(args.options))
    popts["compress_linked"] = 0  # rounds overlap on two streams

    def with_arrivals(times):
        out = []
        for r, a in zip(reqs, times):
            o = None if r.out is None else torch.zeros_like(r.out)
            out.append(serve.Request(r.rid, r.stream, r.kind, float(a), r.items, o, r.size))
        return out

    def run(form, times, budget):
        ex = serve.GpuExecutor(budget, S + 1, **popts)
        sch = serve.serial_scheduler(ex, [n] * S) if form == "serial" else serve.Scheduler(ex, [n] * S, 2)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        done = sch.run(with_arrivals(times))
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        answers = {r.rid: r.out for r in done if r.kind == serve.QUERY}
        info = {"wall_s": wall, "items_per_s": (tot_e + tot_q) / wall, "rounds": sch.rounds,
                "mean_round_size": float(np.mean(sch.round_sizes)), "evictions": sch.evictions}
        info.update(serve.latency_summary(done))
        assert ex.pool.sync() == 0
        ex.close()
        log("%s: %s" % (form, info))
        return info, answers

    zeros = np.zeros(R)
    full = S * n
    reps = max(3, args.steps)

    def median_run(form, times, budget):
        """reps runs of one form; the run with the median wall time, plus
        the medians of its latency figures over the runs."""
        runs = [run(form, times, budget) for _ in range(reps)]
        runs.sort(key=lambda r: r[0]["wall_s"])
        info, answers = runs[len(runs) // 2]
        info = dict(info)
        for key in ("p50_ms", "p99_ms"):
            if key in info:
                info[key] = float(np.median([r[0][key] for r in runs]))
        info["runs"] = len(runs)
        info["wall_s_all"] = [r[0]["wall_s"] for r in runs]
        return info, answers

    for _ in range(args.warmup):
        run("served", zeros, full)
    sat_served, a1 = median_run("served", zeros, full)
    sat_serial, a2 = median_run("serial", zeros, full)
    for rid in a1:
        assert torch.equal(a1[rid], a2[rid]), "served and serial answers differ"
    # latency at 70% of the serial form's capacity (requests per second)
    lam = 0.7 * R / sat_serial["wall_s"]
    arr = synth.poisson_arrivals(synth.key(seed, 0, synth.P_ARRIVALS), R, lam)
    lat_served, _ = median_run("served", arr, full)
    lat_serial, _ = median_run("serial", arr, full)
    budget = (256 << 20) // 4  # 256 MiB of parent entries: a quarter of the graphs resident
    lat_evict, a3 = run("served", arr, budget)
    for rid in a1:
        assert torch.equal(a1[rid], a3[rid]), "answers changed under eviction"
    res = result((tot_e + tot_q) / sat_served["wall_s"], reps, args.warmup, sat_served["wall_s"] * reps, {
        "workload": "serve%d-rmat%d" % (S, scale), "streams": S, "n_per_stream": n, "requests": R,
        "update_fraction": 0.7, "request_sizes": "floor(2^U), U ~ U[8, 22]", "update_edges": tot_e,
        "query_pairs": tot_q, "form": "served (continuous batching, 2 HIP streams)", "options": popts})
    res.update({"saturation": {"served": sat_served, "serial": sat_serial,
                               "speedup": sat_serial["wall_s"] / sat_served["wall_s"]},
                "poisson_rate_per_s": lam,
                "latency_at_0.7_serial_capacity": {"served": lat_served, "serial": lat_serial},
                "latency_with_256MiB_budget": lat_evict})
    return res


def run_bigbatch(args):
    """Update-only throughput against minibatch size, fused vs contracting."""
    import numpy as np
    import torch

    import synth
    import paper_1602_05232_amd as ccgpu
    from paper_1602_05232_amd import tuning

    graphs = {
        "rmat24": lambda: synth.rmat_stream(scale=24, qbatch=1, probes=0),
        "er24": lambda: synth.er_stream(n=1 << 24, batches=1, batch=5 << 24, qbatch=1, probes=0),
    }
    schedules = {
        "fused-rank-filter": tuning.plain_options(1 << 24, "rmat"),
        "fused-rank": dict(update_mode=0, hook=2, block=1024, compress_linked=0),
        "fused-id": dict(update_mode=0, hook=0, block=1024, compress_linked=0),
        "fused-hash": dict(update_mode=0, hook=1, block=1024, compress_linked=0),
        "contract-id": dict(update_mode=2, hook=0),
        "contract-hash": dict(update_mode=2, hook=1),
    }
    table, best_rate, best_cfg = {}, 0.0, None
    total_t, total_e = 0.0, 0
    for gname, make in graphs.items():
        s = make()
        M = len(s.edges)
        E = torch.from_numpy(s.edges).cuda()
        for k in (1, 8, 64):
            bounds = [M * i // k for i in range(k + 1)]
            comps = None
            for sname, opts in schedules.items():
                g = ccgpu.Graph(s.n, **opts)
                g.reserve(max(bounds[i + 1] - bounds[i] for i in range(k)))
                times = []
                for it in range(args.warmup + max(1, args.steps)):
                    g.reset()
                    torch.cuda.synchronize()
                    t0 = time.perf_counter()
                    for i in range(k):
                        g.bulk_update(E[bounds[i]:bounds[i + 1]])
                    c = g.num_components()
                    dt = time.perf_counter() - t0
                    if it >= args.warmup:
                        times.append(dt)
                if g.sync() != 0:
                    raise SystemExit("device reported an error (%s, %s, k=%d)" % (gname, sname, k))
                g.close()
                assert comps is None or c == comps, "component counts differ between schedules"
                comps = c
                t = min(times)
                total_t += sum(times)
                total_e += M * len(times)
                rate = M / t
                table.setdefault(gname, {}).setdefault("minibatches=%d" % k, {})[sname] = {
                    "edges_per_s": rate, "ms": t * 1e3}
                log("%s k=%d %s: %.3f ms, %.3g edges/s, components=%d" % (gname, k, sname, t * 1e3, rate, c))
                if gname == "rmat24" and k == 1 and rate > best_rate:
                    best_rate, best_cfg = rate, sname
        del E
        torch.cuda.empty_cache()
    res = result(total_e / total_t, max(1, args.steps), args.warmup, total_t, {
        "workload": "bigbatch", "graphs": {"rmat24": "R-MAT scale 24, 2^28 edges",
                                           "er24": "n = 2^24, 5n uniform edges"},
        "minibatches": [1, 8, 64], "schedules": schedules})
    res["unit"] = "edges/s (update only)"
    res["table"] = table
    res["best_rmat24_one_minibatch"] = best_cfg
    return res


def run_components(args):
    """Number of components against the fraction of the stream consumed, for
    each workload shape at n = 2^k (k = --components-log2n, default 24; the
    measurement behind Fig. 2, whose streams have about 10^8 vertices)."""
    import numpy as np
    import torch

    import synth
    import paper_1602_05232_amd as ccgpu
    from paper_1602_05232_amd import tuning

    k = args.components_log2n
    if k % 3 or not 12 <= k <= 27:
        raise SystemExit("--components-log2n must be a multiple of 3 in [12, 27] (the 3-D mesh is 2^(k/3) a side)")
    n, L = 1 << k, 1 << (k // 3)
    shapes = {
        "random (ER, 5 edges/vertex)": lambda: synth.er_stream(n=n, batches=80, batch=(5 * n) // 80,
                                                               qbatch=1, probes=0),
        "rmat (scale %d, EF 16)" % k: lambda: synth.rmat_stream(scale=k, qbatch=1, probes=0),
        "grid3d (%d^3)" % L: lambda: synth.grid3d_stream_cfg(L=L, batch=1 << 21, qbatch=1, probes=0),
        "local5 (window 2^12)": lambda: synth.local_stream(n=n, degree=5, window=1 << 12, batch=1 << 21,
                                                           qbatch=1, probes=0),
        "local16 (window 2^12)": lambda: synth.local_stream(n=n, degree=16, window=1 << 12,
                                                            batch=1 << 22, qbatch=1, probes=0),
    }
    traces, total_t, total_e = {}, 0.0, 0
    for name, make in shapes.items():
        log("generating %s" % name)
        s = make()
        E = torch.from_numpy(s.edges).cuda()
        g = ccgpu.Graph(s.n, **tuning.plain_options(s.n, "rmat"))
        g.reserve(int(np.diff(s.eoff).max()))
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        pts = [(0.0, s.n)]
        for i in range(s.num_batches):
            g.bulk_update(E[int(s.eoff[i]):int(s.eoff[i + 1])])
            pts.append((float(s.eoff[i + 1]) / len(s.edges), g.num_components()))
        total_t += time.perf_counter() - t0
        total_e += len(s.edges)
        assert g.sync() == 0
        traces[name] = pts
        log("%s: %d edges, components at end %d" % (name, len(s.edges), pts[-1][1]))
        g.close()
        del E, s
        torch.cuda.empty_cache()
    res = result(total_e / total_t, 1, 0, total_t, {"workload": "component-trace", "n": n,
                                                      "shapes": list(shapes)})
    res["unit"] = "edges/s (one count read per minibatch)"
    res["traces"] = traces
    return res


def run_deep(args):
    """One Bulk-Query of 2^20 uniform pairs on an uncompressed forest of long
    paths (n = 2^24, paths of L random vertices, L = 16, 256, 4096), loaded
    as a state image before each timed call: independent finds with and
    without path halving against Bulk-Find (Section 5) with Phase II by
    pointer jumping and by the response distributor.  Many endpoints share
    each path, the case Bulk-Find's work bound is about.  Every answer is
    checked against the paths' membership."""
    import numpy as np
    import torch

    import synth
    import paper_1602_05232_amd as ccgpu
    from paper_1602_05232_amd import roofline

    n, q = 1 << 24, 1 << 20
    pairs_h = synth.uniform_pairs(synth.key(synth.BASE_SEED + 9, 0, synth.P_QUERIES), 0, q, n)
    pairs = torch.from_numpy(pairs_h).cuda()
    out = torch.empty(q, dtype=torch.uint8, device="cuda")
    stream = torch.cuda.current_stream()
    e0, e1 = roofline.TimingEvent(), roofline.TimingEvent()
    forms = [("independent, halving", dict(find=0, query_halving=1)),
             ("independent, no halving", dict(find=0, query_halving=0)),
             ("bulk-find, pointer jumping", dict(find=1)),
             ("bulk-find, response distributor", dict(find=2))]
    reps = max(3, args.steps)
    table = {}
    for L in (16, 256, 4096):
        parent, path = synth.chain_forest(n, L)
        want = torch.from_numpy((path[pairs_h[:, 0]] == path[pairs_h[:, 1]]).astype(np.uint8))
        img = np.array([n, n - n // L], np.int64).tobytes() + parent.tobytes()
        del parent, path
        row = {}
        for name, o in forms:
            g = ccgpu.Graph(n, hook=0, filter=0, compress_linked=0, **o)
            ts = []
            for _ in range(args.warmup + reps):
                g.load(img)
                e0.record(stream)
                g.bulk_query(pairs, out=out)
                e1.record(stream)
                torch.cuda.synchronize()
                ts.append(e0.elapsed_time(e1))
                if not torch.equal(out.cpu(), want):
                    raise SystemExit("deepforest: wrong answers (L=%d, %s)" % (L, name))
            if g.sync() != 0:
                raise SystemExit("device reported an error (L=%d, %s)" % (L, name))
            g.close()
            ms = sorted(ts[args.warmup:])[reps // 2]
            row[name] = {"ms": ms, "pairs_per_s": q / (ms * 1e-3)}
            log("L=%d %s: %.3f ms" % (L, name, ms))
        table["L%d" % L] = row
    e0.close()
    e1.close()
    best = table["L4096"]["bulk-find, pointer jumping"]
    res = result(best["pairs_per_s"], reps, args.warmup, 0.0, {
        "workload": "deepforest-2^24", "n": n, "queries": q, "path_lengths": [16, 256, 4096],
        "forest": "n / L paths of L random vertices, parent id below child id, loaded as a state image",
        "form": "one Bulk-Query per loaded forest", "options": {"hook": 0, "filter": 0}})
    res.update({"ms_per_step": best["ms"], "by_path_length": table,
                "value_is": "Bulk-Find (pointer jumping) at L = 4096"})
    return res


def compact(r: dict, keys) -> dict:
    out = {"value": r["value"], "unit": r["unit"], "ms_per_step": r["ms_per_step"]}
    for k in keys:
        if k in r:
            out[k] = r[k]
    return out


def run_forms(args) -> dict:
    """Every workload's forms against its plain form, each on its own
    configuration (a few steps each, medians where a form is short)."""
    import copy
    import torch

    sub = copy.copy(args)
    sub.steps, sub.warmup, sub.no_cpu_baseline, sub.options = max(3, min(args.steps, 5)), 1, True, ""
    forms = {}
    r = run_er(sub)
    forms["er16"] = compact(r, ("median_ms_per_pass", "forms", "components", "config", "stream_kernel_options"))
    log("forms: er16 %s" % {k: "%.3f ms" % v["median_ms_per_pass"] for k, v in r["forms"].items()})
    torch.cuda.empty_cache()
    r = run_grid(sub)
    forms["grid4096"] = compact(r, ("forms", "speedup_vs_plain", "components", "config"))
    log("forms: grid4096 %s" % {k: "%.1f ms" % v["ms_per_step"] for k, v in r["forms"].items()})
    torch.cuda.empty_cache()
    r = run_batched(sub)
    forms["batched1024"] = compact(r, ("plain_value", "plain_ms_per_step", "plain_options", "speedup_vs_plain",
                                       "one_launch", "components", "config"))
    log("forms: batched1024 pool %.1f ms, per-graph %.1f ms" % (r["ms_per_step"], r["plain_ms_per_step"]))
    torch.cuda.empty_cache()
    r = run_serve(sub)
    forms["serve64"] = compact(r, ("saturation", "poisson_rate_per_s", "latency_at_0.7_serial_capacity",
                                   "latency_with_256MiB_budget", "config"))
    log("forms: serve64 served/serial saturation speedup %.2f" % r["saturation"]["speedup"])
    torch.cuda.empty_cache()
    return forms


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="rmat24",
                    choices=["rmat24", "er16", "grid4096", "batched1024", "serve64", "bigbatch", "components",
                             "deepforest"])
    ap.add_argument("--requests", type=int, default=1024, help="requests of the serving trace")
    ap.add_argument("--serve-scale", type=int, default=22, help="R-MAT scale of each served graph")
    ap.add_argument("--scale", type=int, default=24, help="R-MAT scale of the rmat24 workload")
    ap.add_argument("--graphs", type=int, default=1024, help="graphs of the batched workload")
    ap.add_argument("--components-log2n", type=int, default=24, help="log2 of n for the components workload")
    ap.add_argument("--options", default="", help="option overrides: JSON object or key=value,key=value")
    ap.add_argument("--cpu-budget", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-roofline", action="store_true")
    ap.add_argument("--no-plain", action="store_true",
                    help="batched1024 only: skip the per-graph form (profiling runs of the pool)")
    ap.add_argument("--no-forms", action="store_true",
                    help="rmat24 only: skip the other workloads' forms (plain vs batched vs served)")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py: the benchmark runs on one GPU only; --gpus %d (WORLD_SIZE=%d) is not supported"
              % (args.gpus, world), file=sys.stderr)
        sys.exit(2)

    from paper_1602_05232_amd import build as hipbuild
    if not os.path.exists(hipbuild.OUT):
        import __graft_entry__
        __graft_entry__.build()
    res = {"rmat24": run_rmat, "er16": run_er, "grid4096": run_grid, "batched1024": run_batched,
           "serve64": run_serve, "bigbatch": run_bigbatch, "components": run_components,
           "deepforest": run_deep}[args.workload](args)
    if args.workload == "rmat24" and not args.no_forms:
        res["forms"] = run_forms(args)
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
