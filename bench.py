#!/usr/bin/env python3
"""Benchmark of the Motifs-k hot path on one MI355X.

    python bench.py [--steps K] [--warmup W] [--gpus 1] [--serve R]

One step = one full pass of the path over one batch of synthetic graphs,
inputs (CSR graphs) and class table already resident in HBM: typed
adjacency, work-unit plan, persistent enumeration with code formation,
table lookup and histograms -- one replay of the batch's captured hipGraph.

Workload: k = 6, one directed graph with n = 700, m = 1500 (power-law
out-degrees up to 60, Poisson in-degrees) plus 30 degree-preserving
randomisations, counted in one launch (31 histograms of 1,530,843 classes).

Printed: one JSON line with subgraphs/s; the roofline of the counting
kernel (its busier issue pipe from the committed counter record over the
kernel's live HIP-event duration, with the HBM, L2 and lane figures beside
it); the CPU oracle on the host cores with every histogram compared; the
plain one-graph-per-launch form on the same graphs; the k = 5 batch (1 + 100
randomisations of n = 1000, m = 3000) as a second reading; the serving
stream (1,000 Poisson requests, served and plain first-come-first-served
under the same arrivals: throughput, p50 / p99); then both counting methods,
the code-formation variants with a k = 6 graph of 2^20 vertices, k = 7, and
the ensemble pipeline.
"""

from __future__ import annotations

import argparse
import json
import os
import sys
import time

HBM_PEAK_GBS = 8000.0
BYTES_PER_SUBGRAPH = 4 + 8 + 8   # k = 6 model: table entry, counter read + write
ROOT = os.path.dirname(os.path.abspath(__file__))
COUNTERS_FILE = os.path.join(ROOT, "profiles", "counting_kernel_counters.json")
DIGESTS_FILE = os.path.join(ROOT, "tests", "golden", "oracle_digests.json")


def _counter_record(kernel):
    """The committed counter record of `kernel` (per-launch means of the
    rocprofv3 --pmc passes, FETCH_SIZE / WRITE_SIZE scaled to bytes), or None
    when the kernel sources changed since it was taken."""
    from paper_1804_09741_amd import profsum as P
    try:
        with open(COUNTERS_FILE) as f:
            rec = json.load(f)
        if rec["source_sha256_16"] != P.source_hash():
            return None
        return rec["kernels"][kernel]
    except (OSError, KeyError, ValueError):
        return None


def _roofline(kernel, kernel_ms, subgraphs=None):
    """Roofline of one counting-kernel launch: the busier issue pipe (VALU
    or SALU wave-instructions per launch from the counter record, over the
    live kernel duration) against 256 CUs x 2.4 GHz x 1, with lane use,
    waits, L2 hit rate, L2 atomics and counter-measured HBM traffic beside
    it, and for k = 6 the 20-byte-per-subgraph HBM model."""
    from paper_1804_09741_amd import profsum as P
    rec = _counter_record(kernel)
    if rec is None:
        r = {"bound": "alu", "achieved": None, "peak": P.ISSUE_PEAK,
             "unit": "wave-instructions/s", "frac": None, "traffic": None,
             "counters": "stale: kernel sources changed since the counter record"}
    else:
        d = P.derived(rec["counters"], kernel_ms / 1e3)
        r = P.issue_roofline(d)
        r["traffic"] = rec["traffic_bytes"]
        for key in ("valu", "salu", "lds"):
            if key in d:
                r[key] = {"insts_per_launch": d[key]["insts_per_launch"], "frac": d[key]["frac"]}
        for key in ("lane_util", "wait_frac", "lds_conflict_frac", "l2_hit",
                    "l2_atomics_per_launch", "l2_atomic_rate", "l2_atomic_frac"):
            if key in d:
                r[key] = d[key]
        r["hbm_measured"] = {"achieved": d["hbm_rate"] / 1e9, "peak": HBM_PEAK_GBS,
                             "unit": "GB/s", "frac": d["hbm_frac"]}
        r["counters"] = "profiles/counting_kernel_counters.json (%d dispatches, %s)" % (
            rec["dispatches"], rec["workload"])
        r["counters_kernel_ms"] = rec["kernel_ms"]
    r["kernel"] = kernel
    r["kernel_ms"] = kernel_ms
    r["peak_derivation"] = ("256 CUs x 2.4 GHz x 1 wave64 instruction per CU-cycle per pipe "
                            "(4 SIMD16 per CU, 4 cycles per wave64 VALU op; 1 scalar unit)")
    if subgraphs is not None:
        a = BYTES_PER_SUBGRAPH * subgraphs / (kernel_ms / 1e3) / 1e9
        r["hbm_model"] = {"bytes_per_subgraph": BYTES_PER_SUBGRAPH, "achieved": a,
                          "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": a / HBM_PEAK_GBS}
    return r


def _kernel_name(k, stats):
    """The counting kernel a batch ran (its stats name the method)."""
    return ("core_kernel<%d>" if stats.get("method") == 2 else "enum_kernel<%d>") % k


def _log(msg):
    print("[bench] " + msg, file=sys.stderr, flush=True)


def _cpu_share():
    """Worker processes for the oracle: the cores this process may run on,
    at most 16 (one GPU's share of its host)."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(16, n))


def _parse():
    p = argparse.ArgumentParser(description=__doc__.split("\n")[1])
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=10)
    p.add_argument("--warmup", type=int, default=2)
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--no-k5", action="store_true", help="skip the k=5 batch reading")
    p.add_argument("--no-plain", action="store_true", help="skip the plain comparator")
    p.add_argument("--cpu-graphs", type=int, default=10,
                   help="graphs of the k=6 batch the single-thread oracle counts")
    p.add_argument("--split", type=int, default=0,
                   help="k=6 split threshold (0: library default)")
    p.add_argument("--k5-split", type=int, default=0,
                   help="k=5 split threshold (0: library default)")
    p.add_argument("--waves-per-cu", type=int, default=0)
    p.add_argument("--method", choices=("auto", "esu", "cores"), default="auto",
                   help="counting method of the batches (auto: the library's choice)")
    p.add_argument("--autotune", action="store_true",
                   help="pick the k=6 batch options with the library's autotuner first")
    p.add_argument("--copy-mib", type=int, default=0,
                   help="also run one device-to-device copy of this many MiB (a kernel of "
                        "known traffic, to scale hardware byte counters)")
    p.add_argument("--no-methods", action="store_true",
                   help="skip timing both counting methods on the k=6 and k=5 batches")
    p.add_argument("--no-variants", action="store_true",
                   help="skip the code-formation variants and the 2^20-vertex graph")
    p.add_argument("--no-k7", action="store_true", help="skip the k=7 reading")
    p.add_argument("--no-ensemble", action="store_true",
                   help="skip the ensemble pipeline (random graphs, counts, z-scores)")
    p.add_argument("--serve", type=int, default=1000, metavar="R",
                   help="requests of the serving stream (0: skip)")
    p.add_argument("--serve-load", type=float, default=0.7,
                   help="open-loop arrival rate as a fraction of the measured capacity")
    return p.parse_args()


def _timed_batch(ctx, M, graphs, table, steps, warmup, torch, **opts):
    """Run `steps` timed passes of one prepared batch; returns a dict."""
    b = ctx.batch(graphs, table, **opts)
    try:
        d_hist = torch.zeros((len(graphs), table.num_classes), dtype=torch.int64, device="cuda:0")
        stream = torch.cuda.current_stream()
        for _ in range(warmup):
            b.run(d_hist, stream)
        torch.cuda.synchronize()
        enum_ms = []
        pass_ms = []
        t0 = time.perf_counter()
        for _ in range(steps):
            b.run(d_hist, stream)
            p_ms, e_ms = b.timing()          # HIP events on the launch stream
            pass_ms.append(p_ms)
            enum_ms.append(e_ms)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        hist, totals = b.read()
        return {"wall_s": t1 - t0, "enum_ms": enum_ms, "pass_ms": pass_ms,
                "hist": hist, "totals": totals, "stats": b.stats()}
    finally:
        b.free()


def _oracle_hist(args):
    """Worker of the CPU legs: the oracle's histogram of one graph as
    ascending (canonical code, count) pairs, and its seconds."""
    rp, col, k = args
    from oracle import oracle as O
    t0 = time.perf_counter()
    h = O.count(rp, col, k)
    return sorted(h.items()), time.perf_counter() - t0


def _oracle_ready(_):
    """Worker warm-up: load the oracle library and its k <= 5 tables."""
    import numpy as np
    from oracle import oracle as O
    O.count(np.zeros(4, np.int32), np.zeros(0, np.int32), 3)
    O.canon_table(5)
    return os.getpid()


def _cpu_legs(I, procs, single_graphs):
    """The oracle on the host, before this process touches the GPU (the
    worker processes start from a process without device state):
      * all 31 graphs of the k = 6 batch, one graph per task on `procs`
        processes -- the reported cpu_baseline;
      * `procs` graphs of the k = 5 batch, one per process;
      * graphs 0..single_graphs-1 of the k = 6 batch on one thread.
    Every histogram is kept for the comparison with the GPU's."""
    import multiprocessing
    from concurrent.futures import ProcessPoolExecutor

    from oracle import oracle as O
    w6 = I.workload_k6_batch()
    w5 = I.workload_k5_batch()
    out = {}
    with ProcessPoolExecutor(max_workers=procs,
                             mp_context=multiprocessing.get_context("spawn")) as pool:
        list(pool.map(_oracle_ready, range(procs)))
        for name, w, idx in (("k6", w6, range(len(w6.graphs))),
                             ("k5", w5, range(min(procs, len(w5.graphs))))):
            t0 = time.perf_counter()
            res = list(pool.map(_oracle_hist, [(*w.graphs[i], w.k) for i in idx]))
            wall = time.perf_counter() - t0
            out[name] = {"workload": w.name, "graphs": list(idx), "wall_s": wall,
                         "hists": [dict(h) for h, _ in res],
                         "cpu_s": sum(t for _, t in res)}
            _log("cpu oracle %s: %d graphs on %d processes in %.1f s" % (
                name, len(idx), procs, wall))
    t0 = time.perf_counter()
    single = [O.count(*w6.graphs[i], 6) for i in range(min(single_graphs, len(w6.graphs)))]
    out["single"] = {"wall_s": time.perf_counter() - t0, "hists": single}
    _log("cpu oracle single thread: %d graphs in %.1f s" % (len(single), out["single"]["wall_s"]))
    return out


def _cpu_report(leg, gpu_hist, class_codes, procs, what):
    """One CPU leg as a report object, its histograms compared with the
    GPU's graph by graph."""
    import numpy as np
    counted = sum(sum(h.values()) for h in leg["hists"])
    match = 0
    for i, h in zip(leg["graphs"], leg["hists"]):
        nz = np.flatnonzero(gpu_hist[i])
        match += int(h == {int(class_codes[j]): int(gpu_hist[i][j]) for j in nz})
    return {"value": counted / leg["wall_s"], "unit": "subgraphs/s", "cores": procs,
            "kind": "oracle",
            "sample": "%s: %d graphs (%d subgraphs), one graph per task on %d processes, "
                      "%.1f s wall, %.0f CPU-s" % (what, len(leg["graphs"]), counted, procs,
                                                    leg["wall_s"], leg["cpu_s"]),
            "host_cpu_count": os.cpu_count(), "hists_match_gpu": match == len(leg["graphs"]),
            "graphs_matching": match}


def _digest_check(name, hist, class_codes, graphs):
    """GPU histograms of every graph against the stored oracle digests
    (tests/golden/oracle_digests.json, written from the oracle alone)."""
    from oracle.digest import dense_digest, graph_digest
    try:
        with open(DIGESTS_FILE) as f:
            recs = json.load(f)[name]
    except (OSError, KeyError, ValueError):
        return None
    ok_in = all(r["graph"] == graph_digest(*g) for r, g in zip(recs, graphs))
    match = sum(int(dense_digest(hist[i], class_codes) == recs[i]["hist"])
                for i in range(len(recs)))
    return {"graphs": len(recs), "inputs_match": ok_in, "graphs_matching": match,
            "all_match": ok_in and match == len(recs) == len(graphs)}


def _plain(ctx, graphs, table, steps, torch, **opts):
    """One prepared single-graph batch per graph, run one after another."""
    bs = [ctx.batch([g], table, **opts) for g in graphs]
    try:
        d = torch.zeros((1, table.num_classes), dtype=torch.int64, device="cuda:0")
        stream = torch.cuda.current_stream()
        for b in bs:
            b.run(d, stream)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            for b in bs:
                b.run(d, stream)
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / steps
    finally:
        for b in bs:
            b.free()


def _methods(ctx, M, I, torch):
    """Both counting methods on the k=6 and k=5 batches: mean pass and
    counting-kernel ms over a few steps, and whether the histograms agree."""
    import numpy as np
    res = {}
    for k, w, steps in ((6, I.workload_k6_batch(), 4), (5, I.workload_k5_batch(), 2)):
        t = ctx.table(k)
        gs = [ctx.load_graph(*g) for g in w.graphs]
        hists = {}
        row = {}
        for name, meth in (("esu", M.METHOD_ESU), ("cores", M.METHOD_CORES)):
            r = _timed_batch(ctx, M, gs, t, steps, 1, torch, method=meth)
            hists[name] = r["hist"]
            row[name] = {"pass_ms": float(np.mean(r["pass_ms"])),
                         "kernel_ms": float(np.mean(r["enum_ms"]))}
        row["equal"] = bool(np.array_equal(hists["esu"], hists["cores"]))
        _log("methods k=%d: esu %.3f ms, cores %.3f ms (kernel), equal=%s" % (
            k, row["esu"]["kernel_ms"], row["cores"]["kernel_ms"], row["equal"]))
        res["k%d" % k] = row
        for g in gs:
            g.free()
    return res


def _variants(ctx, M, I, torch):
    """Code-formation variants of the enumeration: the k=6 and k=5 batches
    with arc tests on bit matrices or on sorted lists and marks in LDS or in
    device memory (kernel and pass ms, histograms equal to the first), then
    one k=6 graph of 2^20 vertices, past the LDS marks limit (the library
    picks lists and device-memory marks by itself)."""
    import numpy as np
    res = {}
    combos = (("bits_lds", M.ADJ_BITS, M.MARKS_LDS), ("lists_lds", M.ADJ_LISTS, M.MARKS_LDS),
              ("lists_global", M.ADJ_LISTS, M.MARKS_GLOBAL))
    for k, w, steps in ((6, I.workload_k6_batch(), 4), (5, I.workload_k5_batch(), 2)):
        t = ctx.table(k)
        gs = [ctx.load_graph(*g) for g in w.graphs]
        row, ref = {}, None
        for name, adj, marks in combos:
            r = _timed_batch(ctx, M, gs, t, steps, 1, torch, method=M.METHOD_ESU, adjacency=adj,
                             marks=marks)
            if ref is None:
                ref = r["hist"]
            row[name] = {"pass_ms": float(np.mean(r["pass_ms"])),
                         "kernel_ms": float(np.mean(r["enum_ms"])),
                         "equal": bool(np.array_equal(ref, r["hist"]))}
        _log("variants k=%d: %s" % (k, ", ".join("%s %.3f ms" % (n, row[n]["kernel_ms"])
                                                  for n, _, _ in combos)))
        res["k%d" % k] = row
        for g in gs:
            g.free()
    w = I.workload_k6_large()
    t = ctx.table(6)
    g = ctx.load_graph(*w.graphs[0])
    try:
        r = _timed_batch(ctx, M, [g], t, 2, 1, torch)
    finally:
        g.free()
    sub = int(r["totals"][0])
    kern = float(np.mean(r["enum_ms"]))
    st = r["stats"]
    res["large"] = {"workload": w.name, "subgraphs": sub, "kernel_ms": kern,
                    "pass_ms": float(np.mean(r["pass_ms"])),
                    "value": sub / (float(np.mean(r["pass_ms"])) / 1e3),
                    "unit": "subgraphs/s", "adjacency": st["adjacency"], "marks": st["marks"],
                    "grid": st["grid"], "units": st["units"],
                    "hbm_model": {"kernel": "enum_lists_kernel<6, 3>",
                                  "bytes_per_subgraph": BYTES_PER_SUBGRAPH,
                                  "achieved": BYTES_PER_SUBGRAPH * sub / (kern / 1e3) / 1e9,
                                  "peak": HBM_PEAK_GBS, "unit": "GB/s",
                                  "frac": BYTES_PER_SUBGRAPH * sub / (kern / 1e3) / 1e9
                                  / HBM_PEAK_GBS}}
    _log("variants: %s, %d subgraphs, pass %.1f ms (kernel %.1f ms), %.3g subgraphs/s" % (
        w.name, sub, res["large"]["pass_ms"], kern, res["large"]["value"]))
    return res


def _k7(ctx, M, I, torch):
    """k = 7 on the 31 graphs of the k = 6 batch (classes by canonical code,
    canonicalised on the device).  A first call sizes the class tables and
    fills the canonical-code cache (its wall time: first_call_ms); the cache
    is then cleared and the timed call starts cold -- every distinct labeled
    code canonicalised again -- which gives `value`; a third call on the
    warm cache is reported beside it."""
    import numpy as np
    w = I.workload_k6_batch()
    gs = [ctx.load_graph(*g) for g in w.graphs]
    try:
        t0 = time.perf_counter()
        ctx.count7(gs)
        first = time.perf_counter() - t0
        ctx.k7_cache_clear()
        t0 = time.perf_counter()
        out, totals, kern = ctx.count7(gs)
        wall = time.perf_counter() - t0
        slots, used = ctx.k7_cache_info()
        t0 = time.perf_counter()
        _, _, kern_warm = ctx.count7(gs)
        wall_warm = time.perf_counter() - t0
    finally:
        for g in gs:
            g.free()
    sub = int(np.sum(totals))
    classes = [len(c) for c, _ in out]
    res = {"workload": w.name.replace("k6_", "k7_"), "subgraphs": sub, "kernel_ms": kern,
           "call_ms": wall * 1e3, "value": sub / (kern / 1e3), "unit": "subgraphs/s (kernel)",
           "cache": "cold (cleared before the call)", "call_value": sub / wall,
           "cache_slots": slots, "cache_used_after": used,
           "warm": {"kernel_ms": kern_warm, "call_ms": wall_warm * 1e3,
                    "value": sub / (kern_warm / 1e3)},
           "first_call_ms": first * 1e3,
           "classes_mean": float(np.mean(classes)), "classes_max": int(max(classes))}
    _log("k=7 on the k=6 batch: %d subgraphs, cold kernel %.1f ms (%.3g/s), call %.1f ms; warm "
         "kernel %.1f ms; first call %.1f ms; cache %d of %d slots" % (
             sub, kern, res["value"], res["call_ms"], kern_warm, res["first_call_ms"], used,
             slots))
    # one graph past the LDS limit (marks and tags in device memory)
    wl = I.workload_k6_large(1 << 17)
    g = ctx.load_graph(*wl.graphs[0])
    try:
        ctx.count7([g])
        ctx.k7_cache_clear()
        t0 = time.perf_counter()
        out, totals, kern = ctx.count7([g])
        wall = time.perf_counter() - t0
    finally:
        g.free()
    sub = int(totals[0])
    res["large"] = {"workload": wl.name.replace("k6_", "k7_"), "subgraphs": sub, "kernel_ms": kern,
                    "call_ms": wall * 1e3, "value": sub / (kern / 1e3),
                    "unit": "subgraphs/s (kernel)", "cache": "cold",
                    "classes": len(out[0][0])}
    _log("k=7 on %s: %d subgraphs, cold kernel %.1f ms (%.3g/s), %d classes" % (
        res["large"]["workload"], sub, kern, res["large"]["value"], res["large"]["classes"]))
    return res


def _ensemble(ctx, M, I, torch, cpu=True, R=100, spa=10, seed=2024):
    """The whole significance pipeline on the device for the k=5 original:
    R degree-preserving random graphs (spa * m accepted switches each),
    H_5 of all R + 1 graphs in one batch, z-scores of every class."""
    import numpy as np
    rp, col = I.k5_batch_graph(0)
    g = ctx.load_graph(rp, col)
    t = ctx.table(5)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    made, acc = ctx.randomise(g, R, seed, spa)
    t1 = time.perf_counter()
    b = ctx.batch([g] + made, t)
    d_hist = torch.zeros((R + 1, t.num_classes), dtype=torch.int64, device="cuda:0")
    d_out = torch.zeros((3, t.num_classes), dtype=torch.float64, device="cuda:0")
    stream = torch.cuda.current_stream()
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    b.run(d_hist, stream)
    ctx.significance(d_hist, t.num_classes, d_out, stream)
    torch.cuda.synchronize()
    t3 = time.perf_counter()
    z = d_out[2].cpu().numpy()
    subgraphs = int(d_hist.sum().item())
    res = {"random_graphs": R, "switches_per_arc": spa, "accepted_min": int(acc.min()),
           "randomise_ms": 1000 * (t1 - t0), "count_and_z_ms": 1000 * (t3 - t2),
           "subgraphs": subgraphs, "classes_z_above_2": int(np.sum(np.isfinite(z) & (z > 2)))}
    if cpu:
        from oracle import oracle as O
        c0 = time.perf_counter()
        O.switch_chain(rp, col, seed, 0, spa * len(col), 8 * spa * len(col) + 1024)
        res["cpu_oracle_randomise_ms_per_graph"] = 1000 * (time.perf_counter() - c0)
    _log("ensemble: %d random graphs in %.1f ms, counts + z-scores %.1f ms" % (
        R, res["randomise_ms"], res["count_and_z_ms"]))
    b.free()
    for h in made + [g]:
        h.free()
    return res


def _serving(ctx, M, I, R, load, torch):
    """Serving workload: R (graph, k) requests of the stream (k uniform in
    3..6, n in [100, 5000]), graphs resident on the device.

    1. plain, closed loop: one mk_count per request, first come first
       served -> plain throughput;
    2. served, closed loop: all requests submitted at once -> capacity;
    3. served, open loop: Poisson arrivals at `load` x capacity -> p50 / p99
       of (completion - arrival) as timed by the server;
    4. plain, open loop: the same arrivals, one mk_count per request in
       arrival order on one thread -> p50 / p99 of (completion - arrival).
    Every served histogram must equal the plain one; those of the requests
    in the stored oracle digests are compared with the oracle too.
    """
    import threading

    import numpy as np

    from oracle.digest import dense_digest

    t0 = time.perf_counter()
    reqs = I.serving_requests(count=R)
    _log("serving: %d requests generated in %.1f s" % (R, time.perf_counter() - t0))
    tables = {k: ctx.table(k) for k in (3, 4, 5, 6)}
    codes = {k: tables[k].class_codes() for k in tables}
    graphs = [ctx.load_graph(*r.graph) for r in reqs]
    try:
        t0 = time.perf_counter()
        plain = [ctx.count(g, tables[r.k])[0] for g, r in zip(graphs, reqs)]
        plain_s = time.perf_counter() - t0
        total = int(sum(int(h.sum()) for h in plain))
        _log("serving: plain FIFO closed loop %.2f s, %d subgraphs" % (plain_s, total))

        srv = ctx.server()
        try:
            t0 = time.perf_counter()
            tickets = [srv.submit(g, r.k) for g, r in zip(graphs, reqs)]
            burst = [srv.wait(t, r.k) for t, r in zip(tickets, reqs)]
            burst_s = time.perf_counter() - t0
            same = all(np.array_equal(h, p) for (h, _), p in zip(burst, plain))
            _log("serving: served closed loop %.2f s" % burst_s)
            rate = load * R / burst_s
            gaps = np.random.default_rng(55).exponential(1.0 / rate, size=R)
            arrivals = np.cumsum(gaps) - gaps[0]
            tickets = [None] * R

            def submitter():
                start = time.perf_counter()
                for i in range(R):
                    delay = arrivals[i] - (time.perf_counter() - start)
                    if delay > 0:
                        time.sleep(delay)
                    tickets[i] = srv.submit(graphs[i], reqs[i].k)

            th = threading.Thread(target=submitter)
            t0 = time.perf_counter()
            th.start()
            lat = []
            for i in range(R):
                while tickets[i] is None:
                    time.sleep(0.0005)
                h, tm = srv.wait(tickets[i], reqs[i].k)
                same &= bool(np.array_equal(h, plain[i]))
                lat.append((tm["done_us"] - tm["submit_us"]) / 1000.0)
            th.join()
            open_s = time.perf_counter() - t0
        finally:
            srv.stop()
        _log("serving: served open loop %.2f s, p50 %.1f ms, p99 %.1f ms" % (
            open_s, np.percentile(lat, 50), np.percentile(lat, 99)))

        # plain FIFO under the same arrivals
        flat = []
        start = time.perf_counter()
        for i in range(R):
            delay = arrivals[i] - (time.perf_counter() - start)
            if delay > 0:
                time.sleep(delay)
            h = ctx.count(graphs[i], tables[reqs[i].k])[0]
            flat.append(1000.0 * (time.perf_counter() - start - arrivals[i]))
            same &= bool(np.array_equal(h, plain[i]))
        fifo_open_s = time.perf_counter() - start
        _log("serving: plain FIFO open loop %.2f s, p50 %.1f ms, p99 %.1f ms" % (
            fifo_open_s, np.percentile(flat, 50), np.percentile(flat, 99)))
    finally:
        for g in graphs:
            g.free()
    # the oracle's histograms of the requests it could count (stored digests)
    checked = matched = 0
    try:
        with open(DIGESTS_FILE) as f:
            chk = json.load(f)["serving"]["checked"]
        for i in range(R):
            rec = chk.get(str(i))
            if rec is not None:
                checked += 1
                matched += int(dense_digest(plain[i], codes[reqs[i].k]) == rec["hist"])
    except (OSError, KeyError, ValueError):
        pass
    by_k = {}
    for r, h in zip(reqs, plain):
        d = by_k.setdefault(str(r.k), {"requests": 0, "subgraphs": 0})
        d["requests"] += 1
        d["subgraphs"] += int(h.sum())
    return {"requests": R, "subgraphs": total, "by_k": by_k,
            "value": total / burst_s, "unit": "subgraphs/s",
            "plain_value": total / plain_s, "speedup_vs_plain": plain_s / burst_s,
            "capacity_req_per_s": R / burst_s, "plain_req_per_s": R / plain_s,
            "open_loop": {"load": load, "rate_req_per_s": rate,
                          "served": {"p50_ms": float(np.percentile(lat, 50)),
                                     "p99_ms": float(np.percentile(lat, 99)),
                                     "throughput": total / open_s, "wall_s": open_s},
                          "plain_fifo": {"p50_ms": float(np.percentile(flat, 50)),
                                         "p99_ms": float(np.percentile(flat, 99)),
                                         "throughput": total / fifo_open_s,
                                         "wall_s": fifo_open_s}},
            "served_equals_alone": bool(same),
            "oracle_checked": checked, "oracle_match": matched == checked}


def main():
    args = _parse()
    if args.gpus != 1:
        print("bench.py runs on one GPU only (no multi-GPU sharding is implemented); "
              "use --gpus 1", file=sys.stderr)
        sys.exit(2)
    import numpy as np

    from paper_1804_09741_amd import inputs as I

    # the oracle on the host cores, before this process touches the GPU
    procs = _cpu_share()
    cpu = None
    if not args.no_cpu_baseline:
        cpu = _cpu_legs(I, procs, args.cpu_graphs)

    import torch  # device buffers and the launch stream only

    from paper_1804_09741_amd import motifs as M

    ctx = M.Context(0)
    if args.copy_mib:
        n = args.copy_mib * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.float32, device="cuda:0")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    w = I.workload_k6_batch()
    _log("k=6 batch generated; building the k=6 table")
    t6 = ctx.table(6)
    _log("k=6 table built in %.1f ms" % t6.build_ms)
    graphs = [ctx.load_graph(*g) for g in w.graphs]
    method = {"auto": M.METHOD_AUTO, "esu": M.METHOD_ESU, "cores": M.METHOD_CORES}[args.method]
    opts = {"method": method} if method else {}
    if args.split:
        opts["split_threshold"] = args.split
    if args.waves_per_cu:
        opts["waves_per_cu"] = args.waves_per_cu
    autotune = None
    if args.autotune:
        tuned, tuned_ms, default_ms = ctx.autotune(graphs, t6, trials=3)
        opts = {kk: v for kk, v in tuned.items() if v}
        autotune = {"opts": opts, "tuned_pass_ms": tuned_ms, "default_pass_ms": default_ms}
        _log("autotune: %s (pass %.3f ms; defaults %.3f ms)" % (opts, tuned_ms, default_ms))
    r = _timed_batch(ctx, M, graphs, t6, args.steps, args.warmup, torch, **opts)
    subgraphs = int(r["totals"].sum())
    ms_per_step = 1000.0 * r["wall_s"] / args.steps
    value = subgraphs / (r["wall_s"] / args.steps)
    enum_ms = float(np.mean(r["enum_ms"]))
    kname = _kernel_name(6, r["stats"])
    cc6 = t6.class_codes()
    out = {
        "metric": "classified k-subgraphs/sec (k=5,6) batched vs plain; p50/p99 solve latency",
        "value": value,
        "unit": "subgraphs/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u64",
        "data": "synthetic",
        "config": {"workload": w.name, "k": 6, "graphs": len(w.graphs), "n": 700, "m": 1500,
                   "subgraphs_per_step": subgraphs},
        "roofline": _roofline(kname, enum_ms, subgraphs),
        "pass_ms": float(np.mean(r["pass_ms"])),
        "batch_stats": r["stats"],
        "batch_opts": opts,
        "autotune": autotune,
        "table_build_ms": {"6": t6.build_ms},
        "parity": {"k6_batch": _digest_check(w.name, r["hist"], cc6, w.graphs)},
    }
    _log("batched k=6: %.3f ms/step, counting kernel %.3f ms" % (ms_per_step, enum_ms))
    # the same pass captured whole (preparation, counting kernel, finish) as
    # one hipGraph: replays timed by the wall clock and by events around them
    rg = _timed_batch(ctx, M, graphs, t6, args.steps, args.warmup, torch,
                      **dict(opts, use_graph=2))
    out["whole_graph"] = {"ms_per_step": 1000.0 * rg["wall_s"] / args.steps,
                          "pass_ms": float(np.mean(rg["pass_ms"])),
                          "value": subgraphs / (rg["wall_s"] / args.steps),
                          "hists_equal": bool(np.array_equal(rg["hist"], r["hist"]))}
    _log("batched k=6, whole pass as one graph: %.3f ms/step" % out["whole_graph"]["ms_per_step"])
    if not args.no_plain:
        plain_s = _plain(ctx, graphs, t6, max(1, args.steps // 5), torch,
                         **({"method": method} if method else {}))
        _log("plain k=6: %.3f ms/pass" % (1000 * plain_s))
        out["plain"] = {"value": subgraphs / plain_s, "ms_per_step": 1000.0 * plain_s,
                        "speedup_batched": plain_s / (r["wall_s"] / args.steps)}
    if cpu is not None:
        out["cpu_baseline"] = _cpu_report(cpu["k6"], r["hist"], cc6, procs,
                                          "all graphs of the k=6 batch")
        single = cpu["single"]
        ns = len(single["hists"])
        ok = all(h == {int(cc6[j]): int(r["hist"][i][j]) for j in np.flatnonzero(r["hist"][i])}
                 for i, h in enumerate(single["hists"]))
        counted = sum(sum(h.values()) for h in single["hists"])
        out["cpu_baseline_single_thread"] = {
            "value": counted / single["wall_s"], "unit": "subgraphs/s", "cores": 1,
            "kind": "oracle", "sample": "graphs 0..%d of the k=6 batch (%d subgraphs), one "
                                        "thread, %.1f s" % (ns - 1, counted, single["wall_s"]),
            "hists_match_gpu": bool(ok)}
    for g in graphs:
        g.free()

    if not args.no_k5:
        w5 = I.workload_k5_batch()
        t5 = ctx.table(5)
        g5 = [ctx.load_graph(*g) for g in w5.graphs]
        o5 = {"split_threshold": args.k5_split} if args.k5_split else {}
        if method:
            o5["method"] = method
        steps5 = max(2, args.steps // 3)
        r5 = _timed_batch(ctx, M, g5, t5, steps5, 1, torch, **o5)
        s5 = int(r5["totals"].sum())
        k5_ms = float(np.mean(r5["enum_ms"]))
        k5name = _kernel_name(5, r5["stats"])
        # work unit of the counting from (k-2)-sets: the connected 3-sets
        # (cores) of the batch, counted by the k = 3 path on the same graphs
        h3, _ = ctx.count_batch(g5, ctx.table(3))
        cores = int(h3.sum())
        cc5 = t5.class_codes()
        k5 = {"workload": w5.name, "value": s5 / (r5["wall_s"] / steps5),
              "subgraphs_per_step": s5, "kernel_ms": k5_ms,
              "pass_ms": float(np.mean(r5["pass_ms"])), "table_build_ms": t5.build_ms,
              "kernel": k5name,
              "roofline": _roofline(k5name, k5_ms,
                                    None if k5name.startswith("core") else s5),
              "cores_per_launch": cores, "cores_per_s": cores / (k5_ms / 1e3),
              "batch_stats": r5["stats"],
              "parity": _digest_check(w5.name, r5["hist"], cc5, w5.graphs)}
        if cpu is not None:
            k5["cpu_baseline"] = _cpu_report(cpu["k5"], r5["hist"], cc5, procs,
                                             "first graphs of the k=5 batch")
        if not args.no_plain:
            p5 = _plain(ctx, g5, t5, 1, torch, **({"method": method} if method else {}))
            k5["plain_value"] = s5 / p5
            k5["speedup_batched"] = p5 / (r5["wall_s"] / steps5)
        out["k5_batch"] = k5
        _log("k=5 batch: %.3f ms/step" % k5["pass_ms"])
        for g in g5:
            g.free()
    if not args.no_methods:
        out["methods"] = _methods(ctx, M, I, torch)
    if not args.no_variants:
        out["variants"] = _variants(ctx, M, I, torch)
    if not args.no_k7:
        out["k7"] = _k7(ctx, M, I, torch)
    if not args.no_ensemble:
        out["ensemble"] = _ensemble(ctx, M, I, torch, cpu=not args.no_cpu_baseline)
    if args.serve:
        out["serving"] = _serving(ctx, M, I, args.serve, args.serve_load, torch)
    ctx.close()
    print(json.dumps(out))


if __name__ == "__main__":
    main()
