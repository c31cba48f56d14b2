#!/usr/bin/env python3
"""Benchmark of the Motifs-k hot path on one MI355X.

    python bench.py [--steps K] [--warmup W] [--gpus 1]

One step = one full pass of the path over one batch of synthetic graphs,
inputs (CSR graphs) and class table already resident in HBM: typed
adjacency, work-unit plan, persistent enumeration with code formation,
table lookup and histograms -- one replay of the batch's captured hipGraph.

Workload: k = 6, one directed graph with n = 700, m = 1500 (power-law
out-degrees up to 60, Poisson in-degrees) plus 30 degree-preserving
randomisations, counted in one launch (31 histograms of 1,530,843 classes).

Printed: one JSON line with subgraphs/s, the roofline of the enumeration
kernel (algorithmic HBM bytes: a 4-byte table entry and an 8-byte counter
read + write per subgraph, over the kernel's HIP-event duration), the CPU
oracle timed on a bounded sample, the plain one-graph-per-launch form on
the same graphs, table build times, and the k = 5 batch (1 + 100
randomisations of n = 1000, m = 3000) as a second reading; then both
counting methods, the code-formation variants (arc tests on bit matrices or
sorted lists, marks in LDS or device memory) with a k = 6 graph of 2^20
vertices, and the ensemble pipeline.
"""

from __future__ import annotations

import argparse
import json
import os
import sys
import time

HBM_PEAK_GBS = 8000.0
BYTES_PER_SUBGRAPH = 4 + 8 + 8
ROOT = os.path.dirname(os.path.abspath(__file__))
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "enum_kernel_hbm_traffic.json")
KERNEL_SOURCES = ("paper_1804_09741_amd/csrc/enum.hip", "paper_1804_09741_amd/csrc/core.hip",
                  "paper_1804_09741_amd/csrc/esu.h", "paper_1804_09741_amd/csrc/internal.h")


def _measured_traffic(kernel):
    """HBM bytes per launch of `kernel` from the committed counter runs
    (FETCH_SIZE + WRITE_SIZE, scaled by a copy of known size), or None when
    the kernel source changed since they were taken."""
    import hashlib
    try:
        with open(TRAFFIC_FILE) as f:
            rec = json.load(f)
        h = hashlib.sha256()
        for name in KERNEL_SOURCES:
            with open(os.path.join(ROOT, name), "rb") as f:
                h.update(f.read())
        if h.hexdigest()[:16] != rec["source_sha256_16"]:
            return None
        return rec["kernels"][kernel]["traffic_bytes"]
    except (OSError, KeyError, ValueError):
        return None


def _kernel_name(k, stats):
    """The counting kernel a batch ran (its stats name the method)."""
    return ("core_kernel<%d>" if stats.get("method") == 2 else "enum_kernel<%d>") % k


def _log(msg):
    print("[bench] " + msg, file=sys.stderr, flush=True)


def _parse():
    p = argparse.ArgumentParser(description=__doc__.split("\n")[1])
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=10)
    p.add_argument("--warmup", type=int, default=2)
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--no-k5", action="store_true", help="skip the k=5 batch reading")
    p.add_argument("--no-plain", action="store_true", help="skip the plain comparator")
    p.add_argument("--cpu-graphs", type=int, default=10,
                   help="graphs of the batch the CPU oracle counts (bounded sample)")
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
    p.add_argument("--serve", type=int, default=0, metavar="R",
                   help="also run the serving workload with R requests (0: skip)")
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


def _oracle_total(args):
    """Worker of the parallel CPU baseline: the oracle's count of one graph."""
    rp, col, k = args
    from oracle import oracle as O
    h = O.count(rp, col, k)
    return sum(h.values())


def _oracle_ready(_):
    """Worker warm-up: load the oracle library."""
    import numpy as np
    from oracle import oracle as O
    O.count(np.zeros(4, np.int32), np.zeros(0, np.int32), 3)
    return os.getpid()


def _cpu_parallel(graphs, k, procs):
    """The oracle over every graph of the workload, one graph per task, in
    `procs` worker processes, timed from the first task to the last result
    after the workers are up.  Called before this process touches the GPU,
    so the workers start from a process without device state."""
    import multiprocessing
    from concurrent.futures import ProcessPoolExecutor
    with ProcessPoolExecutor(max_workers=procs,
                             mp_context=multiprocessing.get_context("spawn")) as pool:
        list(pool.map(_oracle_ready, range(procs)))
        t0 = time.perf_counter()
        totals = list(pool.map(_oracle_total, [(rp, col, k) for rp, col in graphs]))
        wall = time.perf_counter() - t0
    counted = int(sum(totals))
    return {"value": counted / wall, "unit": "subgraphs/s", "cores": procs, "kind": "oracle",
            "sample": "all %d graphs of the batch (%d subgraphs), %d processes, %.1f s" % (
                len(graphs), counted, procs, wall),
            "totals": [int(x) for x in totals]}


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
                    "roofline": {"bound": "hbm", "kernel": "enum_lists_kernel<6, 3>",
                                 "achieved": BYTES_PER_SUBGRAPH * sub / (kern / 1e3) / 1e9,
                                 "peak": HBM_PEAK_GBS, "unit": "GB/s",
                                 "frac": BYTES_PER_SUBGRAPH * sub / (kern / 1e3) / 1e9 / HBM_PEAK_GBS,
                                 "bytes_per_subgraph": BYTES_PER_SUBGRAPH}}
    _log("variants: %s, %d subgraphs, pass %.1f ms (kernel %.1f ms), %.3g subgraphs/s" % (
        w.name, sub, res["large"]["pass_ms"], kern, res["large"]["value"]))
    return res


def _k7(ctx, M, I, torch):
    """k = 7 on the 31 graphs of the k = 6 batch (classes by canonical code,
    canonicalised on the device): two calls.  The first, on a context that
    has not counted k = 7 yet, grows the class tables and fills the
    context's canonical-code cache (its wall time is reported as
    first_call_ms); the second, timed, finds that cache warm."""
    import numpy as np
    w = I.workload_k6_batch()
    gs = [ctx.load_graph(*g) for g in w.graphs]
    try:
        t0 = time.perf_counter()
        ctx.count7(gs)
        torch.cuda.synchronize()
        first = time.perf_counter() - t0
        t0 = time.perf_counter()
        out, totals, kern = ctx.count7(gs)
        wall = time.perf_counter() - t0
    finally:
        for g in gs:
            g.free()
    sub = int(np.sum(totals))
    classes = [len(c) for c, _ in out]
    res = {"workload": w.name.replace("k6_", "k7_"), "subgraphs": sub, "kernel_ms": kern,
           "call_ms": wall * 1e3, "value": sub / (kern / 1e3), "unit": "subgraphs/s (kernel)",
           "cache": "warm", "first_call_ms": first * 1e3,
           "classes_mean": float(np.mean(classes)), "classes_max": int(max(classes))}
    _log("k=7 on the k=6 batch: %d subgraphs, kernel %.1f ms (%.3g/s), call %.1f ms (warm cache; "
         "first call %.1f ms), %.0f classes per graph" % (sub, kern, res["value"], res["call_ms"],
                                                          res["first_call_ms"], res["classes_mean"]))
    # one graph past the LDS limit (marks and tags in device memory)
    wl = I.workload_k6_large(1 << 17)
    g = ctx.load_graph(*wl.graphs[0])
    try:
        ctx.count7([g])
        t0 = time.perf_counter()
        out, totals, kern = ctx.count7([g])
        wall = time.perf_counter() - t0
    finally:
        g.free()
    sub = int(totals[0])
    res["large"] = {"workload": wl.name.replace("k6_", "k7_"), "subgraphs": sub, "kernel_ms": kern,
                    "call_ms": wall * 1e3, "value": sub / (kern / 1e3),
                    "unit": "subgraphs/s (kernel)", "classes": len(out[0][0])}
    _log("k=7 on %s: %d subgraphs, kernel %.1f ms (%.3g/s), %d classes" % (
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
    """Serving workload: R (graph, k) requests, graphs resident on the device.

    1. plain: one request per launch, first come first served (mk_count);
    2. served, closed loop: all requests submitted at once -> capacity;
    3. served, open loop: Poisson arrivals at `load` x capacity -> p50/p99 of
       (completion - submission) as timed by the server.
    Every served histogram must equal the plain one.
    """
    import threading

    import numpy as np

    reqs = I.serving_requests(count=R)
    _log("serving: %d requests generated" % R)
    for k in (3, 4, 5, 6):
        ctx.table(k)
    graphs = [ctx.load_graph(*r.graph) for r in reqs]
    tables = {k: ctx.table(k) for k in (3, 4, 5, 6)}
    t0 = time.perf_counter()
    plain = [ctx.count(g, tables[r.k])[0] for g, r in zip(graphs, reqs)]
    plain_s = time.perf_counter() - t0
    total = int(sum(int(h.sum()) for h in plain))
    _log("serving: plain FIFO %.2f s, %d subgraphs" % (plain_s, total))

    srv = ctx.server()
    try:
        t0 = time.perf_counter()
        tickets = [srv.submit(g, r.k) for g, r in zip(graphs, reqs)]
        burst = [srv.wait(t, r.k) for t, r in zip(tickets, reqs)]
        burst_s = time.perf_counter() - t0
        same = all(np.array_equal(h, p) for (h, _), p in zip(burst, plain))
        _log("serving: closed loop %.2f s" % burst_s)
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
    for g in graphs:
        g.free()
    return {"requests": R, "subgraphs": total, "value": total / burst_s,
            "plain_value": total / plain_s, "speedup_vs_plain": plain_s / burst_s,
            "capacity_req_per_s": R / burst_s, "open_loop_rate_req_per_s": rate,
            "open_loop_throughput": total / open_s,
            "p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
            "served_equals_alone": bool(same)}


def main():
    args = _parse()
    if args.gpus != 1:
        print("bench.py runs on one GPU only (no multi-GPU sharding is implemented); "
              "use --gpus 1", file=sys.stderr)
        sys.exit(2)
    import numpy as np

    from paper_1804_09741_amd import inputs as I

    # the oracle on all host cores, before this process touches the GPU
    cpu_par = None
    if not args.no_cpu_baseline:
        procs = max(1, min(16, os.cpu_count() or 1, 31))
        cpu_par = _cpu_parallel(I.workload_k6_batch().graphs, 6, procs)
        _log("cpu oracle, %d processes: %s" % (procs, cpu_par["sample"]))

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
    tuned = None
    if args.autotune:
        tuned, tuned_ms = ctx.autotune(graphs, t6, trials=2)
        opts = {kk: v for kk, v in tuned.items() if kk != "debug_flags" and v}
        _log("autotune: %s (pass %.3f ms)" % (opts, tuned_ms))
    r = _timed_batch(ctx, M, graphs, t6, args.steps, args.warmup, torch, **opts)
    subgraphs = int(r["totals"].sum())
    ms_per_step = 1000.0 * r["wall_s"] / args.steps
    value = subgraphs / (r["wall_s"] / args.steps)
    enum_ms = float(np.mean(r["enum_ms"]))
    algo_bytes = BYTES_PER_SUBGRAPH * subgraphs
    achieved = algo_bytes / (enum_ms * 1e-3) / 1e9
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
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS,
                     "traffic": _measured_traffic(_kernel_name(6, r["stats"])),
                     "kernel": _kernel_name(6, r["stats"]), "kernel_ms": enum_ms,
                     "bytes_per_subgraph": BYTES_PER_SUBGRAPH},
        "pass_ms": float(np.mean(r["pass_ms"])),
        "batch_stats": r["stats"],
        "batch_opts": opts,
        "table_build_ms": {"6": t6.build_ms},
    }
    _log("batched k=6: %.3f ms/step, enum kernel %.3f ms" % (ms_per_step, enum_ms))
    if not args.no_plain:
        plain_s = _plain(ctx, graphs, t6, max(1, args.steps // 5), torch,
                         **({"method": method} if method else {}))
        _log("plain k=6: %.3f ms/pass" % (1000 * plain_s))
        out["plain"] = {"value": subgraphs / plain_s, "ms_per_step": 1000.0 * plain_s,
                        "speedup_batched": plain_s / (r["wall_s"] / args.steps)}

    # CPU oracle on a bounded sample of the same workload (graph by graph)
    if not args.no_cpu_baseline:
        from oracle import oracle as O
        cc = t6.class_codes()
        ns = min(args.cpu_graphs, len(w.graphs))
        t0 = time.perf_counter()
        ok = True
        counted = 0
        for i in range(ns):
            h = O.count(*w.graphs[i], 6)
            counted += sum(h.values())
            nz = np.flatnonzero(r["hist"][i])
            ok &= h == {int(cc[j]): int(r["hist"][i][j]) for j in nz}
        cpu_s = time.perf_counter() - t0
        _log("cpu oracle: %d graphs in %.1f s" % (ns, cpu_s))
        out["cpu_baseline"] = {"value": counted / cpu_s, "unit": "subgraphs/s", "cores": 1,
                               "kind": "oracle",
                               "sample": "graphs 0..%d of the batch (%d subgraphs), single "
                                         "thread, %.1f s" % (ns - 1, counted, cpu_s),
                               "matches_gpu": bool(ok)}
        totals = cpu_par.pop("totals")
        cpu_par["totals_match_gpu"] = totals == [int(x) for x in r["totals"]]
        out["cpu_baseline_parallel"] = cpu_par
    for g in graphs:
        g.free()

    if not args.no_k5:
        w5 = I.workload_k5_batch()
        t5 = ctx.table(5)
        g5 = [ctx.load_graph(*g) for g in w5.graphs]
        o5 = {"split_threshold": args.k5_split} if args.k5_split else {}
        if method:
            o5["method"] = method
        r5 = _timed_batch(ctx, M, g5, t5, max(2, args.steps // 3), 1, torch, **o5)
        s5 = int(r5["totals"].sum())
        k5 = {"workload": w5.name, "value": s5 / (r5["wall_s"] / max(2, args.steps // 3)),
              "subgraphs_per_step": s5, "kernel_ms": float(np.mean(r5["enum_ms"])),
              "pass_ms": float(np.mean(r5["pass_ms"])), "table_build_ms": t5.build_ms,
              "kernel": _kernel_name(5, r5["stats"]),
              "traffic": _measured_traffic(_kernel_name(5, r5["stats"])),
              "batch_stats": r5["stats"]}
        if not args.no_plain:
            p5 = _plain(ctx, g5, t5, 1, torch, **({"method": method} if method else {}))
            k5["plain_value"] = s5 / p5
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
