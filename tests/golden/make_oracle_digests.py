#!/usr/bin/env python3
"""Write tests/golden/oracle_digests.json: the CPU oracle's histograms of
every graph of the full-size workloads, as digests.

    python tests/golden/make_oracle_digests.py [--procs P]

Only the oracle (``oracle/``) and the seeded input generators
(``paper_1804_09741_amd/inputs.py``, which hold none of the method's
arithmetic) are called; nothing here touches the GPU library.  For each
graph the file holds the digest of its CSR arrays, the oracle's number of
connected k-sets, its number of classes and the digest of its histogram as
(canonical code, count) pairs (``oracle/digest.py``).  The GPU tests
recompute the digest from the GPU histograms and compare; a graph whose
input digest differs is reported as a changed input.

Workloads:
  * k = 3: directed G(200, 800);
  * k = 4: directed Chung-Lu n = 2000, m = 10000;
  * k = 5 batch: the Chung-Lu original (n = 1000, m = 3000) and its 100
    randomisations, all 101 graphs;
  * k = 6 batch: the power-law original (n = 700, m = 1500) and its 30
    randomisations, all 31 graphs;
  * k = 7 on the 31 graphs of the k = 6 batch;
  * serving stream: every request of the first 1000 whose size estimate
    (sum over vertices of C(undirected degree, k - 1), the stars of the
    request) is at most 1e8 subgraphs.

The whole run is about 6,000 CPU-seconds of oracle (the k = 5 batch holds
1.4e10 5-sets), one graph per task over the worker processes.
"""

from __future__ import annotations

import argparse
import json
import multiprocessing
import os
import sys
import time
from math import comb

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)
sys.path.insert(0, os.path.dirname(HERE))

OUT = os.path.join(HERE, "oracle_digests.json")
SERVE_COUNT = 1000
SERVE_LIMIT = 10 ** 8


def star_estimate(row_ptr, col, k):
    """Sum over vertices of C(undirected degree, k - 1)."""
    import numpy as np
    n = len(row_ptr) - 1
    src = np.repeat(np.arange(n, dtype=np.int64), np.diff(row_ptr))
    dst = np.asarray(col, dtype=np.int64)
    key = np.unique(np.minimum(src, dst) * n + np.maximum(src, dst))
    deg = np.bincount(key // n, minlength=n) + np.bincount(key % n, minlength=n)
    return sum(comb(int(d), k - 1) for d in deg)


def _graph(spec):
    from paper_1804_09741_amd import inputs as I
    kind, idx = spec
    if kind == "k3":
        return 3, I.workload_k3_er().graphs[0]
    if kind == "k4":
        return 4, I.workload_k4_chunglu().graphs[0]
    if kind == "k5":
        return 5, I.k5_batch_graph(idx)
    if kind == "k6":
        return 6, I.k6_batch_graph(idx)
    if kind == "k7":
        return 7, I.k6_batch_graph(idx)
    if kind == "serve":
        return I.serving_request(idx)
    raise ValueError(kind)


def _job(spec):
    from oracle import oracle as O
    from oracle.digest import dict_digest, graph_digest
    k, (rp, col) = _graph(spec)
    t0 = time.perf_counter()
    h = O.count(rp, col, k)
    return spec, {"k": k, "n": len(rp) - 1, "m": len(col), "graph": graph_digest(rp, col),
                  "total": int(sum(h.values())), "classes": len(h), "hist": dict_digest(h),
                  "oracle_s": round(time.perf_counter() - t0, 2)}


def _serve_size(i):
    from paper_1804_09741_amd import inputs as I
    k, (rp, col) = I.serving_request(i)
    return i, k, star_estimate(rp, col, k)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--procs", type=int, default=os.cpu_count() or 1)
    args = ap.parse_args()
    ctx = multiprocessing.get_context("spawn")
    t0 = time.perf_counter()
    with ctx.Pool(args.procs) as pool:
        sizes = pool.map(_serve_size, range(SERVE_COUNT))
        chosen = [i for i, _, est in sizes if est <= SERVE_LIMIT]
        print("serving: %d of %d requests within %g" % (len(chosen), SERVE_COUNT, SERVE_LIMIT),
              flush=True)
        specs = ([("k5", i) for i in range(101)] + [("k7", i) for i in range(31)] +
                 [("serve", i) for i in chosen] + [("k6", i) for i in range(31)] +
                 [("k3", 0), ("k4", 0)])
        res = {}
        for n_done, (spec, rec) in enumerate(pool.imap_unordered(_job, specs), 1):
            res[spec] = rec
            if n_done % 25 == 0 or n_done == len(specs):
                print("%d / %d graphs, %.0f s" % (n_done, len(specs), time.perf_counter() - t0),
                      flush=True)
    out = {
        "about": "CPU oracle histograms of the full-size workloads as digests "
                 "(oracle/digest.py); written by tests/golden/make_oracle_digests.py, "
                 "which calls only oracle/ and the seeded generators",
        "k3_er_n200_m800": [res[("k3", 0)]],
        "k4_chunglu_n2000_m10000": [res[("k4", 0)]],
        "k5_batch101_chunglu_n1000_m3000": [res[("k5", i)] for i in range(101)],
        "k6_batch31_powerlaw_n700_m1500": [res[("k6", i)] for i in range(31)],
        "k7_batch31_powerlaw_n700_m1500": [res[("k7", i)] for i in range(31)],
        "serving": {"requests": SERVE_COUNT, "limit": SERVE_LIMIT,
                    "estimate": "sum over vertices of C(undirected degree, k - 1)",
                    "checked": {str(i): res[("serve", i)] for i in chosen}},
    }
    with open(OUT, "w") as f:
        json.dump(out, f, indent=0, sort_keys=False)
        f.write("\n")
    print("wrote %s in %.0f s" % (OUT, time.perf_counter() - t0))


if __name__ == "__main__":
    main()
