"""Summaries of rocprofv3 CSV output (kernel statistics and counter passes).

    python -m paper_1804_09741_amd.profsum stats DIR --out FILE.md --command CMD
    python -m paper_1804_09741_amd.profsum counters DIR [DIR ...] --copy-mib MIB
        --bench-log LOG --out-md FILE.md --out-json FILE.json --command CMD [CMD ...]
    python -m paper_1804_09741_amd.profsum pmc DIR [DIR ...] --kernels REGEX
        --out FILE.md --command CMD [CMD ...] [--per NAME=COUNT ...]

`stats` turns `run_kernel_stats.csv` of a `--kernel-trace --stats` run into a
Markdown table.  `counters` averages every counter of every pass (one
`--pmc` run per directory) per kernel and dispatch, and writes

* a Markdown table of all counters of the enumeration kernels and of the
  calibration copy;
`pmc` averages every counter of the kernels whose names match REGEX, per
dispatch, over one or more `--pmc` runs, optionally also per unit of work
(`--per "k7_kernel<0>=2058308995"`: subgraphs of one dispatch).

* the HBM traffic record that bench.py reports: FETCH_SIZE and WRITE_SIZE
  (KiB per dispatch) of each enumeration kernel, each scaled by what the
  same counter reads for the device-to-device copy of `--copy-mib` MiB
  (which reads and writes exactly that many bytes), with a hash of the
  kernel sources so that a stale record is not used.
"""

from __future__ import annotations

import argparse
import csv
import hashlib
import json
import os
import re
from collections import defaultdict

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
KERNEL_SOURCES = ("paper_1804_09741_amd/csrc/enum.hip", "paper_1804_09741_amd/csrc/core.hip",
                  "paper_1804_09741_amd/csrc/esu.h", "paper_1804_09741_amd/csrc/internal.h")
COPY_KERNEL = "__amd_rocclr_copyBuffer"


def source_hash() -> str:
    h = hashlib.sha256()
    for name in KERNEL_SOURCES:
        with open(os.path.join(ROOT, name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def short_name(name: str) -> str:
    """`void mk::enum_kernel<6>(mk::DevGraph const*, ...)` -> `enum_kernel<6>`."""
    s = re.sub(r"^void ", "", name.strip())
    depth = 0
    for i, ch in enumerate(s):
        if ch == "<":
            depth += 1
        elif ch == ">":
            depth -= 1
        elif ch == "(" and depth == 0:
            s = s[:i]
            break
    return s[4:] if s.startswith("mk::") else s


def _csv(path):
    with open(path, newline="") as f:
        return list(csv.DictReader(f))


def stats_table(d: str):
    rows = _csv(os.path.join(d, "run_kernel_stats.csv"))
    out = ["| kernel | calls | avg (us) | min (us) | max (us) | share |",
           "|---|---:|---:|---:|---:|---:|"]
    for r in rows:
        out.append("| `%s` | %s | %.1f | %.1f | %.1f | %s%% |" % (
            short_name(r["Name"]), r["Calls"], float(r["AverageNs"]) / 1e3,
            float(r["MinNs"]) / 1e3, float(r["MaxNs"]) / 1e3, r["Percentage"]))
    return out


def counter_means(dirs, copy_bytes):
    """{kernel: {counter: mean per dispatch}}, {kernel: dispatches}.

    In each pass the calibration copy is the copy dispatch with the largest
    reading: the run's other copies move a few KiB of counters and
    histograms."""
    acc = defaultdict(lambda: defaultdict(list))
    for d in dirs:
        per = defaultdict(float)
        names = {}
        for r in _csv(os.path.join(d, "run_counter_collection.csv")):
            key = (int(r["Dispatch_Id"]), r["Counter_Name"])
            per[key] += float(r["Counter_Value"])
            names[int(r["Dispatch_Id"])] = short_name(r["Kernel_Name"])
        by_counter = defaultdict(dict)
        for (disp, cname), v in per.items():
            by_counter[cname][disp] = v
        for cname, vals in by_counter.items():
            copies = [v for disp, v in vals.items() if names[disp] == COPY_KERNEL]
            if copies:
                acc[COPY_KERNEL + " (%d MiB)" % (copy_bytes >> 20)][cname].append(max(copies))
            for disp, v in vals.items():
                if names[disp].startswith(("enum_kernel", "core_kernel")):
                    acc[names[disp]][cname].append(v)
    means = {k: {c: sum(v) / len(v) for c, v in cs.items()} for k, cs in acc.items()}
    counts = {k: max(len(v) for v in cs.values()) for k, cs in acc.items()}
    return means, counts


def kernel_counter_means(dirs, pattern):
    """{kernel: {counter: mean per dispatch}}, {kernel: dispatches} for the
    kernels whose short names match `pattern`."""
    acc = defaultdict(lambda: defaultdict(list))
    rx = re.compile(pattern)
    for d in dirs:
        per = defaultdict(float)
        names = {}
        for r in _csv(os.path.join(d, "run_counter_collection.csv")):
            key = (int(r["Dispatch_Id"]), r["Counter_Name"])
            per[key] += float(r["Counter_Value"])
            names[int(r["Dispatch_Id"])] = short_name(r["Kernel_Name"])
        for (disp, cname), v in per.items():
            if rx.search(names[disp]):
                acc[names[disp]][cname].append(v)
    means = {k: {c: sum(v) / len(v) for c, v in cs.items()} for k, cs in acc.items()}
    counts = {k: max(len(v) for v in cs.values()) for k, cs in acc.items()}
    return means, counts


def _bench_record(path):
    with open(path) as f:
        lines = [ln for ln in f.read().splitlines() if ln.startswith("{")]
    return json.loads(lines[-1])


def main(argv=None):
    ap = argparse.ArgumentParser(description="summaries of rocprofv3 CSV output")
    sub = ap.add_subparsers(dest="cmd", required=True)
    s = sub.add_parser("stats")
    s.add_argument("dir")
    s.add_argument("--out", required=True)
    s.add_argument("--title", default="rocprofv3 kernel summary")
    s.add_argument("--command", required=True)
    s.add_argument("--note", default="")
    c = sub.add_parser("counters")
    c.add_argument("dirs", nargs="+")
    c.add_argument("--copy-mib", type=int, required=True)
    c.add_argument("--bench-log", required=True)
    c.add_argument("--out-md", required=True)
    c.add_argument("--out-json", required=True)
    c.add_argument("--title", default="enum_kernel hardware counters")
    c.add_argument("--command", nargs="+", required=True)
    q = sub.add_parser("pmc")
    q.add_argument("dirs", nargs="+")
    q.add_argument("--kernels", required=True)
    q.add_argument("--out", required=True)
    q.add_argument("--title", default="hardware counters")
    q.add_argument("--command", nargs="+", required=True)
    q.add_argument("--per", nargs="*", default=[], metavar="KERNEL=UNITS")
    q.add_argument("--note", default="")
    a = ap.parse_args(argv)

    if a.cmd == "pmc":
        means, counts = kernel_counter_means(a.dirs, a.kernels)
        per = {}
        for item in a.per:
            name, units = item.rsplit("=", 1)
            per[name] = float(units)
        kerns = sorted(means)
        lines = ["# " + a.title, "",
                 "One rocprofv3 `--pmc` run per counter set, from /tmp with TMPDIR=/tmp; "
                 "$R is the repository root:", "", "```"] + a.command + ["```", "",
                 "Mean per dispatch over " + ", ".join(
                     "%s: %d dispatches" % (k, counts[k]) for k in kerns) + ".", ""]
        heads = []
        for k in kerns:
            heads.append(k)
            if k in per:
                heads.append("%s per unit" % k)
        lines += ["| counter | " + " | ".join(heads) + " |", "|---|" + "---:|" * len(heads)]
        for cname in sorted({c for k in kerns for c in means[k]}):
            cells = []
            for k in kerns:
                v = means[k].get(cname, float("nan"))
                cells.append("%.4g" % v)
                if k in per:
                    cells.append("%.4g" % (v / per[k]))
            lines.append("| %s | " % cname + " | ".join(cells) + " |")
        if per:
            lines += ["", "Units per dispatch: " + ", ".join(
                "%s %.6g" % (k, v) for k, v in sorted(per.items())) + "."]
        if a.note:
            lines += ["", a.note]
        with open(a.out, "w") as f:
            f.write("\n".join(lines) + "\n")
        return

    if a.cmd == "stats":
        lines = ["# " + a.title, "",
                 "Command (from /tmp with TMPDIR=/tmp; $R is the repository root):", "",
                 "```", a.command, "```", "",
                 "Kernel sources (enum.hip, core.hip, esu.h, internal.h) sha256[:16] = `%s`." % source_hash(),
                 "Durations in microseconds.", ""]
        lines += stats_table(a.dir)
        if a.note:
            lines += ["", a.note]
        with open(a.out, "w") as f:
            f.write("\n".join(lines) + "\n")
        return

    copy_bytes = a.copy_mib << 20
    means, counts = counter_means(a.dirs, copy_bytes)
    copy_key = COPY_KERNEL + " (%d MiB)" % a.copy_mib
    cal = means[copy_key]
    fetch_scale = copy_bytes / (cal["FETCH_SIZE"] * 1024.0)
    write_scale = copy_bytes / (cal["WRITE_SIZE"] * 1024.0)
    bench = _bench_record(a.bench_log)
    def kernel(k, stats):
        # the method the batch ran: 1 enumeration, 2 counting from (k-2)-sets
        return ("core_kernel<%d>" if stats.get("method") == 2 else "enum_kernel<%d>") % k

    per_launch = {kernel(6, bench["batch_stats"]): (bench["config"]["workload"],
                                                   bench["config"]["subgraphs_per_step"])}
    if "k5_batch" in bench:
        per_launch[kernel(5, bench["k5_batch"]["batch_stats"])] = (
            bench["k5_batch"]["workload"], bench["k5_batch"]["subgraphs_per_step"])
    bps = bench["roofline"]["bytes_per_subgraph"]
    rec = {"source_sha256_16": source_hash(), "sources": list(KERNEL_SOURCES),
           "calibration": {"kernel": COPY_KERNEL + " (torch copy_ of %d MiB)" % a.copy_mib,
                           "bytes": copy_bytes, "FETCH_SIZE_KiB": cal["FETCH_SIZE"],
                           "WRITE_SIZE_KiB": cal["WRITE_SIZE"], "fetch_scale": fetch_scale,
                           "write_scale": write_scale},
           "kernels": {}}
    for kern, (wl, sub_) in sorted(per_launch.items()):
        m = means[kern]
        fb = m["FETCH_SIZE"] * 1024.0 * fetch_scale
        wb = m["WRITE_SIZE"] * 1024.0 * write_scale
        rec["kernels"][kern] = {"workload": wl, "dispatches": counts[kern], "fetch_bytes": fb,
                                "write_bytes": wb, "traffic_bytes": fb + wb,
                                "subgraphs_per_launch": sub_,
                                "algorithmic_bytes": bps * sub_}
    with open(a.out_json, "w") as f:
        json.dump(rec, f, indent=1)
        f.write("\n")

    kerns = sorted(k for k in means if k.startswith(("enum_kernel", "core_kernel"))) + [copy_key]
    lines = ["# " + a.title, "",
             "One rocprofv3 `--pmc` run per counter set, from /tmp with TMPDIR=/tmp; "
             "$R is the repository root:", "", "```"] + a.command + [
             "```", "",
             "Kernel sources (enum.hip, core.hip, esu.h, internal.h) sha256[:16] = `%s`." % rec["source_sha256_16"],
             "Mean per dispatch over %s." % ", ".join(
                 "%s: %d dispatches" % (k, counts[k]) for k in kerns[:-1]), "",
             "| counter | " + " | ".join(kerns) + " |",
             "|---|" + "---:|" * len(kerns)]
    names = sorted({c for k in kerns for c in means[k]})
    for cname in names:
        lines.append("| %s | " % cname + " | ".join(
            "%.4g" % means[k].get(cname, float("nan")) for k in kerns) + " |")
    lines += ["", "HBM traffic per launch (FETCH_SIZE x %.4f + WRITE_SIZE x %.4f, KiB -> bytes; "
              "the factors make the %d MiB copy read and write %d MiB):" % (
                  fetch_scale, write_scale, a.copy_mib, a.copy_mib), "",
              "| kernel | workload | read (MB) | written (MB) | algorithmic (MB) | "
              "traffic / algorithmic |", "|---|---|---:|---:|---:|---:|"]
    for kern, r in rec["kernels"].items():
        lines.append("| %s | %s | %.1f | %.1f | %.1f | %.3f |" % (
            kern, r["workload"], r["fetch_bytes"] / 1e6, r["write_bytes"] / 1e6,
            r["algorithmic_bytes"] / 1e6, r["traffic_bytes"] / r["algorithmic_bytes"]))
    with open(a.out_md, "w") as f:
        f.write("\n".join(lines) + "\n")


if __name__ == "__main__":
    main()
