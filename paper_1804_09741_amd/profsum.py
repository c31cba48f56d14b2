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


# MI355X figures used by the rooflines (vendor-published unit counts and
# clock).  Issue: every compute unit has four SIMD16 vector units -- a wave64
# VALU instruction occupies one for four cycles, so a CU completes at most
# one wave64 VALU instruction per cycle -- and one scalar unit that issues
# one SALU instruction per cycle; the LDS takes one instruction per cycle.
NUM_CUS = 256
CLOCK_HZ = 2.4e9
ISSUE_PEAK = NUM_CUS * CLOCK_HZ          # wave-instructions/s per pipe
HBM_PEAK_BPS = 8.0e12
# L2 atomics: 16 channels per XCD, 8 XCDs, one 64-bit atomic per channel and
# cycle (an assumption of the channel design, stated as such)
L2_ATOMIC_PEAK = 8 * 16 * CLOCK_HZ


def derived(c: dict, kernel_s: float) -> dict:
    """Issue, lane, wait, L2 and HBM figures of one kernel launch from its
    per-dispatch counter means `c` (FETCH_SIZE / WRITE_SIZE already scaled to
    bytes as `fetch_bytes` / `write_bytes`) and its duration in seconds."""
    out = {}
    pipes = {"VALU": "SQ_INSTS_VALU", "SALU": "SQ_INSTS_SALU", "LDS": "SQ_INSTS_LDS"}
    for name, key in pipes.items():
        if key in c and kernel_s > 0:
            rate = c[key] / kernel_s
            out[name.lower()] = {"insts_per_launch": c[key], "rate": rate,
                                 "frac": rate / ISSUE_PEAK}
    if c.get("SQ_ACTIVE_INST_VALU"):
        out["lane_util"] = c.get("SQ_THREAD_CYCLES_VALU", 0.0) / (64.0 * c["SQ_ACTIVE_INST_VALU"])
    if c.get("SQ_WAVE_CYCLES"):
        out["wait_frac"] = c.get("SQ_WAIT_ANY", 0.0) / c["SQ_WAVE_CYCLES"]
    if c.get("SQ_ACTIVE_INST_LDS"):
        out["lds_conflict_frac"] = c.get("SQ_LDS_BANK_CONFLICT", 0.0) / c["SQ_ACTIVE_INST_LDS"]
    hits, miss = c.get("TCC_HIT_sum"), c.get("TCC_MISS_sum")
    if hits is not None and miss is not None and hits + miss > 0:
        out["l2_hit"] = hits / (hits + miss)
    if "TCC_ATOMIC_sum" in c and kernel_s > 0:
        out["l2_atomics_per_launch"] = c["TCC_ATOMIC_sum"]
        out["l2_atomic_rate"] = c["TCC_ATOMIC_sum"] / kernel_s
        out["l2_atomic_frac"] = out["l2_atomic_rate"] / L2_ATOMIC_PEAK
    if "fetch_bytes" in c and "write_bytes" in c and kernel_s > 0:
        t = c["fetch_bytes"] + c["write_bytes"]
        out["hbm_bytes_per_launch"] = t
        out["hbm_rate"] = t / kernel_s
        out["hbm_frac"] = t / kernel_s / HBM_PEAK_BPS
    return out


def issue_roofline(d: dict) -> dict:
    """The busier of the VALU and SALU issue pipes as the binding roofline."""
    cand = [(d[p]["frac"], p) for p in ("valu", "salu") if p in d]
    if not cand:
        return {}
    frac, pipe = max(cand)
    return {"bound": "alu", "pipe": pipe.upper(), "achieved": d[pipe]["rate"],
            "peak": ISSUE_PEAK, "unit": "wave-instructions/s", "frac": frac}


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
    c.add_argument("--stats-dir", default="",
                   help="a --kernel-trace --stats run of the same command: kernel durations")
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
    # kernel durations: a --kernel-trace --stats run of the same command
    # (counter passes serialise and slow the kernels), else the bench log
    kernel_ms = {}
    if a.stats_dir:
        for r in _csv(os.path.join(a.stats_dir, "run_kernel_stats.csv")):
            kernel_ms[short_name(r["Name"])] = float(r["AverageNs"]) / 1e6
    else:
        kernel_ms[kernel(6, bench["batch_stats"])] = bench["roofline"]["kernel_ms"]
        if "k5_batch" in bench:
            kernel_ms[kernel(5, bench["k5_batch"]["batch_stats"])] = bench["k5_batch"]["kernel_ms"]
    rec = {"source_sha256_16": source_hash(), "sources": list(KERNEL_SOURCES),
           "calibration": {"kernel": COPY_KERNEL + " (torch copy_ of %d MiB)" % a.copy_mib,
                           "bytes": copy_bytes, "FETCH_SIZE_KiB": cal["FETCH_SIZE"],
                           "WRITE_SIZE_KiB": cal["WRITE_SIZE"], "fetch_scale": fetch_scale,
                           "write_scale": write_scale},
           "commands": a.command,
           "kernels": {}}
    for kern, (wl, sub_) in sorted(per_launch.items()):
        m = means[kern]
        fb = m["FETCH_SIZE"] * 1024.0 * fetch_scale
        wb = m["WRITE_SIZE"] * 1024.0 * write_scale
        cm = dict(m)
        cm["fetch_bytes"], cm["write_bytes"] = fb, wb
        rec["kernels"][kern] = {"workload": wl, "dispatches": counts[kern], "fetch_bytes": fb,
                                "write_bytes": wb, "traffic_bytes": fb + wb,
                                "subgraphs_per_launch": sub_,
                                "kernel_ms": kernel_ms.get(kern),
                                "counters": cm}
    with open(a.out_json, "w") as f:
        json.dump(rec, f, indent=1)
        f.write("\n")

    kerns = sorted(k for k in means if k.startswith(("enum_kernel", "core_kernel"))) + [copy_key]
    lines = ["# " + a.title, "",
             "One rocprofv3 `--pmc` run per counter set (and one `--kernel-trace --stats` run "
             "for the durations), from /tmp with TMPDIR=/tmp; $R is the repository root:", "",
             "```"] + a.command + [
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
              "| kernel | workload | read (MB) | written (MB) | subgraphs | bytes / subgraph |",
              "|---|---|---:|---:|---:|---:|"]
    for kern, r in rec["kernels"].items():
        lines.append("| %s | %s | %.1f | %.1f | %.4g | %.3f |" % (
            kern, r["workload"], r["fetch_bytes"] / 1e6, r["write_bytes"] / 1e6,
            r["subgraphs_per_launch"], r["traffic_bytes"] / r["subgraphs_per_launch"]))
    lines += ["", "Derived per launch (issue peak %.4g wave-instructions/s per pipe = %d CUs x "
              "%.1f GHz x 1; HBM peak %.0f TB/s; L2 atomic peak %.4g/s = 128 channels x %.1f GHz):"
              % (ISSUE_PEAK, NUM_CUS, CLOCK_HZ / 1e9, HBM_PEAK_BPS / 1e12, L2_ATOMIC_PEAK,
                 CLOCK_HZ / 1e9), "",
              "| kernel | ms | VALU frac | SALU frac | LDS frac | lanes active | waves waiting | "
              "LDS bank-conflict / LDS-active | L2 hit | L2 atomics | atomic frac | HBM frac |",
              "|---|---:|---:|---:|---:|---:|---:|---:|---:|---:|---:|---:|"]
    for kern, r in rec["kernels"].items():
        ms = r["kernel_ms"] or float("nan")
        d = derived(r["counters"], ms / 1e3)
        g = lambda key: d.get(key, float("nan"))
        lines.append("| %s | %.3f | %.3f | %.3f | %.3f | %.3f | %.3f | %.3f | %.3f | %.4g | "
                     "%.4f | %.4f |" % (
                         kern, ms, d.get("valu", {}).get("frac", float("nan")),
                         d.get("salu", {}).get("frac", float("nan")),
                         d.get("lds", {}).get("frac", float("nan")), g("lane_util"),
                         g("wait_frac"), g("lds_conflict_frac"), g("l2_hit"),
                         g("l2_atomics_per_launch"), g("l2_atomic_frac"), g("hbm_frac")))
    with open(a.out_md, "w") as f:
        f.write("\n".join(lines) + "\n")


if __name__ == "__main__":
    main()
