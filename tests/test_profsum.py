"""The profile summariser's arithmetic on small hand-made rocprofv3 CSV
files (no GPU): per-dispatch means, the copy-kernel calibration of the
byte counters, and the traffic record bench.py reads."""

import csv
import json
import os

from paper_1804_09741_amd import profsum as P

HEADER = ["Correlation_Id", "Dispatch_Id", "Agent_Id", "Queue_Id", "Process_Id", "Thread_Id",
          "Grid_Size", "Kernel_Id", "Kernel_Name", "Workgroup_Size", "LDS_Block_Size",
          "Scratch_Size", "VGPR_Count", "Accum_VGPR_Count", "SGPR_Count", "Counter_Name",
          "Counter_Value", "Start_Timestamp", "End_Timestamp"]


def _pass(d, counter, rows):
    os.makedirs(d, exist_ok=True)
    with open(os.path.join(d, "run_counter_collection.csv"), "w", newline="") as f:
        w = csv.writer(f)
        w.writerow(HEADER)
        for disp, name, val in rows:
            w.writerow([disp, disp, "Agent 1", 1, 1, 1, 64, 1, name, 64, 0, 0, 8, 0, 16,
                        counter, val, 0, 1])


def test_counters_and_traffic_record(tmp_path):
    copy = "__amd_rocclr_copyBuffer"
    enum6 = "void mk::enum_kernel<6>(mk::DevGraph const*, int)"
    # a 1 MiB copy reads 512 KiB and writes 1024 KiB by the counters; a small
    # copy is ignored; two dispatches of the kernel, counters split in two rows
    _pass(tmp_path / "p1", "FETCH_SIZE", [(1, copy, 512.0), (2, copy, 1.0), (3, enum6, 100.0),
                                          (3, enum6, 100.0), (4, enum6, 600.0)])
    _pass(tmp_path / "p2", "WRITE_SIZE", [(1, copy, 1024.0), (3, enum6, 50.0), (4, enum6, 150.0)])
    bench = {"config": {"workload": "w6", "subgraphs_per_step": 1000},
             "roofline": {"kernel_ms": 2.0}, "batch_stats": {"method": 1}}
    log = tmp_path / "bench.log"
    log.write_text("[bench] noise\n" + json.dumps(bench) + "\n")
    out_md, out_json = tmp_path / "c.md", tmp_path / "t.json"
    P.main(["counters", str(tmp_path / "p1"), str(tmp_path / "p2"), "--copy-mib", "1",
            "--bench-log", str(log), "--out-md", str(out_md), "--out-json", str(out_json),
            "--command", "cmd"])
    rec = json.loads(out_json.read_text())
    assert rec["calibration"]["fetch_scale"] == 2.0 and rec["calibration"]["write_scale"] == 1.0
    k = rec["kernels"]["enum_kernel<6>"]
    assert k["dispatches"] == 2
    # mean FETCH_SIZE (200 + 600) / 2 = 400 KiB, x 2 -> 800 KiB; WRITE (50 + 150) / 2 = 100 KiB
    assert k["fetch_bytes"] == 800 * 1024 and k["write_bytes"] == 100 * 1024
    assert k["traffic_bytes"] == 900 * 1024
    assert k["subgraphs_per_launch"] == 1000 and k["kernel_ms"] == 2.0
    assert k["counters"]["fetch_bytes"] == 800 * 1024
    assert rec["source_sha256_16"] == P.source_hash()
    assert "| enum_kernel<6> | w6 |" in out_md.read_text()


def test_short_names():
    assert P.short_name("void mk::core_kernel<5>(mk::DevGraph const*, HIP_vector_type<int, 4u>)") \
        == "core_kernel<5>"
    assert P.short_name("mk::fill_kernel(unsigned int*, unsigned int, unsigned long)") == "fill_kernel"
    assert P.short_name("__amd_rocclr_copyBuffer") == "__amd_rocclr_copyBuffer"


def test_pmc_means_per_dispatch_and_unit(tmp_path):
    k7 = "void mk::k7_kernel<0>(mk::DevGraph const*, int)"
    other = "mk::fill_kernel(unsigned int*, unsigned int, unsigned long)"
    _pass(tmp_path / "p1", "SQ_INSTS_VALU", [(1, k7, 300.0), (1, k7, 100.0), (2, k7, 800.0),
                                             (3, other, 5.0)])
    _pass(tmp_path / "p2", "SQ_WAVES", [(1, k7, 64.0), (2, k7, 64.0), (3, other, 1.0)])
    out = tmp_path / "pmc.md"
    P.main(["pmc", str(tmp_path / "p1"), str(tmp_path / "p2"), "--kernels", "k7_kernel",
            "--out", str(out), "--command", "cmd", "--per", "k7_kernel<0>=200"])
    text = out.read_text()
    assert "k7_kernel<0>: 2 dispatches" in text and "fill_kernel" not in text
    # VALU: (400 + 800) / 2 = 600 per dispatch, 3 per unit of 200
    assert "| SQ_INSTS_VALU | 600 | 3 |" in text
    assert "| SQ_WAVES | 64 | 0.32 |" in text


def test_derived_rooflines():
    """Issue, lane, wait, L2 and HBM figures from counter means."""
    c = {"SQ_INSTS_VALU": P.ISSUE_PEAK * 1e-3 * 0.5, "SQ_INSTS_SALU": P.ISSUE_PEAK * 1e-3 * 0.25,
         "SQ_ACTIVE_INST_VALU": 100.0, "SQ_THREAD_CYCLES_VALU": 3200.0,
         "SQ_WAVE_CYCLES": 10.0, "SQ_WAIT_ANY": 4.0, "TCC_HIT_sum": 3.0, "TCC_MISS_sum": 1.0,
         "TCC_ATOMIC_sum": P.L2_ATOMIC_PEAK * 1e-3 * 0.1,
         "fetch_bytes": 4e9, "write_bytes": 4e9}
    d = P.derived(c, 1e-3)
    assert abs(d["valu"]["frac"] - 0.5) < 1e-12 and abs(d["salu"]["frac"] - 0.25) < 1e-12
    assert d["lane_util"] == 0.5 and d["wait_frac"] == 0.4 and d["l2_hit"] == 0.75
    assert abs(d["l2_atomic_frac"] - 0.1) < 1e-12
    assert abs(d["hbm_frac"] - 1.0) < 1e-12   # 8e9 bytes in 1 ms = 8 TB/s
    r = P.issue_roofline(d)
    assert r["bound"] == "alu" and r["pipe"] == "VALU" and abs(r["frac"] - 0.5) < 1e-12
