"""The rocprofv3 summaries behind the committed traffic record: the
calibration copy sets the scale, and each pass is counted at its most
frequent launch (the tuned schedule of the timed steps), not at the
autotuner's other candidates."""
import csv
import json

from paper_2106_03872_amd import profiling

FIELDS = ["Dispatch_Id", "Kernel_Name", "Grid_Size", "Counter_Name", "Counter_Value"]
XA = "void ks::xapply_kernel<96, ks::XShape<32, 256>, double, true, false>(int)"


def _write(d, counter, rows):
    d.mkdir(parents=True)
    with open(d / "run_counter_collection.csv", "w", newline="") as fh:
        w = csv.DictWriter(fh, fieldnames=FIELDS)
        w.writeheader()
        for i, (name, grid, value) in enumerate(rows):
            w.writerow({"Dispatch_Id": i, "Kernel_Name": name, "Grid_Size": grid, "Counter_Name": counter,
                        "Counter_Value": value})


def test_traffic_record_scales_and_picks_the_timed_launch(tmp_path):
    copy = "__amd_rocclr_copyBuffer"
    # small copies share the calibration copy's grid; the autotuner's other
    # candidate (grid 100) runs three times, the tuned launch (grid 200) five
    fetch = [(copy, 131072, 3.0), (copy, 131072, 524288.0), (copy, 131072, 524290.0)]
    fetch += [(XA, 100, 9.0e5)] * 3 + [(XA, 200, 1.0e6)] * 5
    write = [(copy, 131072, 7.0), (copy, 131072, 1048576.0), (copy, 131072, 1048576.0)]
    write += [(XA, 100, 4.0e6)] * 3 + [(XA, 200, 2.0e6)] * 5
    _write(tmp_path / "f", "FETCH_SIZE", fetch)
    _write(tmp_path / "w", "WRITE_SIZE", write)
    rec = profiling.traffic_record(str(tmp_path / "f"), str(tmp_path / "w"), 512, "cfg3_96")
    assert abs(rec["fetch_scale"] - 1048576.0 / 524289.0) < 1e-4
    assert rec["write_scale"] == 1.0
    k = rec["kernels"]["xapply"]
    assert (k["grid"], k["dispatches"]) == (200, 5)
    assert "XShape<32, 256>" in k["kernel"]
    assert k["bytes_per_launch"] == round((1.0e6 * 1048576.0 / 524289.0 + 2.0e6) * 1024)
    assert rec["csrc_sha256"] == profiling.csrc_fingerprint()
    json.dumps(rec)


def test_stats_table(tmp_path):
    p = tmp_path / "s.csv"
    with open(p, "w", newline="") as fh:
        w = csv.DictWriter(fh, fieldnames=["Name", "Calls", "TotalDurationNs", "AverageNs", "Percentage"])
        w.writeheader()
        w.writerow({"Name": XA, "Calls": 4, "TotalDurationNs": 6.0e6, "AverageNs": 1.5e6, "Percentage": 60.0})
        w.writerow({"Name": "ks::dots_kernel(int)", "Calls": 2, "TotalDurationNs": 4.0e6, "AverageNs": 2.0e6,
                    "Percentage": 40.0})
    t = profiling.stats_table(str(p)).splitlines()
    assert t[2].startswith("| `xapply_kernel<96, XShape<32, 256>, double, true, false>` | 4 | 6.000 | 1500.00")
    assert "dots_kernel" in t[3]


def _write_counters(d, rows):
    """rows: (kernel, grid, counter, value) -> run_counter_collection.csv in d."""
    d.mkdir(parents=True)
    with open(d / "run_counter_collection.csv", "w", newline="") as fh:
        w = csv.DictWriter(fh, fieldnames=FIELDS)
        w.writeheader()
        for i, (name, grid, counter, value) in enumerate(rows):
            w.writerow({"Dispatch_Id": i, "Kernel_Name": name, "Grid_Size": grid, "Counter_Name": counter,
                        "Counter_Value": value})


GP = "void ks::(anonymous namespace)::gproj_gemm_kernel<float>(float const*, long long, int)"


def test_mfma_table_busy_fraction_and_flops(tmp_path):
    c = {"SQ_INSTS_MFMA": 100.0, "SQ_INSTS_VALU_MFMA_MOPS_BF16": 1000.0, "SQ_VALU_MFMA_BUSY_CYCLES": 1024 * 50.0,
         "GRBM_GUI_ACTIVE": 8 * 200.0, "SQ_LDS_BANK_CONFLICT": 30.0, "SQ_INSTS_LDS": 10.0}
    rows = [(GP, 4096, k, v) for k, v in c.items()] * 2
    rows += [(XA, 100, "SQ_INSTS_MFMA", 0.0)]                     # no matrix work: left out
    _write_counters(tmp_path / "m", rows)
    t = profiling.mfma_table(str(tmp_path / "m"), model_flops=512000.0).splitlines()
    assert len(t) == 3
    assert t[2] == "| `gproj_gemm_kernel<float>` | 2 | 5.12e+05 | 5.12e+05 | 0.250 | 3.00 |  |"


def test_mfma_table_clock_from_dispatch_time(tmp_path):
    """The clock column: GRBM_GUI_ACTIVE per XCD over the dispatch's duration
    (1600 active cycles summed over 8 XCDs in 100 ns: 2 GHz)."""
    d = tmp_path / "c"
    d.mkdir()
    names = FIELDS + ["Start_Timestamp", "End_Timestamp"]
    c = {"SQ_INSTS_MFMA": 1.0, "SQ_VALU_MFMA_BUSY_CYCLES": 1024.0, "GRBM_GUI_ACTIVE": 1600.0,
         "SQ_LDS_BANK_CONFLICT": 0.0, "SQ_INSTS_LDS": 1.0}
    with open(d / "run_counter_collection.csv", "w", newline="") as fh:
        w = csv.DictWriter(fh, fieldnames=names)
        w.writeheader()
        for disp, (t0, t1) in enumerate(((1000, 1100), (5000, 5080))):
            for k, v in c.items():
                w.writerow({"Dispatch_Id": disp, "Kernel_Name": GP, "Grid_Size": 4096, "Counter_Name": k,
                            "Counter_Value": v, "Start_Timestamp": t0, "End_Timestamp": t1})
    t = profiling.mfma_table(str(d)).splitlines()
    assert t[2].endswith("| 2.25 |")                        # mean of 2.0 and 2.5 GHz


def test_waves_table_fractions(tmp_path):
    c = {"SQ_WAVE_CYCLES": 1000.0, "SQ_ACTIVE_INST_ANY": 300.0, "SQ_WAIT_ANY": 500.0, "SQ_WAIT_INST_ANY": 200.0,
         "SQ_ACTIVE_INST_VALU": 150.0, "SQ_ACTIVE_INST_LDS": 80.0, "SQ_LDS_BANK_CONFLICT": 50.0, "SQ_INSTS_LDS": 100.0}
    _write_counters(tmp_path / "s", [(XA, 200, k, v) for k, v in c.items()])
    t = profiling.waves_table([str(tmp_path / "s")]).splitlines()
    assert t[2] == "| `xapply_kernel<96, XShape<32, 256>, double, true, false>` | 0.300 | 0.500 | 0.200 | 0.150 | 0.080 | 0.500 |"
    # a name filter picks the complex64 instantiation of a mixed run, even
    # where the FP64 one has more dispatches
    xf = XA.replace("double", "float")
    rows = [(XA, 200, k, v) for k, v in c.items()] * 3 + [(xf, 200, k, v / 2 if k == "SQ_WAIT_ANY" else v)
                                                           for k, v in c.items()]
    rows = [(n.replace("(int)", "(int, double, float)"), g, k, v) for n, g, k, v in rows]   # parameters do not match
    _write_counters(tmp_path / "m", rows)
    t = profiling.waves_table([str(tmp_path / "m")], match=", float,").splitlines()
    assert len(t) == 3 and t[2].startswith("| `xapply_kernel<96, XShape<32, 256>, float, true, false>` | 0.300 | 0.250 |")
    t = profiling.waves_table([str(tmp_path / "m")], match=", double,").splitlines()
    assert len(t) == 3 and t[2].startswith("| `xapply_kernel<96, XShape<32, 256>, double, true, false>` | 0.300 | 0.500 |")


def test_durations_split_and_kernel_traffic(tmp_path):
    p = tmp_path / "trace.csv"
    with open(p, "w", newline="") as fh:
        w = csv.DictWriter(fh, fieldnames=["Dispatch_Id", "Kernel_Name", "Start_Timestamp", "End_Timestamp"])
        w.writeheader()
        w.writerow({"Dispatch_Id": 1, "Kernel_Name": GP, "Start_Timestamp": 0, "End_Timestamp": 2000})
        w.writerow({"Dispatch_Id": 2, "Kernel_Name": GP, "Start_Timestamp": 0, "End_Timestamp": 4000})
        w.writerow({"Dispatch_Id": 3, "Kernel_Name": "void ks::xapply_kernel<120, x>(int)", "Start_Timestamp": 0,
                    "End_Timestamp": 1})
        w.writerow({"Dispatch_Id": 4, "Kernel_Name": GP, "Start_Timestamp": 0, "End_Timestamp": 9000})
    t = profiling.durations_table(str(p), "gproj", "<120", ("small", "large")).splitlines()
    assert t[2] == "| large | `gproj_gemm_kernel<float>` | 1 | 9.0 | 9.0 | 9.0 |"
    assert t[3] == "| small | `gproj_gemm_kernel<float>` | 2 | 3.0 | 2.0 | 4.0 |"
    _write_counters(tmp_path / "f", [(GP, 4096, "FETCH_SIZE", 100.0)])
    _write_counters(tmp_path / "w", [(GP, 4096, "WRITE_SIZE", 50.0)])
    rec = tmp_path / "rec.json"
    rec.write_text(json.dumps({"fetch_scale": 2.0, "write_scale": 1.0}))
    t = profiling.kernel_traffic_table(str(tmp_path / "f"), str(tmp_path / "w"), "gproj", str(rec)).splitlines()
    assert t[2] == f"| `gproj_gemm_kernel<float>` | 1 | 100 | 50 | {(100 * 2 + 50) * 1024 / 1e6:.1f} |"
