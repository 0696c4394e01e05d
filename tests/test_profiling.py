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
