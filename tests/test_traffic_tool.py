"""The rocprofv3 counter post-processing (paper_1507_08101_amd/traffic.py) on hand-written
counter files: the copy probe calibrates bytes per counted KiB, the first dispatch of a
recurrence gets weight 1/steps, and the result is the calibrated read + write bytes."""
import csv
import json
import os

from paper_1507_08101_amd import traffic

HEAD = ["Correlation_Id", "Dispatch_Id", "Agent_Id", "Queue_Id", "Process_Id", "Thread_Id", "Grid_Size",
        "Kernel_Id", "Kernel_Name", "Workgroup_Size", "LDS_Block_Size", "Scratch_Size", "VGPR_Count",
        "Accum_VGPR_Count", "SGPR_Count", "Counter_Name", "Counter_Value", "Start_Timestamp", "End_Timestamp"]


def _write(d, counter, rows):
    os.makedirs(d, exist_ok=True)
    with open(os.path.join(d, "x_counter_collection.csv"), "w", newline="") as fh:
        w = csv.writer(fh)
        w.writerow(HEAD)
        for i, (name, v) in enumerate(rows):
            w.writerow([i, i, "Agent 1", 1, 1, 1, 1, 1, name, 512, 0, 0, 8, 0, 8, counter, v, 0, 1])


def test_traffic_from_counter_files(tmp_path):
    mib = 64
    kib = mib * 1024
    # copy probe: FETCH reads half the bytes (factor 2), WRITE reads them exactly
    _write(tmp_path / "cf", "FETCH_SIZE", [("copyBuffer", 5.0), ("sellcs::probe_copy_kernel", kib / 2)])
    _write(tmp_path / "cw", "WRITE_SIZE", [("sellcs::probe_copy_kernel", kib)])
    k = "prod_kernel<0, 8, 4, true>"
    _write(tmp_path / "f", "FETCH_SIZE", [("other", 1.0), (f"void sellcs::{k}(x)", 100.0)]
           + [(f"void sellcs::{k}(x)", 200.0)] * 3)
    _write(tmp_path / "w", "WRITE_SIZE", [(f"void sellcs::{k}(x)", 50.0)] * 4)
    out = tmp_path / "t.json"
    traffic.main(["--kernel", k, "--fetch", str(tmp_path / "f"), "--write", str(tmp_path / "w"),
                  "--copy-fetch", str(tmp_path / "cf"), "--copy-write", str(tmp_path / "cw"),
                  "--copy-mib", str(mib), "--steps", "10", "--algorithmic-bytes", "100000", "--hash", "abc",
                  "--out", str(out)])
    d = json.loads(out.read_text())
    assert d["copy_probe"]["fetch_scale"] == 2.0 and d["copy_probe"]["write_scale"] == 1.0
    fetch_kib = (100.0 + 9 * 200.0) / 10
    assert abs(d["read_bytes_per_launch"] - fetch_kib * 1024 * 2.0) < 1e-6
    assert abs(d["write_bytes_per_launch"] - 50.0 * 1024) < 1e-6
    assert abs(d["traffic_bytes_per_launch"] - (fetch_kib * 2048 + 51200)) < 1e-6
    assert d["kernel_source_hash"] == "abc" and d["kernel_KiB_per_dispatch"]["dispatches"] == 4
