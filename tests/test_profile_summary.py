"""The rocprofv3 summaries behind the bench's traffic and instruction figures
(host logic, synthetic CSV files in rocprofv3's column layout): the copy
calibration, and per-launch figures over the last N dispatches in dispatch
order (the event-timed pass at the end of a run)."""
import csv
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
K = "void tdh::stage_tiled<8, 8, 4, 6, 3, false, 256, 76>(tdh::StageArgs)"


def _write(path, header, rows):
    os.makedirs(os.path.dirname(path), exist_ok=True)
    with open(path, "w", newline="") as f:
        w = csv.writer(f, quoting=csv.QUOTE_NONNUMERIC)
        w.writerow(header)
        w.writerows(rows)


def _run(tmp_path, last):
    # six dispatches of the kernel, written out of dispatch order; durations
    # 1..6 ms and counters 10..60 follow the dispatch id
    ids = [4, 1, 6, 2, 5, 3]
    trace = tmp_path / "prof" / "run_kernel_trace.csv"
    _write(str(trace), ["Kind", "Dispatch_Id", "Kernel_Name", "Start_Timestamp", "End_Timestamp"],
           [["KERNEL_DISPATCH", i, K, 1000000 * i, 1000000 * i + 1000000 * i] for i in ids])
    _write(str(tmp_path / "prof" / "run_kernel_stats.csv"),
           ["Name", "Calls", "TotalDurationNs", "AverageNs", "Percentage", "MinNs", "MaxNs", "StdDev"],
           [[K, 6, 21e6, 3.5e6, 100.0, 1e6, 6e6, 0.0]])
    for cnt, d in (("FETCH_SIZE", "fetch"), ("WRITE_SIZE", "write")):
        _write(str(tmp_path / d / "run_counter_collection.csv"),
               ["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"],
               [[i, K, cnt, 10.0 * i] for i in ids])
        # the copy: 1 GiB moved, the counter reads 2^19 (fetch) or 2^20 (write) units
        _write(str(tmp_path / ("copy_" + d) / "run_counter_collection.csv"),
               ["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"],
               [[1, "__amd_rocclr_copyBuffer", cnt, float(1 << 19) if d == "fetch" else float(1 << 20)]])
    _write(str(tmp_path / "sq" / "run_counter_collection.csv"),
           ["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"],
           [[i, K, "SQ_INSTS_VALU", 100.0 * i] for i in ids])
    out_md, out_js = tmp_path / "s.md", tmp_path / "s.json"
    cmd = [sys.executable, "-m", "paper_2609_37859_amd.profile_summary", "--stats", str(tmp_path / "prof"),
           "--fetch", str(tmp_path / "fetch"), "--write", str(tmp_path / "write"),
           "--copy-fetch", str(tmp_path / "copy_fetch"), "--copy-write", str(tmp_path / "copy_write"),
           "--kernel", "stage_tiled", "--sq", str(tmp_path / "sq"), "--out", str(out_md), "--json", str(out_js),
           "--alg-bytes", "1e6"]
    if last:
        cmd += ["--last", str(last)]
    subprocess.run(cmd, check=True, cwd=ROOT, capture_output=True)
    return json.load(open(out_js)), open(out_md).read()


def test_copy_calibration_and_every_dispatch(tmp_path):
    js, md = _run(tmp_path, 0)
    assert js["fetch_factor"] == 2048.0 and js["write_factor"] == 1024.0
    assert js["avg_launch_ms"] == 3.5                      # from the stats file
    assert abs(js["hbm_read_bytes_per_launch"] - 35.0 * 2048) < 1e-9
    assert abs(js["hbm_write_bytes_per_launch"] - 35.0 * 1024) < 1e-9
    assert js["sq"]["SQ_INSTS_VALU"] == 350.0
    assert "Timed launches" not in md


def test_last_dispatches_in_dispatch_order(tmp_path):
    js, md = _run(tmp_path, 2)                             # dispatches 5 and 6
    assert js["avg_launch_ms"] == 5.5 and js["launches"] == 2 and js["avg_launch_ms_all"] == 3.5
    assert abs(js["hbm_read_bytes_per_launch"] - 55.0 * 2048) < 1e-9
    assert abs(js["hbm_write_bytes_per_launch"] - 55.0 * 1024) < 1e-9
    assert js["sq"]["SQ_INSTS_VALU"] == 550.0
    # traffic over the algorithmic bytes of those two launches
    assert abs(js["traffic_over_algorithmic"] - 2 * 55.0 * 3072 / 1e6) < 1e-12
    assert "the last 2 dispatches" in md
