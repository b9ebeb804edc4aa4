"""The profile summariser's arithmetic on synthetic rocprofv3 CSV rows (CPU):
per-kernel counter means with a KiB range, launch-shape tables and the
marker-range selection of timed launches."""
import csv
import os

import pytest

from paper_1709_00178_amd import profsum

COUNTER_FIELDS = ["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"]
TRACE_FIELDS = ["Kernel_Name", "Start_Timestamp", "End_Timestamp", "Grid_Size_X", "Workgroup_Size_X"]


def _write(path, fields, rows):
    with open(path, "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=fields)
        w.writeheader()
        for r in rows:
            w.writerow(r)


def test_kib_range():
    assert profsum.kib_range(":") == (0.0, float("inf"))
    assert profsum.kib_range("300000:") == (300000.0, float("inf"))
    assert profsum.kib_range("150000:200000") == (150000.0, 200000.0)
    assert profsum.kib_range(":10") == (0.0, 10.0)


def test_counter_means_keep_one_workload(tmp_path):
    d = tmp_path / "run_FETCH_SIZE"
    os.makedirs(d)
    rows = []
    # one kernel coding two shapes: 3 dispatches near 1000 KiB, 2 near 100 KiB
    for i, v in enumerate([1000.0, 1002.0, 998.0, 100.0, 104.0]):
        rows.append({"Dispatch_Id": i, "Kernel_Name": "k<1>", "Counter_Name": "FETCH_SIZE",
                     "Counter_Value": v})
    rows.append({"Dispatch_Id": 9, "Kernel_Name": "copy_kernel", "Counter_Name": "FETCH_SIZE",
                 "Counter_Value": 50.0})
    rows.append({"Dispatch_Id": 9, "Kernel_Name": "k<1>", "Counter_Name": "WRITE_SIZE",
                 "Counter_Value": 7.0})
    _write(d / "run_counter_collection.csv", COUNTER_FIELDS, rows)
    allm = profsum.counter_means(str(tmp_path), "FETCH_SIZE")
    assert allm["k<1>"] == (pytest.approx(640.8), 5)
    big = profsum.counter_means(str(tmp_path), "FETCH_SIZE", profsum.kib_range("500:"))
    assert big["k<1>"] == (pytest.approx(1000.0), 3) and "copy_kernel" not in big
    small = profsum.counter_means(str(tmp_path), "FETCH_SIZE", profsum.kib_range(":500"))
    assert small["k<1>"] == (pytest.approx(102.0), 2) and small["copy_kernel"] == (50.0, 1)
    (v, n), name = profsum.find(big, "k<")
    assert name == "k<1>" and n == 3
    with pytest.raises(SystemExit):
        profsum.find(small, "k")  # matches two kernel names


def test_grid_table_and_marked_launches(tmp_path):
    stats = tmp_path / "run_kernel_stats.csv"
    stats.write_text("Name,Calls,AverageNs,MinNs,MaxNs,Percentage\n")
    rows = [
        # two launch shapes of one kernel, in microseconds: 10, 12 and 100
        {"Kernel_Name": "k<1>", "Start_Timestamp": 0, "End_Timestamp": 10000,
         "Grid_Size_X": 64, "Workgroup_Size_X": 64},
        {"Kernel_Name": "k<1>", "Start_Timestamp": 20000, "End_Timestamp": 32000,
         "Grid_Size_X": 64, "Workgroup_Size_X": 64},
        {"Kernel_Name": "k<1>", "Start_Timestamp": 50000, "End_Timestamp": 150000,
         "Grid_Size_X": 4096, "Workgroup_Size_X": 256},
        {"Kernel_Name": "other", "Start_Timestamp": 0, "End_Timestamp": 5000,
         "Grid_Size_X": 64, "Workgroup_Size_X": 64},
    ]
    _write(tmp_path / "run_kernel_trace.csv", TRACE_FIELDS, rows)
    table = profsum.grid_table(str(stats), "k<").splitlines()
    assert len(table) == 4  # header, rule, one row per launch shape
    assert "| 64 | 64 | 2 | 11.0 | 11.0 | 10.0 | 12.0 |" in table[2]
    assert "| 4096 | 256 | 1 | 100.0 |" in table[3]
    _write(tmp_path / "run_marker_api_trace.csv", ["Function", "Start_Timestamp", "End_Timestamp"],
           [{"Function": "timed", "Start_Timestamp": 15000, "End_Timestamp": 200000}])
    d = profsum.marked_launches(str(stats), "timed", "k<1>")
    assert d == [12.0, 100.0]
