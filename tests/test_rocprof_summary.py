"""Host logic of the rocprofv3 summaries: per-dispatch means, the derived counter
figures and the copy-scaled traffic, on small hand-made counter files."""
import csv

import pytest

from paper_2306_11544_amd import rocprof_summary as rs


def _counters(path, rows):
    with open(path, "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"])
        w.writeheader()
        for d, k, c, v in rows:
            w.writerow({"Dispatch_Id": d, "Kernel_Name": k, "Counter_Name": c, "Counter_Value": v})


def _field(text, key):
    for line in text.splitlines():
        if line.startswith(key + ":"):
            return float(line.split(":", 1)[1].split()[0])
    raise KeyError(key)


def test_pmc_means_and_derived(tmp_path):
    a, b = tmp_path / "a.csv", tmp_path / "b.csv"
    # two dispatches of the kernel (one counter split over two rows, as per-XCD rows
    # are), one of another kernel that must be ignored
    _counters(a, [(1, "k_force_cells<0>", "SQ_INSTS_VALU", 600), (1, "k_force_cells<0>", "SQ_INSTS_VALU", 400),
                  (2, "k_force_cells<0>", "SQ_INSTS_VALU", 3000), (3, "k_bin", "SQ_INSTS_VALU", 1e9)])
    _counters(b, [(1, "k_force_cells<0>", "SQ_ACTIVE_INST_VALU", 100), (2, "k_force_cells<0>", "SQ_ACTIVE_INST_VALU", 100),
                  (1, "k_force_cells<0>", "SQ_THREAD_CYCLES_VALU", 3200), (2, "k_force_cells<0>", "SQ_THREAD_CYCLES_VALU", 3200)])
    out = rs.pmc([str(a), str(b)], "k_force_cells", ["cmd a", "cmd b"], candidates=6400)
    assert _field(out, "SQ_INSTS_VALU") == pytest.approx(2000.0)
    assert _field(out, "derived lane_utilisation") == pytest.approx(0.5)
    assert _field(out, "derived valu_lane_insts_per_candidate") == pytest.approx(2000 * 64 / 6400)
    assert _field(out, "derived active_valu_lane_insts_per_candidate") == pytest.approx(2000 * 64 / 6400 * 0.5)
    assert "command: cmd a" in out and "command: cmd b" in out


def test_pmc_without_candidates_has_no_per_candidate_line(tmp_path):
    a = tmp_path / "a.csv"
    _counters(a, [(1, "kk", "SQ_ACTIVE_INST_VALU", 10), (1, "kk", "SQ_THREAD_CYCLES_VALU", 640)])
    out = rs.pmc([str(a)], "kk", ["c"])
    assert _field(out, "derived lane_utilisation") == pytest.approx(1.0)
    assert "per_candidate" not in out


def test_last_dispatches_takes_the_latest_by_start_time(tmp_path):
    p = tmp_path / "trace.csv"
    with open(p, "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=["Kernel_Name", "Start_Timestamp", "End_Timestamp"])
        w.writeheader()
        # written out of order; durations 10, 20, 30, 40 us by start time, plus another kernel
        for start, dur in ((3000, 30), (1000, 10), (4000, 40), (2000, 20)):
            w.writerow({"Kernel_Name": "k_force_cells<0>", "Start_Timestamp": start * 1000,
                        "End_Timestamp": start * 1000 + dur * 1000})
        w.writerow({"Kernel_Name": "k_bin", "Start_Timestamp": 9_000_000, "End_Timestamp": 9_900_000})
    line = rs.last_dispatches(str(p), "k_force_cells", 2)
    assert "mean 35.000 us" in line and "min 30.000" in line and "max 40.000" in line
    with pytest.raises(SystemExit):
        rs.last_dispatches(str(p), "k_force_cells", 5)
