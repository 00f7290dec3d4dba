"""The rocprofv3 summaries behind profiles/: kernel names, per-launch HBM
traffic scaled by a copy kernel, counter averages and the derived MFMA-busy
and LDS-conflict figures, on small hand-written CSV files."""

import csv
import os

import pytest

from paper_2301_05844_amd import profiling

AGENT = ["Agent_Type", "Simd_Count", "Num_Xcc"]
COUNTER = ["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"]


def _write(path, header, rows):
    os.makedirs(os.path.dirname(path), exist_ok=True)
    with open(path, "w", newline="") as f:
        w = csv.writer(f, quoting=csv.QUOTE_ALL)
        w.writerow(header)
        w.writerows(rows)


def _run(tmp, name, rows):
    d = os.path.join(tmp, name)
    _write(os.path.join(d, "run_agent_info.csv"), AGENT, [["CPU", 0, 0], ["GPU", 1024, 8]])
    _write(os.path.join(d, "run_counter_collection.csv"), COUNTER, rows)
    return d


def test_short_name_keeps_template_arguments():
    n = "void bbp::(anonymous namespace)::k_visit4p<2, 2, double, 2>(bbp::VisitArgs)"
    assert profiling.short_name(n) == "k_visit4p<2, 2, double, 2>"


def test_traffic_scales_by_the_copy(tmp_path):
    k = "void bbp::k_visit4p<2, 2, double, 2>(bbp::VisitArgs)"
    # two dispatches of the kernel; counters split over two XCD rows each
    fetch = _run(str(tmp_path), "fetch", [[1, k, "FETCH_SIZE", 50], [1, k, "FETCH_SIZE", 50],
                                          [2, k, "FETCH_SIZE", 150], [2, k, "FETCH_SIZE", 150]])
    write = _run(str(tmp_path), "write", [[1, k, "WRITE_SIZE", 400], [2, k, "WRITE_SIZE", 600]])
    # the copy of 1 MiB reads FETCH_SIZE 512 KiB (0.5x) and WRITE_SIZE 1024 KiB (1x)
    cf = _run(str(tmp_path), "cf", [[1, "void copy(float*)", "FETCH_SIZE", 512]])
    cw = _run(str(tmp_path), "cw", [[1, "void copy(float*)", "WRITE_SIZE", 1024]])
    r = profiling.traffic("k_visit", "fit_visit", 2, fetch, write, cf, cw, 1 << 20, "")
    assert r["fetch_kib_per_dispatch"] == pytest.approx(200.0)
    assert r["write_kib_per_dispatch"] == pytest.approx(500.0)
    assert r["fetch_bytes_per_launch"] == pytest.approx(200.0 * 1024 / 0.5)
    assert r["write_bytes_per_launch"] == pytest.approx(500.0 * 1024)
    assert r["launches"] == 2


def test_counter_summary_and_derived_figures(tmp_path):
    k = "void bbp::k_env<2, double>(bbp::EnvArgs)"
    # GRBM_GUI_ACTIVE sums 8 XCDs: 8000 -> 1000 clocks; 1024 SIMDs -> 1.024e6
    # SIMD clocks, of which the MFMA units were busy 256000 (25%)
    p1 = _run(str(tmp_path), "p1", [[1, k, "GRBM_GUI_ACTIVE", 8000],
                                    [1, k, "SQ_VALU_MFMA_BUSY_CYCLES", 256000]])
    p2 = _run(str(tmp_path), "p2", [[1, k, "GRBM_GUI_ACTIVE", 8000],
                                    [1, k, "SQ_LDS_BANK_CONFLICT", 10],
                                    [1, k, "SQ_LDS_IDX_ACTIVE", 40]])
    md = profiling.counters_markdown([p1, p2], ["k_env"], "t", ["cmd"])
    assert "## `k_env<2, double>`" in md
    assert "| MFMA busy (derived) | 25.0% |" in md
    assert "| LDS bank-conflict share (derived) | 25.0% |" in md
    assert "1024 SIMDs in 8 XCDs" in md
