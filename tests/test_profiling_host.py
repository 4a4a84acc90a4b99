"""Host logic of the rocprofv3 summaries (CPU): per-kernel and per-grid trace statistics and the
HBM traffic scaled by a plain copy of known size, on small synthetic CSV files."""
import csv
import json
import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
from paper_1902_08112_amd import profiling  # noqa: E402


def _write_csv(path, header, rows):
    with open(path, "w", newline="") as f:
        w = csv.writer(f)
        w.writerow(header)
        w.writerows(rows)


def test_trace_stats_per_kernel_and_grid(tmp_path):
    trace = tmp_path / "kernel_trace.csv"
    rows = []
    t = 1000
    # k_a at two grids (the larger one is the finest level), k_b once; durations in ns
    for name, grid, dur in [("void pff::k_a<double, 1>(CellParams, int)", 4096, 30000),
                            ("void pff::k_a<double, 1>(CellParams, int)", 4096, 50000),
                            ("void pff::k_a<double, 1>(CellParams, int)", 512, 5000),
                            ("k_b", 256, 15000)]:
        rows.append([name, grid, 1, 1, t, t + dur])
        t += dur + 100
    _write_csv(trace, ["Kernel_Name", "Grid_Size_X", "Grid_Size_Y", "Grid_Size_Z", "Start_Timestamp",
                       "End_Timestamp"], rows)
    got = list(profiling.trace_rows(str(trace)))
    assert [g for _, g, _ in got] == [4096, 4096, 512, 256]
    assert got[0][0] == "k_a<double, 1>"
    assert got[0][2] == pytest.approx(30e-6)
    out = tmp_path / "summary.md"
    profiling.main(["stats", "--trace", str(trace), "--out", str(out), "--command", "cmd",
                    "--kernel", "k_a<double, 1>", "--kernel", "k_b"])
    text = out.read_text()
    assert "Kernel dispatches: 4, total kernel time 0.100 ms." in text
    assert ("Dominant kernel `k_a<double, 1>` at grid 4096: 2 dispatches, mean 40.00 us, median 40.00 us, "
            "min 30.00 us, max 50.00 us.") in text
    assert "Kernel `k_b` at grid 256: 1 dispatches, mean 15.00 us" in text
    assert "| `k_a<double, 1>` | 3 | 0.085 | 28.33 | 5.00 | 50.00 | 85.0 |" in text
    assert "| `k_a<double, 1>` | 512 | 1 | 0.005 | 5.00 | 5.0 |" in text
    assert "cmd" in text


def test_traffic_scaled_by_copy(tmp_path):
    header = ["Kernel_Name", "Grid_Size", "Counter_Name", "Counter_Value"]
    # the copy of 1 MiB reads as 512 KiB fetched (scale 2) and 1024 KiB written (scale 1)
    fetch_rows = [["k_x<double>", 4096, "FETCH_SIZE", v] for v in (100.0, 300.0, 200.0)]
    fetch_rows += [["__amd_rocclr_copyBuffer", 131072, "FETCH_SIZE", 512.0]] * 2
    fetch_rows += [["__amd_rocclr_copyBuffer", 64, "FETCH_SIZE", 1.0]]          # another grid: ignored
    fetch_rows += [["k_x<double>", 512, "FETCH_SIZE", 9999.0]]                    # a coarser level: ignored
    write_rows = [["k_x<double>", 4096, "WRITE_SIZE", 50.0]]
    write_rows += [["__amd_rocclr_copyBuffer", 131072, "WRITE_SIZE", 1024.0]]
    _write_csv(tmp_path / "f.csv", header, fetch_rows)
    _write_csv(tmp_path / "w.csv", header, write_rows)
    out = tmp_path / "t.json"
    profiling.main(["traffic", "--fetch", str(tmp_path / "f.csv"), "--write", str(tmp_path / "w.csv"),
                    "--kernel", "k_x<double>", "--grid", "4096", "--copy-kernel", "copyBuffer",
                    "--copy-grid", "131072", "--copy-bytes", str(1024 * 1024), "--algorithmic-bytes", "409600",
                    "--workload", "w", "--out", str(out), "--command", "cmd",
                    "--sources", "paper_1902_08112_amd/csrc/vec.hip"])
    rec = json.loads(out.read_text())
    assert rec["fetch_size"]["scale"] == pytest.approx(2.0)
    assert rec["fetch_size"]["bytes_per_launch"] == pytest.approx(200.0 * 1024 * 2)   # median of 100, 300, 200
    assert rec["write_size"]["scale"] == pytest.approx(1.0)
    assert rec["write_size"]["bytes_per_launch"] == pytest.approx(50.0 * 1024)
    assert rec["hbm_bytes_per_launch"] == pytest.approx(409600 + 51200)
    assert rec["traffic_over_algorithmic"] == pytest.approx((409600 + 51200) / 409600)
    assert rec["sources_sha"] == profiling.sources_sha(["paper_1902_08112_amd/csrc/vec.hip"])
    # without grids: the kernel's largest grid and the largest copy, as chosen above by hand
    out2 = tmp_path / "t2.json"
    profiling.main(["traffic", "--fetch", str(tmp_path / "f.csv"), "--write", str(tmp_path / "w.csv"),
                    "--kernel", "k_x<double>", "--copy-kernel", "copyBuffer", "--copy-bytes", str(1024 * 1024),
                    "--algorithmic-bytes", "409600", "--workload", "w", "--out", str(out2), "--command", "cmd",
                    "--sources", "paper_1902_08112_amd/csrc/vec.hip"])
    rec2 = json.loads(out2.read_text())
    assert rec2["grid"] == 4096
    assert rec2["hbm_bytes_per_launch"] == pytest.approx(rec["hbm_bytes_per_launch"])


def test_traffic_without_samples_fails(tmp_path):
    header = ["Kernel_Name", "Grid_Size", "Counter_Name", "Counter_Value"]
    _write_csv(tmp_path / "f.csv", header, [["k_y", 4096, "FETCH_SIZE", 1.0]])
    _write_csv(tmp_path / "w.csv", header, [["k_y", 4096, "WRITE_SIZE", 1.0]])
    with pytest.raises(SystemExit):
        profiling.main(["traffic", "--fetch", str(tmp_path / "f.csv"), "--write", str(tmp_path / "w.csv"),
                        "--kernel", "k_y", "--copy-kernel", "copyBuffer", "--copy-bytes", "1",
                        "--algorithmic-bytes", "1", "--workload", "w", "--out", str(tmp_path / "t.json"),
                        "--command", "cmd", "--sources", "paper_1902_08112_amd/csrc/vec.hip"])


def test_counters_means_and_sq_ratios(tmp_path):
    header = ["Kernel_Name", "Grid_Size", "Counter_Name", "Counter_Value"]
    rows = []
    for v in (1.0, 3.0):  # two dispatches at the finest grid
        rows += [["void pff::k_q<double, 0>(CellParams)", 4096, "SQ_WAVES", 10 * v],
                 ["void pff::k_q<double, 0>(CellParams)", 4096, "SQ_INSTS_VALU", 1000 * v],
                 ["void pff::k_q<double, 0>(CellParams)", 4096, "SQ_WAVE_CYCLES", 4000 * v],
                 ["void pff::k_q<double, 0>(CellParams)", 4096, "SQ_ACTIVE_INST_VALU", 1000 * v]]
    rows += [["void pff::k_q<double, 0>(CellParams)", 64, "SQ_WAVES", 1.0]]   # a coarser level: ignored
    _write_csv(tmp_path / "c.csv", header, rows)
    out = tmp_path / "c.md"
    profiling.main(["counters", "--csv", str(tmp_path / "c.csv"), "--kernel", "k_q<double, 0>",
                    "--out", str(out), "--command", "cmd"])
    text = out.read_text()
    assert "## `k_q<double, 0>` at grid 4096 (2 dispatches)" in text
    assert "| SQ_WAVES | 20 |" in text
    assert "| VALU instructions per wave | 100 |" in text
    assert "| VALU busy / lifetime | 0.25 |" in text
    assert "LDS instructions per wave" not in text
    # a kernel that did not run is noted; none at all is an error
    profiling.main(["counters", "--csv", str(tmp_path / "c.csv"), "--kernel", "k_q<double, 0>", "--kernel",
                    "k_missing", "--out", str(out), "--command", "cmd"])
    assert "No dispatches of `k_missing`." in out.read_text()
    with pytest.raises(SystemExit):
        profiling.main(["counters", "--csv", str(tmp_path / "c.csv"), "--kernel", "k_missing",
                        "--out", str(out), "--command", "cmd"])


def test_short_names_keep_namespaced_kernels():
    # a kernel in an unnamed namespace demangles with a parenthesis before its own name
    assert profiling.short("void pff::(anonymous namespace)::k_x<4, 8, 8>(pff::CellParams, int, double*)") == \
        "k_x<4, 8, 8>"
    assert profiling.short("void pff::k_q1_3d_slab<double, 0, false>(pff::CellParams, int)") == \
        "k_q1_3d_slab<double, 0, false>"
    assert profiling.short("__amd_rocclr_copyBuffer") == "__amd_rocclr_copyBuffer"
