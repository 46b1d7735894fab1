"""The profile condenser on small synthetic rocprofv3 CSV files: kernel statistics, HBM bytes
from FETCH_SIZE / WRITE_SIZE scaled by a calibration copy, and FP64 matrix-core work from
the MFMA counters."""
import csv

import pytest

from paper_1611_03189_amd import profile_summary as ps


def write_csv(path, rows):
    with open(path, "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=list(rows[0].keys()))
        w.writeheader()
        w.writerows(rows)


def counter_row(disp, name, counter, value, t0=0, t1=1000):
    return {"Dispatch_Id": str(disp), "Kernel_Name": name, "Counter_Name": counter,
            "Counter_Value": str(value), "Start_Timestamp": str(t0), "End_Timestamp": str(t1)}


def test_kernel_stats(tmp_path):
    p = tmp_path / "stats.csv"
    write_csv(p, [{"Name": "void hs::k_gemm<double, 64, 64, 16>(a, b)", "Calls": "4", "TotalDurationNs": "2000000",
                   "AverageNs": "500000", "Percentage": "50.0"}])
    out = ps.summarize(str(p), "cmd", "title")
    assert "# title" in out and "# command: cmd" in out
    line = [ln for ln in out.splitlines() if "k_gemm" in ln][0].split()
    assert line[-4:] == ["4", "2.00", "500.0", "50.00"]


def test_hbm_bytes_scaled_by_the_calibration_copy(tmp_path):
    f, w = tmp_path / "f.csv", tmp_path / "w.csv"
    # the copy of 1 MiB reads as 512 KiB fetched and 1024 KiB written: scales 2 and 1
    write_csv(f, [counter_row(1, "copy_kernel(x)", "FETCH_SIZE", 512.0), counter_row(2, "void hs::k_a(x)", "FETCH_SIZE", 10.0),
                  counter_row(3, "void hs::k_a(x)", "FETCH_SIZE", 30.0)])
    write_csv(w, [counter_row(1, "copy_kernel(x)", "WRITE_SIZE", 1024.0), counter_row(2, "void hs::k_a(x)", "WRITE_SIZE", 4.0),
                  counter_row(3, "void hs::k_a(x)", "WRITE_SIZE", 4.0)])
    res = ps.pmc_summary(str(f), str(w), "copy_kernel", 1048576.0)
    k = res["kernels"]["k_a"]
    assert k["fetch_kib"] == pytest.approx(20.0) and k["write_kib"] == pytest.approx(4.0)
    assert k["hbm_bytes"] == pytest.approx(20.0 * 1024 * 2 + 4.0 * 1024 * 1)


def test_mfma_rate_and_fraction(tmp_path):
    p = tmp_path / "m.csv"
    name = "void hs::k_gemm<double, 32, 32, 64>(t)"
    # two dispatches of 1 ms each; 78.6e9 / 512 MOPS per dispatch = 78.6 GFLOP each: 78.6 TFLOP/s
    mops = 78.6e9 / 512
    rows = []
    for d in (1, 2):
        rows += [counter_row(d, name, "SQ_INSTS_VALU_MFMA_MOPS_F64", mops, 0, 1000000),
                 counter_row(d, name, "SQ_VALU_MFMA_BUSY_CYCLES", 128.0 * 50, 0, 1000000),
                 counter_row(d, name, "GRBM_GUI_ACTIVE", 100.0, 0, 1000000)]
    rows.append(counter_row(3, "void hs::k_fill<double>(x)", "SQ_INSTS_VALU_MFMA_MOPS_F64", 0.0))
    write_csv(p, rows)
    out = ps.mfma_summary(str(p), "cmd")
    lines = [ln for ln in out.splitlines() if not ln.startswith("#")]
    assert len(lines) == 1                       # kernels without MFMA work are left out
    f = lines[0].split()
    assert f[-6:] == ["2.00", "157.20", "78.60", "1.0000", "64.000", "0.5000"]
