"""Host logic of the measurement, without a GPU: the counter summaries (the
copy calibration, the per-class byte counts, the per-kernel counter table and
the limiter record) on small synthetic rocprofv3 CSV files, the bench's use of
the hash-stamped records, and its refusal of more than one GPU."""
import csv

from paper_2605_29598_amd import profiling as P

FIELDS = ["Correlation_Id", "Dispatch_Id", "Agent_Id", "Queue_Id", "Process_Id", "Thread_Id", "Grid_Size",
          "Kernel_Id", "Kernel_Name", "Workgroup_Size", "LDS_Block_Size", "Scratch_Size", "VGPR_Count",
          "Accum_VGPR_Count", "SGPR_Count", "Counter_Name", "Counter_Value", "Start_Timestamp", "End_Timestamp"]


def _csv(path, rows):
    with open(path, "w", newline="") as fh:
        w = csv.DictWriter(fh, fieldnames=FIELDS)
        w.writeheader()
        for i, (kernel, counter, value) in enumerate(rows):
            w.writerow({"Correlation_Id": i, "Dispatch_Id": i, "Agent_Id": "Agent 1", "Queue_Id": 1,
                        "Process_Id": 1, "Thread_Id": 1, "Grid_Size": 256, "Kernel_Id": 1,
                        "Kernel_Name": kernel, "Workgroup_Size": 256, "LDS_Block_Size": 1024,
                        "Scratch_Size": 0, "VGPR_Count": 64, "Accum_VGPR_Count": 0, "SGPR_Count": 32,
                        "Counter_Name": counter, "Counter_Value": value, "Start_Timestamp": 0,
                        "End_Timestamp": 1})
    return str(path)


def test_traffic_summary_scales_by_the_copy(tmp_path):
    copy = "void copy_kernel(double*)"
    # the probe copies 1 MiB: FETCH_SIZE reads 512 KiB (factor 2), WRITE_SIZE 1024 KiB (factor 1)
    cf = _csv(tmp_path / "cf.csv", [(copy, "FETCH_SIZE", 512.0), ("void small()", "FETCH_SIZE", 1.0)])
    cw = _csv(tmp_path / "cw.csv", [(copy, "WRITE_SIZE", 1024.0)])
    k1 = "void imx::k_mv2<5, double, false>(int const*)"
    k2 = "void imx::k_dots<double, 4, 7, false>(double const*)"
    f = _csv(tmp_path / "f.csv", [(k1, "FETCH_SIZE", 100.0), (k1, "FETCH_SIZE", 300.0), (k2, "FETCH_SIZE", 50.0)])
    w = _csv(tmp_path / "w.csv", [(k1, "WRITE_SIZE", 10.0), (k1, "WRITE_SIZE", 30.0), (k2, "WRITE_SIZE", 0.0)])
    rec = P.summarize(f, w, cf, cw, 1 << 20)
    assert rec["calibration"]["fetch_factor"] == 2.0 and rec["calibration"]["write_factor"] == 1.0
    assert rec["kernels"]["pass2"]["dispatches"] == 2
    assert rec["kernels"]["pass2"]["bytes_per_launch"] == 1024.0 * (2.0 * 200.0 + 20.0)
    assert rec["kernels"]["dots"]["bytes_per_launch"] == 1024.0 * 2.0 * 50.0
    assert rec["kernel_source_hash"] == P.kernel_source_hash()


def test_counter_table_means_per_kernel(tmp_path):
    k1 = "void imx::k_explicit_gc<5, double>(int const*, long)"
    k2 = "void imx::k_givens(double*)"
    a = _csv(tmp_path / "a.csv", [(k1, "SQ_WAVES", 10.0), (k1, "SQ_WAVES", 30.0), (k2, "SQ_WAVES", 1.0)])
    b = _csv(tmp_path / "b.csv", [(k1, "VALUBusy", 12.5)])
    t = P.counter_table([a, b], match="k_explicit")
    lines = t.splitlines()
    assert lines[0] == "| kernel | dispatches | VGPR | AGPR | SGPR | LDS B | WG | SQ_WAVES | VALUBusy |"
    assert len(lines) == 3
    assert lines[2] == "| `imx::k_explicit_gc<5, double>` | 2 | 64 | 0 | 32 | 1024 | 256 | 20 | 12.5 |"


def test_limiter_record_keeps_busy_fractions_and_waves(tmp_path):
    k1 = "void imx::k_mv1_gc<5, double, 2, true>(int const*)"
    k2 = "void imx::k_mv1_gc<5, float, 2, true>(int const*)"
    a = _csv(tmp_path / "a.csv", [(k1, "VALUBusy", 50.0), (k1, "VALUBusy", 60.0), (k1, "OccupancyPercent", 50.0),
                                  (k1, "SQ_WAVES", 7.0), (k2, "LdsUtil", 40.0)])
    rec = P.limiter_record([a], match="k_mv1", command="cmd")
    assert rec["kernel_source_hash"] == P.kernel_source_hash() and rec["command"] == "cmd"
    r1 = rec["kernels"]["imx::k_mv1_gc<5, double, 2, true>"]
    # the means per dispatch, 32 wave slots over 4 SIMDs, and no counter outside the limiter set
    assert r1["VALUBusy"] == 55.0 and r1["waves_per_simd"] == 4.0 and "SQ_WAVES" not in r1
    assert rec["kernels"]["imx::k_mv1_gc<5, float, 2, true>"] == {"dispatches": 1, "LdsUtil": 40.0}


def test_bench_reads_limiters_only_for_the_current_kernels(tmp_path, monkeypatch):
    import json
    import bench
    k = "void imx::k_mv2<5, double, false, true, true>(int const*)"
    a = _csv(tmp_path / "a.csv", [(k, "VALUBusy", 61.0), (k, "LdsUtil", 17.0)])
    rec = P.limiter_record([a])
    (tmp_path / "profiles").mkdir()
    path = tmp_path / "profiles" / "pmc_limiters_w.json"
    path.write_text(json.dumps(rec))
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    got = bench.measured_limiters("w", {"pass2": "k_mv2<"})
    assert got == {"pass2": {"kernel": "imx::k_mv2<5, double, false, true, true>", "VALUBusy": 61.0,
                             "LdsUtil": 17.0}}
    rec["kernel_source_hash"] = "0" * 16   # taken from other kernels: not used
    path.write_text(json.dumps(rec))
    assert bench.measured_limiters("w", {"pass2": "k_mv2<"}) is None


def test_bench_refuses_more_than_one_gpu():
    """The build runs on one GPU: bench.py --gpus N with N > 1 exits with a
    message instead of timing anything."""
    import json
    import os
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    r = subprocess.run([sys.executable, os.path.join(root, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120, cwd=root)
    assert r.returncode == 2
    assert "one GPU" in json.loads(r.stdout.strip().splitlines()[-1])["error"]
