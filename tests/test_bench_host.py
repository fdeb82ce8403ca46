"""Host-side checks of bench.py's contract and of its counter conversion (no GPU)."""
import csv
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

COLS = ["Correlation_Id", "Dispatch_Id", "Agent_Id", "Queue_Id", "Process_Id", "Thread_Id", "Grid_Size",
        "Kernel_Id", "Kernel_Name", "Workgroup_Size", "LDS_Block_Size", "Scratch_Size", "VGPR_Count",
        "Accum_VGPR_Count", "SGPR_Count", "Counter_Name", "Counter_Value", "Start_Timestamp", "End_Timestamp"]


def _write_run(d, counter, rows):
    os.makedirs(d, exist_ok=True)
    with open(os.path.join(d, "run_counter_collection.csv"), "w", newline="") as f:
        w = csv.writer(f)
        w.writerow(COLS)
        for i, (name, grid, value) in enumerate(rows):
            w.writerow([i + 1, i + 1, "Agent 1", 1, 1, 1, grid, 1, name, 256, 0, 0, 8, 0, 32, counter, value, 0, 1])


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2 and "one GPU" in r.stderr


def test_traffic_conversion_uses_the_calibration_copies_and_finest_sweep(tmp_path):
    """Calibration = the copy dispatches before the first solver kernel (a copy made
    by the solver itself must not count); the sweep is found under its current
    template name and its largest grid; bytes = KiB x 1024 x factor."""
    import bench
    gib = float(1 << 20)
    sweep = "void stk::k_p_sweep3c<double, 64, 16, false>(stk::Box, int, int, double const*)"
    coarse = "void stk::k_p_sweep3c<double, 64, 16, false>(stk::Box, int, int, double const*)"
    fetch = [("__amd_rocclr_copyBuffer", 131072, gib / 2.0)] * 3 + [
        ("void stk::k_pack(stk::Box)", 1000, 10.0),
        ("__amd_rocclr_copyBuffer", 131072, gib / 4.0),        # the solver's own copy
        (sweep, 524288, 300000.0), (sweep, 524288, 310000.0), (coarse, 32768, 5000.0)]
    write = [("__amd_rocclr_copyBuffer", 131072, gib)] * 3 + [
        ("void stk::k_pack(stk::Box)", 1000, 10.0),
        ("__amd_rocclr_copyBuffer", 131072, gib / 2.0),
        (sweep, 524288, 130000.0), (sweep, 524288, 130000.0), (coarse, 32768, 900.0)]
    _write_run(str(tmp_path / "f"), "FETCH_SIZE", fetch)
    _write_run(str(tmp_path / "w"), "WRITE_SIZE", write)
    out = str(tmp_path / "traffic.json")
    e = bench.traffic_from_counters(str(tmp_path / "f"), str(tmp_path / "w"), path=out)
    assert e["fetch_factor"] == pytest.approx(2.0) and e["write_factor"] == pytest.approx(1.0)
    assert e["dispatches"] == 2 and e["fetch_kib_per_dispatch"] == pytest.approx(305000.0)
    assert e["bytes_per_launch"] == pytest.approx(305000.0 * 1024 * 2.0 + 130000.0 * 1024)
    assert e["kernel_source_hash"] == bench.kernel_source_hash()
    assert json.load(open(out))["entries"]["1/256/0"]["bytes_per_launch"] == pytest.approx(e["bytes_per_launch"])


def test_side_legs_report_failures_without_losing_the_line():
    """A failing measurement leg becomes an error field; after a HIP error the
    later GPU legs are skipped and host-only legs still run."""
    import bench

    class HipFailure(Exception):
        status = -4

    legs = bench.Legs()
    assert legs.run("ok", lambda a, b: a + b, 2, 3) == 5
    r = legs.run("no convergence", lambda: (_ for _ in ()).throw(RuntimeError("solve did not converge")))
    assert r == {"error": "RuntimeError: solve did not converge"} and legs.gpu_ok
    r = legs.run("device", lambda: (_ for _ in ()).throw(HipFailure("launch failed")))
    assert r["error"].startswith("HipFailure") and not legs.gpu_ok
    assert "skipped" in legs.run("later gpu leg", lambda: 1)
    assert legs.run("host leg", lambda: 7, gpu=False) == 7
