"""Host logic of bench.py (no GPU): the one-GPU guard, the HBM-counter
ingest (calibration scaling, post-convergence dispatches left out) and the
conditions under which the measured traffic is reported."""
import csv
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402

STENCIL = "void fit::stencil_kernel<double, 32, 8, 0, fit::OpCocgPX<double> >(fit::GridView)"
NEG = "void at::native::neg_kernel_cuda(float)"


def _csv(path, counter, rows):
    with open(path, "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"])
        w.writeheader()
        for i, (name, val) in enumerate(rows):
            w.writerow({"Dispatch_Id": i, "Kernel_Name": name, "Counter_Name": counter, "Counter_Value": val})


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_counter_ingest_scales_by_the_calibration_copy(tmp_path):
    copy_bytes = 1024 * 1000  # 1000 KiB each way
    # FETCH_SIZE reads half of the copy's bytes (scale 2); WRITE_SIZE is exact
    _csv(tmp_path / "f.csv", "FETCH_SIZE",
         [(STENCIL, 300.0), (STENCIL, 310.0), (STENCIL, 1.0), (NEG, 500.0), (NEG, 500.0)])
    _csv(tmp_path / "w.csv", "WRITE_SIZE", [(STENCIL, 200.0), (STENCIL, 200.0), (NEG, 1000.0)])
    info = {"copy_bytes_each_way": copy_bytes, "tile": [32, 8, 12]}
    for name in ("f.log", "w.log"):
        (tmp_path / name).write_text("noise\n" + json.dumps(info) + "\n")
    out = tmp_path / "traffic.json"
    bench.ingest_counters(str(tmp_path / "f.csv"), str(tmp_path / "w.csv"), str(tmp_path / "f.log"),
                          str(tmp_path / "w.log"), ["cmd"], out_path=str(out))
    t = json.loads(out.read_text())
    assert t["fetch_dispatches"] == 2  # the 1-KiB dispatch after convergence is left out
    assert t["fetch_scale"] == pytest.approx(2.0)
    assert t["write_scale"] == pytest.approx(1.0)
    assert t["fetch_bytes_per_launch"] == pytest.approx(305.0 * 1024 * 2.0)
    assert t["write_bytes_per_launch"] == pytest.approx(200.0 * 1024)
    assert t["tile"] == [32, 8, 12]
    assert t["kernel_source_hash"] == bench.kernel_source_hash()


def test_counter_runs_with_different_tiles_are_rejected(tmp_path):
    _csv(tmp_path / "f.csv", "FETCH_SIZE", [(STENCIL, 300.0), (NEG, 500.0)])
    _csv(tmp_path / "w.csv", "WRITE_SIZE", [(STENCIL, 200.0), (NEG, 1000.0)])
    (tmp_path / "f.log").write_text(json.dumps({"copy_bytes_each_way": 1024, "tile": [32, 8, 12]}) + "\n")
    (tmp_path / "w.log").write_text(json.dumps({"copy_bytes_each_way": 1024, "tile": [48, 8, 12]}) + "\n")
    with pytest.raises(SystemExit):
        bench.ingest_counters(str(tmp_path / "f.csv"), str(tmp_path / "w.csv"), str(tmp_path / "f.log"),
                              str(tmp_path / "w.log"), ["cmd"], out_path=str(tmp_path / "t.json"))


def test_traffic_is_reported_only_for_the_same_source_and_tile(tmp_path):
    p = tmp_path / "t.json"
    p.write_text(json.dumps({"kernel_source_hash": bench.kernel_source_hash(), "tile": [32, 8, 12],
                             "bytes_per_launch": 7.0e8}))
    assert bench.measured_traffic((32, 8, 12), str(p)) == 7.0e8
    assert bench.measured_traffic((48, 8, 12), str(p)) is None
    p.write_text(json.dumps({"kernel_source_hash": "0" * 16, "tile": [32, 8, 12], "bytes_per_launch": 7.0e8}))
    assert bench.measured_traffic((32, 8, 12), str(p)) is None
