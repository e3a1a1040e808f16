"""Host logic of bench.py (CPU): the one-GPU guard, the traffic ingest and
its calibration, and the plan-info parsing."""

import csv
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def _write_counters(path, counter, rows):
    with open(path, "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=["Kernel_Name", "Counter_Name", "Counter_Value"])
        w.writeheader()
        for name, v in rows:
            w.writerow({"Kernel_Name": name, "Counter_Name": counter, "Counter_Value": v})


def test_traffic_ingest_scales_by_the_calibration_copy(tmp_path, monkeypatch):
    # a 1024 MiB copy reads FETCH = half its size and WRITE = its size: FETCH
    # is scaled by 2, WRITE by 1; each pass averages over its dispatches
    kib = 1024 * 1024.0
    fetch = [("__amd_rocclr_copyBuffer", kib / 2),
             ("fast2d::x_fwd_kernel(...)", 100.0), ("fast2d::x_fwd_kernel(...)", 300.0),
             ("fast2d::z_fused_kernel<1, true>(...)", 50.0),
             ("fast2d::x_inv_kernel(...)", 10.0)]
    write = [("__amd_rocclr_copyBuffer", kib),
             ("fast2d::x_fwd_kernel(...)", 40.0), ("fast2d::x_fwd_kernel(...)", 40.0),
             ("fast2d::z_fused_kernel<1, true>(...)", 5.0),
             ("fast2d::x_inv_kernel(...)", 1.0)]
    fcsv, wcsv = tmp_path / "f.csv", tmp_path / "w.csv"
    _write_counters(fcsv, "FETCH_SIZE", fetch)
    _write_counters(wcsv, "WRITE_SIZE", write)
    out = tmp_path / "traffic.json"
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(out))
    data = bench.ingest_traffic(str(fcsv), str(wcsv), 1, 1024)
    e = data["2d-4096x4096-sources-1000steps:x_r2c_fwd"]
    assert e["fetch_scale"] == pytest.approx(2.0) and e["write_scale"] == pytest.approx(1.0)
    assert e["bytes_per_launch"] == pytest.approx((200.0 * 2.0 + 40.0) * 1024.0)
    assert e["dispatches"] == 2
    assert e["source_hash"] == bench.kernel_source_hash()
    assert json.loads(out.read_text()) == data
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(out))
    assert bench.measured_traffic("2d-4096x4096-sources-1000steps", "z_fused") == \
        pytest.approx((50.0 * 2.0 + 5.0) * 1024.0)


def test_plan_grids_parses_the_plan_info():
    info = ("ndim=2 patches=1 solver=psatd precision=fp32 ...\n"
            "  x_r2c_fwd  items=5632 grid=5632 block=512 lds=1 mpt=0 ppt=0 lines=1 bytes=1 (autotuned)\n"
            "  z_fused    items=2048 grid=256 block=512 lds=1 mpt=0 ppt=0 lines=1 bytes=1\n")

    class P:
        pass
    p = P()
    p.info = info
    assert bench.plan_grids(p) == {"x_r2c_fwd": 5632, "z_fused": 256}


def test_kernel_names_map_to_passes():
    assert bench.pass_of_kernel("void psatd::line_pass_kernel<float, 0, 4>(psatd::PatchDev const*)") == "x_r2c_fwd"
    assert bench.pass_of_kernel("void psatd::line_pass_kernel<float, 3, 8>(...)") == "y_c2c_inv"
    assert bench.pass_of_kernel("void psatd::fused_z_kernel<float, 2, 0, 2>(...)") == "z_fused"
    assert bench.pass_of_kernel("psatd::fast2d::z_fused_kernel<1, true>(...)") == "z_fused"
    assert bench.pass_of_kernel("__amd_rocclr_copyBuffer") is None


def test_component_errors_use_coupled_sets():
    import numpy as np
    rng = np.random.default_rng(0)
    ref = [rng.normal(size=(8, 8)) * s for s in (1, 1e-3, 1, 1e-3, 1, 1e-3)]
    got = [r.copy() for r in ref]
    got[5] = got[5] * (1 + 1e-2)
    e = bench.component_errors(got, ref, 2)
    assert e["Bz"][0] > 5e-3 and e["Bz"][1] > 5e-3  # the s set is small as a whole
    assert e["Ex"] == (0.0, 0.0)
    e3 = bench.component_errors(got, ref, 3)
    assert e3["Bz"][1] < 1e-4  # in 3D the set is all six components
