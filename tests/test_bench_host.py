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
        w = csv.DictWriter(f, fieldnames=["Dispatch_Id", "Kernel_Name", "Grid_Size",
                                          "Counter_Name", "Counter_Value"])
        w.writeheader()
        for i, (name, grid, v) in enumerate(rows):
            w.writerow({"Dispatch_Id": i + 1, "Kernel_Name": name, "Grid_Size": grid,
                        "Counter_Name": counter, "Counter_Value": v})


def _run(kernels, early, late):
    """The calibration copy, then trial dispatches at plan time (other grids,
    value `early`), then six steps of the final plan."""
    return ([("__amd_rocclr_copyBuffer", 1, None)] + [(k, 7, early[k]) for k in kernels] * 3 +
            [(k, 9, late[k]) for k in kernels] * 6)


def test_traffic_ingest_scales_by_the_calibration_copy(tmp_path, monkeypatch):
    # a 1024 MiB copy reads FETCH = half its size and WRITE = its size: FETCH
    # is scaled by 2, WRITE by 1; only the final dispatches count (the
    # autotuner's trial launches come first), and a pass launched per length
    # sums its kernels
    kib = 1024 * 1024.0
    ks = ["wave2d::(anonymous namespace)::wave_x_kernel<0, 32>(...)",
          "wave2d::(anonymous namespace)::wave_x_kernel<0, 64>(...)",
          "wave2d::wave_z_fused_kernel<0>(...)",
          "wave2d::(anonymous namespace)::wave_x_kernel<1, 32>(...)",
          "wave2d::(anonymous namespace)::wave_x_kernel<1, 64>(...)"]
    fetch = _run(ks, {k: 999.0 for k in ks}, dict(zip(ks, (100.0, 300.0, 50.0, 10.0, 20.0))))
    write = _run(ks, {k: 999.0 for k in ks}, dict(zip(ks, (40.0, 40.0, 5.0, 1.0, 2.0))))
    fetch[0] = (fetch[0][0], 1, kib / 2)
    write[0] = (write[0][0], 1, kib)
    fcsv, wcsv = tmp_path / "f.csv", tmp_path / "w.csv"
    _write_counters(fcsv, "FETCH_SIZE", fetch)
    _write_counters(wcsv, "WRITE_SIZE", write)
    out = tmp_path / "traffic.json"
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(out))
    data = bench.ingest_traffic(str(fcsv), str(wcsv), 3, 1024)
    e = data["2d-256patches-64to512-vacuum-500steps:x_r2c_fwd"]
    assert e["fetch_scale"] == pytest.approx(2.0) and e["write_scale"] == pytest.approx(1.0)
    assert e["bytes_per_launch"] == pytest.approx(((100.0 + 300.0) * 2.0 + 80.0) * 1024.0)
    assert e["source_hash"] == bench.kernel_source_hash()
    assert json.loads(out.read_text()) == data
    assert bench.measured_traffic("2d-256patches-64to512-vacuum-500steps", "z_fused") == \
        pytest.approx((50.0 * 2.0 + 5.0) * 1024.0)
    assert bench.measured_traffic("2d-256patches-64to512-vacuum-500steps", "x_c2r_inv") == \
        pytest.approx((30.0 * 2.0 + 3.0) * 1024.0)


def test_traffic_ingest_sums_one_kernel_launched_at_several_grids(tmp_path, monkeypatch):
    # one kernel name serving several lengths (one launch per length, at its
    # own grid) counts once per launch, not averaged over its launches
    kib = 1024 * 1024.0
    z = "wave2d::wave_z_fused_kernel<0>(...)"
    zs = "wave2d::wave_z_set_kernel<0, 64>(...)"
    steps = [(z, 10, 100.0), (z, 20, 300.0), (zs, 30, 50.0)] * 4
    fetch = [("__amd_rocclr_copyBuffer", 1, kib / 2)] + steps
    write = [("__amd_rocclr_copyBuffer", 1, kib)] + [(n, g, v / 10) for n, g, v in steps]
    fcsv, wcsv = tmp_path / "f.csv", tmp_path / "w.csv"
    _write_counters(fcsv, "FETCH_SIZE", fetch)
    _write_counters(wcsv, "WRITE_SIZE", write)
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(tmp_path / "traffic.json"))
    data = bench.ingest_traffic(str(fcsv), str(wcsv), 3, 1024)
    e = data["2d-256patches-64to512-vacuum-500steps:z_fused"]
    assert e["bytes_per_launch"] == pytest.approx((450.0 * 2.0 + 45.0) * 1024.0)
    assert e["dispatches"] == 12


def test_final_dispatches_skip_the_autotuner_trials():
    rows = [("a", 1), ("b", 4), ("a", 2), ("b", 4), ("c", 5),   # trials
            ("a", 2), ("b", 3), ("c", 8), ("a", 2), ("b", 3), ("c", 8)]
    assert bench.final_dispatches(rows) == rows[5:]


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
    assert bench.pass_of_kernel("void psatd::ct::ct_line_kernel<float, 1, 96>(...)") == "x_c2r_inv"
    assert bench.pass_of_kernel("void psatd::wave2d::(anonymous namespace)::wave_x_kernel<0, 128>("
                                "psatd::PatchDev const*)") == "x_r2c_fwd"
    assert bench.pass_of_kernel("void psatd::wave2d::wave_z_fused_kernel<0>(...)") == "z_fused"
    assert bench.pass_of_kernel("void psatd::wave2d::(anonymous namespace)::wave_z3_fused_kernel<1>(...)") == "z_fused"
    assert bench.pass_of_kernel("void psatd::wave2d::wave_z_set_kernel<0, 256>(...)") == "z_fused"
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
