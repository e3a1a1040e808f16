"""GPU parity: the HIP path against the FP64 oracle on the same seeded inputs.

Tolerances (relative L2 over E and B):
  FP64 storage   1e-12 (the FP64 oracle target)
  FP32 storage   1e-5  (the FP32 target).  The FP32 path rounds to FP32 when
                 it stores to HBM, so the inputs the oracle sees are the same
                 FP32-rounded arrays, upcast.
Sizes span several tiles and ragged tails (line counts not multiples of the
tile, radix-3 factors, length-1 x transforms).
"""

import numpy as np
import pytest

import fixtures
from gpu_support import compare, fields_to_device, from_device, run_gpu, run_oracle, say

pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-12, "fp32": 1e-5}


def _w(index, shape, steps):
    return fixtures.workload(index, shape=shape, steps=steps)


# ----------------------------------------------------------------- workload 0, full size
@pytest.mark.parametrize("precision,path", [("fp64", "plain"), ("fp64", "fused"),
                                            ("fp32", "fused"), ("fp32", "plain")])
def test_workload0_vacuum_128(precision, path):
    w = fixtures.workload(0)
    say(f"workload0 {precision} {path} 128x128 x {w.steps} steps")
    err = compare(run_gpu(w, precision, path, w.steps), run_oracle(w, precision, w.steps),
                  precision=precision)
    assert err < TOL[precision]


# ----------------------------------------------------------------- 2D, sources, ragged
SHAPES_2D = [(48, 64), (6, 8), (12, 18), (18, 12), (96, 64), (64, 96), (2, 4), (4, 2), (36, 24)]


@pytest.mark.parametrize("shape", SHAPES_2D)
@pytest.mark.parametrize("precision,path", [("fp64", "plain"), ("fp64", "fused"),
                                            ("fp32", "fused")])
def test_2d_sources_rho(shape, precision, path):
    w = _w(1, shape, 6)
    say(f"2d rho {shape} {precision} {path}")
    err = compare(run_gpu(w, precision, path, w.steps), run_oracle(w, precision, w.steps),
                  precision=precision)
    assert err < TOL[precision]


@pytest.mark.parametrize("shape", [(48, 64), (12, 18)])
@pytest.mark.parametrize("precision,path", [("fp64", "plain"), ("fp32", "fused")])
def test_2d_sources_jform(shape, precision, path):
    w = _w(1, shape, 5)
    say(f"2d J-form {shape} {precision} {path}")
    err = compare(run_gpu(w, precision, path, w.steps, form="J"),
                  run_oracle(w, precision, w.steps, form="J"),
                  precision=precision)
    assert err < TOL[precision]


# ----------------------------------------------------------------- 3D
SHAPES_3D = [(8, 6, 12), (12, 8, 18), (16, 16, 16), (6, 12, 8)]


@pytest.mark.parametrize("shape", SHAPES_3D)
@pytest.mark.parametrize("precision,path", [("fp64", "plain"), ("fp64", "fused"),
                                            ("fp32", "fused")])
def test_3d_sources_rho(shape, precision, path):
    w = _w(2, shape, 4)
    say(f"3d rho {shape} {precision} {path}")
    err = compare(run_gpu(w, precision, path, w.steps), run_oracle(w, precision, w.steps),
                  precision=precision)
    assert err < TOL[precision]


@pytest.mark.parametrize("precision,path", [("fp64", "plain"), ("fp32", "fused")])
def test_3d_vacuum_plane_waves(precision, path):
    w = fixtures.workload(4, shape=(16, 24, 32), steps=6)
    w.sources = False
    say(f"3d vacuum packets {precision} {path}")
    err = compare(run_gpu(w, precision, path, w.steps), run_oracle(w, precision, w.steps),
                  precision=precision)
    assert err < TOL[precision]


@pytest.mark.parametrize("order", [2, 8, 128])
def test_order_p(order):
    w = _w(1, (32, 48), 4)
    say(f"order {order}")
    err = compare(run_gpu(w, "fp64", "plain", w.steps, order=order),
                  run_oracle(w, "fp64", w.steps, order=order), precision="fp64")
    assert err < TOL["fp64"]


# ----------------------------------------------------------------- radix-4 line passes
# PSATD_FLAG_RADIX4_LINES: the generic line passes as radix-4 (then radix-2 and
# radix-3) stages at 4 points per thread; lengths with radix-3 factors, odd
# powers of two and length-1 x transforms included.
@pytest.mark.parametrize("index,shape", [(1, (12, 18)), (1, (36, 24)), (1, (96, 64)), (1, (2, 4)),
                                         (1, (64, 96)), (2, (12, 8, 18)), (2, (16, 16, 16)),
                                         (2, (6, 12, 8))])
@pytest.mark.parametrize("precision,path", [("fp64", "plain"), ("fp64", "fused"),
                                            ("fp32", "fused")])
def test_radix4_line_passes(index, shape, precision, path):
    w = _w(index, shape, 3)
    say(f"radix-4 lines {shape} {precision} {path}")
    err = compare(run_gpu(w, precision, path, w.steps, radix4_lines=True),
                  run_oracle(w, precision, w.steps),
                  precision=precision)
    assert err < TOL[precision]


def test_radix4_line_passes_batched():
    w = fixtures.workload(3, npatches=24, steps=3)
    err = compare(run_gpu(w, "fp32", "fused", w.steps, radix4_lines=True),
                  run_oracle(w, "fp32", w.steps))
    assert err < TOL["fp32"]


# ----------------------------------------------------------------- fused modes per thread
# An untuned plan takes the smallest compiled modes-per-thread count whose
# workgroup holds the z lines: long z lines fall back to the larger counts.
@pytest.mark.parametrize("index,shape,mpt", [
    (1, (1024, 8), 2), (1, (2048, 8), 4), (1, (4096, 4), 8), (1, (1536, 6), 4),
    (2, (1024, 2, 4), 2), (2, (2048, 2, 4), 4), (2, (1536, 4, 2), 4)])
def test_fused_modes_per_thread_fallbacks(index, shape, mpt):
    import paper_1608_05739_amd as pk
    w = _w(index, shape, 2)
    plan = pk.Plan(w.patches, precision="fp32", source_mode="rho", path="fused")
    info = plan.info
    plan.close()
    assert f"mpt={mpt} " in info, info
    say(f"fused fp32 {shape}: mpt={mpt}")
    err = compare(run_gpu(w, "fp32", "fused", w.steps), run_oracle(w, "fp32", w.steps))
    assert err < TOL["fp32"]


# ----------------------------------------------------------------- fused plans, long z lines
# z lines longer than a workgroup of the fused pass holds: the fused plan runs
# the plain z passes (transform, update, transform) for them instead.
@pytest.mark.parametrize("index,shape,precision", [
    (1, (4096, 4), "fp64"), (1, (3072, 6), "fp64"), (2, (4096, 2, 4), "fp32"),
    (2, (2048, 2, 2), "fp64")])
def test_fused_plan_with_too_long_z_lines_runs_plain_z_passes(index, shape, precision):
    import paper_1608_05739_amd as pk
    w = _w(index, shape, 3)
    plan = pk.Plan(w.patches, precision=precision, source_mode="rho", path="fused")
    info = plan.info
    plan.close()
    assert "update" in info and "z_fused" not in info, info
    say(f"fused {precision} {shape}: plain z passes")
    err = compare(run_gpu(w, precision, "fused", w.steps), run_oracle(w, precision, w.steps),
                  precision=precision)
    assert err < TOL[precision]


# the radix-4 option keeps the default schedule for lines over 2048 points
@pytest.mark.parametrize("shape,precision,path", [((4096, 4), "fp32", "plain"),
                                                  ((4, 4096), "fp64", "plain"),
                                                  ((4096, 8), "fp32", "fused")])
def test_radix4_option_with_4096_point_lines(shape, precision, path):
    w = _w(1, shape, 3)
    say(f"radix-4 option {shape} {precision} {path}")
    err = compare(run_gpu(w, precision, path, w.steps, radix4_lines=True),
                  run_oracle(w, precision, w.steps), precision=precision)
    assert err < TOL[precision]


# ----------------------------------------------------------------- compile-time line tiles
# Tiles of the compile-time line kernels stay inside one run of the tile map
# (z in 2D x passes, y in 3D x passes, z in y passes): where the tile does not
# divide that run, its last tile is shorter.
@pytest.mark.parametrize("index,shape", [(1, (96, 128)), (1, (48, 96)), (2, (48, 96, 64)),
                                         (2, (18, 12, 64)), (2, (24, 32, 96))])
@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_compile_time_line_tiles_split_at_the_tile_map(index, shape, precision):
    import paper_1608_05739_amd as pk
    w = _w(index, shape, 3)
    plan = pk.Plan(w.patches, precision=precision, source_mode="rho", path="fused")
    info = plan.info
    plan.close()
    # (FP32 plans take the wave-resident x passes, and a 3D FP32 plan shows
    # the compile-time kernels only in y passes of a compiled length; FP64
    # plans show them in the x passes)
    want = "kernel=wave" if precision == "fp32" else "kernel=compile-time"
    assert want in info, info
    say(f"compile-time tiles {shape} {precision}")
    err = compare(run_gpu(w, precision, "fused", w.steps), run_oracle(w, precision, w.steps),
                  precision=precision)
    assert err < TOL[precision]


# ----------------------------------------------------------------- wave-resident x passes
# 2D FP32 plans run the x passes as wave-resident transforms over tiles of
# consecutive rows; every compiled row length nx / 2, row counts that leave a
# partial last tile, both paths, with sources.
@pytest.mark.parametrize("shape", [(36, 64), (18, 96), (24, 128), (12, 192), (54, 256),
                                   (6, 384), (72, 512), (6, 768), (18, 1024), (12, 2048)])
@pytest.mark.parametrize("path", ["fused", "plain"])
def test_wave_x_passes_every_row_length(shape, path):
    import paper_1608_05739_amd as pk
    w = _w(1, shape, 3)
    plan = pk.Plan(w.patches, precision="fp32", source_mode="rho", path=path)
    info = plan.info
    plan.close()
    assert info.count("kernel=wave") >= 2, info
    say(f"wave x passes {shape} fp32 {path}")
    err = compare(run_gpu(w, "fp32", path, w.steps), run_oracle(w, "fp32", w.steps))
    assert err < TOL["fp32"]


# ----------------------------------------------------------------- wave-resident 3D y passes
# 3D FP32 plans with y lines of a compiled length run the y passes as
# wave-resident transforms over tiles of consecutive z of one kx; every
# compiled y length, z counts that leave a partial last tile.
@pytest.mark.parametrize("shape", [(36, 32, 8), (18, 48, 12), (24, 64, 6), (12, 96, 4),
                                   (24, 128, 4), (6, 192, 4), (18, 256, 2), (6, 384, 2),
                                   (12, 512, 2), (6, 1024, 2)])
def test_wave_y_passes_every_line_length(shape):
    import paper_1608_05739_amd as pk
    w = _w(2, shape, 3)
    plan = pk.Plan(w.patches, precision="fp32", source_mode="rho", path="fused")
    info = plan.info
    plan.close()
    ylines = [ln for ln in info.splitlines() if ln.strip().startswith("y_c2c")]
    assert len(ylines) == 2 and all(ln.endswith("kernel=wave") for ln in ylines), info
    say(f"wave y passes {shape}")
    err = compare(run_gpu(w, "fp32", "fused", w.steps), run_oracle(w, "fp32", w.steps))
    assert err < TOL["fp32"]


# ----------------------------------------------------------------- wave-resident 3D z pass
# 3D FP32 fused plans with z lines of 32 to 512 points run the wave-resident z
# pass (outputs accumulated input by input); every compiled length, line
# counts that leave a partial last item, all three PSATD forms.
@pytest.mark.parametrize("shape", [(32, 6, 12), (64, 4, 8), (128, 2, 6), (256, 2, 4),
                                   (512, 4, 2)])
@pytest.mark.parametrize("form", ["rho", "J", "vacuum"])
def test_wave_z3_every_length_and_form(shape, form):
    import paper_1608_05739_amd as pk
    if form == "vacuum":
        w = fixtures.workload(4, shape=shape, steps=4)
        w.sources = False
    else:
        w = _w(2, shape, 4)
    mode = {"rho": "rho", "J": "j", "vacuum": "vacuum"}[form]
    plan = pk.Plan(w.patches, precision="fp32", source_mode=mode, path="fused")
    info = plan.info
    plan.close()
    assert [ln for ln in info.splitlines() if "z_fused" in ln][0].endswith("kernel=wave"), info
    say(f"wave z 3d {shape} {form}")
    err = compare(run_gpu(w, "fp32", "fused", w.steps, form=form if form != "vacuum" else "rho"),
                  run_oracle(w, "fp32", w.steps, form=form if form != "vacuum" else "rho"))
    assert err < TOL["fp32"]


# ----------------------------------------------------------------- batched patches
def test_batched_patches_workload3_subset():
    w = fixtures.workload(3, npatches=24, steps=3)
    say(f"batched 24 patches, {w.cells} cells")
    for precision, path in (("fp32", "fused"), ("fp64", "plain")):
        err = compare(run_gpu(w, precision, path, w.steps), run_oracle(w, precision, w.steps),
                  precision=precision)
        assert err < TOL[precision]


def test_batched_patch_equals_patch_alone():
    w = fixtures.workload(3, npatches=6, steps=2)
    E_all, B_all = run_gpu(w, "fp32", "fused", 2)
    for p in (0, 3, 5):
        Ep, Bp = run_gpu(w, "fp32", "fused", 2, patches=[w.patches[p]], E0=[w.E0[p]], B0=[w.B0[p]],
                         schedule=[None])
        for c in range(3):
            assert np.array_equal(E_all[p][c], Ep[0][c])
            assert np.array_equal(B_all[p][c], Bp[0][c])


# ----------------------------------------------------------------- graph replay
def test_graph_replay_equals_eager():
    w = fixtures.workload(0, steps=10)
    a = run_gpu(w, "fp32", "fused", 10, graph=False)
    b = run_gpu(w, "fp32", "fused", 10, graph=True)
    for pa, pb in zip(a[0] + a[1], b[0] + b[1]):
        for x, y in zip(pa, pb):
            assert np.array_equal(x, y)


def test_graph_with_parallel_length_launches_equals_eager():
    # a batch of patches of several sizes: the graph runs the per-length
    # launches of each pass as parallel branches
    import paper_1608_05739_amd as pk
    w = fixtures.workload(3, npatches=24, steps=6)
    plan = pk.Plan(w.patches, precision="fp32", source_mode="vacuum", path="fused")
    info = plan.info
    plan.close()
    assert "kernel=wave" in info, info
    a = run_gpu(w, "fp32", "fused", 6, graph=False)
    b = run_gpu(w, "fp32", "fused", 6, graph=True)
    for pa, pb in zip(a[0] + a[1], b[0] + b[1]):
        for x, y in zip(pa, pb):
            assert np.array_equal(x, y)


def test_repeated_runs_bitwise_identical():
    w = _w(1, (64, 96), 3)
    a = run_gpu(w, "fp32", "fused", 3)
    b = run_gpu(w, "fp32", "fused", 3)
    for pa, pb in zip(a[0] + a[1], b[0] + b[1]):
        for x, y in zip(pa, pb):
            assert np.array_equal(x, y)


def test_autotuned_plan_matches_oracle():
    """Autotuning picks launch grids, tiles, modes per thread and the radix
    schedule of each line pass; whatever it picks must pass parity (every
    candidate schedule is also tested on its own: the default plans and the
    radix-4 tests above)."""
    import paper_1608_05739_amd as pk
    import torch
    w = fixtures.workload(3, npatches=12, steps=3)
    plan = pk.Plan(w.patches, precision="fp32", source_mode="vacuum", path="fused", autotune=True)
    assert "(autotuned)" in plan.info
    say(plan.info)
    E = fields_to_device(w.E0, plan, "fp32")
    B = fields_to_device(w.B0, plan, "fp32")
    plan.push(E, B, steps=3)
    torch.cuda.synchronize()
    Eo = [from_device(t, plan) for t in E]
    Bo = [from_device(t, plan) for t in B]
    plan.close()
    n = len(w.patches)
    got = ([[Eo[c][p] for c in range(3)] for p in range(n)], [[Bo[c][p] for c in range(3)] for p in range(n)])
    err = compare(got, run_oracle(w, "fp32", 3), "autotuned", "fp32")
    assert err < TOL["fp32"]