"""GPU-side boundary behaviour: documented status codes, workspace handling."""

import pytest

import paper_1608_05739_amd as pk
from gpu_support import say

pytestmark = pytest.mark.gpu


def _patch(nx=16, nz=8):
    return pk.Patch(2, (nx, 1, nz), (0.1, 0.1, 0.1), 0.05)


def _fields(n, dtype, k=3):
    import torch
    return [torch.zeros(n, dtype=dtype, device="cuda:0") for _ in range(k)]


def test_sources_require_single_step():
    import torch
    say("boundary: nsteps > 1 with sources")
    plan = pk.Plan([_patch()], source_mode="rho")
    E, B, J = (_fields(plan.total_elements, torch.float32) for _ in range(3))
    ro, rn = _fields(plan.total_elements, torch.float32, 2)
    with pytest.raises(pk.PsatdError) as ei:
        plan.push(E, B, J, ro, rn, steps=2)
    assert ei.value.status == -1
    plan.push(E, B, J, ro, rn, steps=1)
    torch.cuda.synchronize()


def test_missing_sources_rejected():
    import torch
    plan = pk.Plan([_patch()], source_mode="rho")
    E, B = (_fields(plan.total_elements, torch.float32) for _ in range(2))
    with pytest.raises(pk.PsatdError):
        plan.push(E, B, None, None, None)


def test_workspace_lifecycle():
    import torch
    say("boundary: workspace")
    plan = pk.Plan([_patch()], allocate_workspace=False)
    E, B = (_fields(plan.total_elements, torch.float32) for _ in range(2))
    with pytest.raises(pk.PsatdError) as ei:
        plan.push(E, B)
    assert ei.value.status == -5
    small = torch.empty(plan.workspace_size // 4 - 64, dtype=torch.int32, device="cuda:0")
    with pytest.raises(pk.PsatdError) as ei:
        plan.set_workspace(small)
    assert ei.value.status == -5
    ws = torch.empty(plan.workspace_size // 4 + 64, dtype=torch.int32, device="cuda:0")
    plan.set_workspace(ws)
    plan.push(E, B, steps=3)
    torch.cuda.synchronize()


def test_dtype_mismatch_rejected_by_binding():
    import torch
    plan = pk.Plan([_patch()], precision="fp64")
    E, B = (_fields(plan.total_elements, torch.float32) for _ in range(2))
    with pytest.raises(TypeError):
        plan.push(E, B)


def test_fused_plan_takes_plain_z_passes_where_lines_do_not_fit():
    # FP64 2D holds at most 2048 modes of a z line per workgroup of the fused
    # pass: a fused plan with nz = 4096 runs the plain z passes instead
    plan = pk.Plan([pk.Patch(2, (8, 1, 4096), (1.0, 1.0, 1.0), 0.5)], precision="fp64",
                   path="fused")
    assert plan.pass_names == ["x_r2c_fwd", "z_c2c_fwd", "update", "z_c2c_inv", "x_c2r_inv"]
    plan.close()
    # a length the planner does not take at all is still an error
    with pytest.raises(pk.PsatdError) as ei:
        pk.Plan([pk.Patch(2, (8, 1, 8192), (1.0, 1.0, 1.0), 0.5)], precision="fp64", path="fused")
    assert ei.value.status == -2


def test_pass_metadata():
    plan = pk.Plan([_patch()], source_mode="rho")
    assert plan.pass_names == ["x_r2c_fwd", "z_fused", "x_c2r_inv"]
    assert all(b > 0 for b in plan.pass_bytes)
    assert "z_fused" in plan.info


# ----------------------------------------------------------------- graphs and capture
def _laser_fields(plan, w, dtype):
    import numpy as np
    import torch

    def pack(arrs):
        flat = np.zeros(plan.total_elements, dtype)
        for off, a in zip(plan.offsets, arrs):
            flat[off:off + a.size] = np.asarray(a, dtype).ravel()
        return torch.from_numpy(flat).to("cuda:0")

    E = [pack([w.E0[i][c] for i in range(len(w.patches))]) for c in range(3)]
    B = [pack([w.B0[i][c] for i in range(len(w.patches))]) for c in range(3)]
    return E, B


@pytest.mark.parametrize("graph", [False, True])
def test_push_inside_caller_capture_replays_like_eager(graph):
    """A push recorded in the caller's own stream capture (torch.cuda.graph)
    replays bitwise like eager pushes, replay after replay, with eager work of
    the program in between."""
    import numpy as np
    import torch
    import fixtures
    say(f"boundary: push under torch.cuda.graph capture (plan graph flag {graph})")
    w = fixtures.workload(3, npatches=5, steps=3)
    plan = pk.Plan(w.patches, precision="fp32", source_mode="vacuum", graph=graph)
    E, B = _laser_fields(plan, w, np.float32)
    Ee, Be = [t.clone() for t in E], [t.clone() for t in B]
    g = torch.cuda.CUDAGraph()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        plan.push(E, B, steps=1)  # warm-up outside the capture
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    plan.push(Ee, Be, steps=1)
    with torch.cuda.graph(g):
        plan.push(E, B, steps=1)
    for r in range(3):
        g.replay()
        plan.push(Ee, Be, steps=1)
        junk = torch.ones(1 << 20, device="cuda:0") * (r + 1)  # eager work in between
        torch.cuda.synchronize()
        del junk
        for a, b in zip(E + B, Ee + Be):
            assert torch.equal(a, b), f"replay {r} differs from eager"
    plan.close()


def test_graph_plan_alternating_buffers_matches_eager_and_allocates_nothing():
    """A graph plan pushed on two alternating field sets (as a PIC loop
    swapping buffers would) equals the eager plan bitwise, and the pushes
    leave the device's free memory unchanged (no allocation per push)."""
    import numpy as np
    import torch
    import fixtures
    say("boundary: graph plan, alternating field buffers")
    w = fixtures.workload(3, npatches=6, steps=3)
    pg = pk.Plan(w.patches, precision="fp32", source_mode="vacuum", graph=True)
    pe = pk.Plan(w.patches, precision="fp32", source_mode="vacuum")
    A = _laser_fields(pg, w, np.float32)
    Bset = ([t * 0.5 for t in A[0]], [t * 0.5 for t in A[1]])
    Ae = ([t.clone() for t in A[0]], [t.clone() for t in A[1]])
    Be = ([t.clone() for t in Bset[0]], [t.clone() for t in Bset[1]])
    pg.push(*A, steps=1)
    pe.push(*Ae, steps=1)
    torch.cuda.synchronize()
    free0 = torch.cuda.mem_get_info()[0]
    for n in range(6):
        pg.push(*(A if n % 2 else Bset), steps=2)
        pe.push(*(Ae if n % 2 else Be), steps=2)
    torch.cuda.synchronize()
    assert torch.cuda.mem_get_info()[0] == free0
    for a, b in zip(A[0] + A[1] + Bset[0] + Bset[1], Ae[0] + Ae[1] + Be[0] + Be[1]):
        assert torch.equal(a, b)
    pg.close()
    pe.close()


def test_checkpoint_resume_is_bitwise(tmp_path):
    """Two runs of 50 steps with the fields saved and reloaded in between
    (torch.save / torch.load) equal 100 steps in one run, bitwise: the plan
    keeps no state across pushes."""
    import numpy as np
    import torch
    import fixtures
    say("boundary: 2 x 50 steps with save/load == 100 steps")
    w = fixtures.workload(1, shape=(96, 128), steps=100)
    sched = w.schedule[0]

    def run(plan, E, B, n0, n1):
        for n in range(n0, n1):
            J, ro, rn = sched.sources(n, dtype=np.float32)
            dev = [torch.from_numpy(np.ascontiguousarray(a).ravel()).to("cuda:0") for a in J + [ro, rn]]
            plan.push(E, B, dev[:3], dev[3], dev[4], steps=1)

    plan = pk.Plan(w.patches, precision="fp32", source_mode="rho")
    E, B = _laser_fields(plan, w, np.float32)
    E2, B2 = [t.clone() for t in E], [t.clone() for t in B]
    run(plan, E, B, 0, 100)
    run(plan, E2, B2, 0, 50)
    torch.cuda.synchronize()
    path = tmp_path / "fields.pt"
    torch.save({"E": [t.cpu() for t in E2], "B": [t.cpu() for t in B2]}, path)
    plan.close()
    del E2, B2
    state = torch.load(path, weights_only=True)
    plan2 = pk.Plan(w.patches, precision="fp32", source_mode="rho")
    E2 = [t.to("cuda:0") for t in state["E"]]
    B2 = [t.to("cuda:0") for t in state["B"]]
    run(plan2, E2, B2, 50, 100)
    torch.cuda.synchronize()
    for a, b in zip(E + B, E2 + B2):
        assert torch.equal(a, b)
    plan2.close()


def test_workspace_beyond_device_memory_reports_oom():
    """Two 2048 x 1024 x 1024 patches with sources need ~378 GB of workspace,
    more than the device holds: planning returns PSATD_ERR_OOM and frees what
    it had allocated."""
    import torch
    say("boundary: workspace larger than the device -> PSATD_ERR_OOM")
    free0 = torch.cuda.mem_get_info()[0]
    patches = [pk.Patch(3, (2048, 1024, 1024), (0.1, 0.1, 0.1), 0.05, offset=o)
               for o in (0, 2048 * 1024 * 1024)]
    with pytest.raises(pk.PsatdError) as ei:
        pk.Plan(patches, precision="fp32", source_mode="rho")
    assert ei.value.status == -3
    torch.cuda.synchronize()
    assert torch.cuda.mem_get_info()[0] >= free0 - (64 << 20)


def test_plans_work_after_an_out_of_memory_plan():
    """After a plan fails with PSATD_ERR_OOM the runtime's error state is
    clear: the next plan and push succeed."""
    import torch
    with pytest.raises(pk.PsatdError):
        pk.Plan([pk.Patch(3, (2048, 1024, 1024), (0.1, 0.1, 0.1), 0.05, offset=o)
                 for o in (0, 2048 * 1024 * 1024)], precision="fp32", source_mode="rho")
    plan = pk.Plan([_patch()])
    E, B = (_fields(plan.total_elements, torch.float32) for _ in range(2))
    plan.push(E, B, steps=2)
    torch.cuda.synchronize()
    plan.close()


def test_plan_created_before_torch_touches_the_gpu():
    # A fresh process whose first GPU call is the library's: torch must still
    # find the GPU afterwards (one HIP runtime in the process), and the plan
    # must run on torch's tensors.
    import subprocess
    import sys
    say("boundary: plan before torch's first GPU call (subprocess)")
    code = (
        "import paper_1608_05739_amd as pk\n"
        "plan = pk.Plan([pk.Patch(2, (16, 1, 8), (0.1, 0.1, 0.1), 0.05)])\n"
        "import torch\n"
        "E = [torch.zeros(plan.total_elements, device='cuda:0') for _ in range(3)]\n"
        "B = [torch.ones(plan.total_elements, device='cuda:0') for _ in range(3)]\n"
        "plan.push(E, B, steps=2)\n"
        "torch.cuda.synchronize()\n"
        "assert all(bool(torch.isfinite(t).all()) for t in E + B)\n"
        "print('ok')\n")
    import os
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, timeout=120,
                       cwd=root)
    assert r.returncode == 0 and r.stdout.strip().endswith("ok"), r.stdout[-2000:] + r.stderr[-2000:]
