"""psatd_push_scratch: the entry point for callers that cannot allocate.

It must compute what psatd_push computes (same kernels, so bitwise equal),
call after call on the library's one device-resident array -- here a larger
input, then a smaller one -- allocate nothing, and reject plans whose
workspace exceeds the array."""

import numpy as np
import pytest

import fixtures
import paper_1608_05739_amd as pk
from gpu_support import fields_to_device, say

pytestmark = pytest.mark.gpu


def _run(w, push_scratch, precision="fp32", mode="vacuum", steps=3):
    import torch
    plan = pk.Plan(w.patches, precision=precision, source_mode=mode,
                   allocate_workspace=not push_scratch)
    E = fields_to_device(w.E0, plan, precision)
    B = fields_to_device(w.B0, plan, precision)
    dt = np.float32 if precision == "fp32" else np.float64
    push = plan.push_scratch if push_scratch else plan.push
    for n in range(steps):
        if mode == "vacuum":
            push(E, B, steps=1)
        else:
            srcs = [w.schedule[p].sources(n, dtype=dt) for p in range(len(w.patches))]
            J = fields_to_device([s[0] for s in srcs], plan, precision)
            ro = fields_to_device([[s[1]] for s in srcs], plan, precision)[0]
            rn = fields_to_device([[s[2]] for s in srcs], plan, precision)[0]
            push(E, B, J, ro, rn, steps=1)
    torch.cuda.synchronize()
    out = [t.cpu().numpy() for t in E + B]
    plan.close()
    return out


def test_scratch_push_equals_push_larger_then_smaller_input():
    import torch
    big = fixtures.workload(3, npatches=8, steps=3)
    small = fixtures.workload(3, npatches=2, steps=3)
    say(f"push_scratch: {big.cells} cells, then {small.cells} cells")
    ref_big = _run(big, False)
    ref_small = _run(small, False)
    torch.cuda.synchronize()
    free0 = torch.cuda.mem_get_info()[0]
    got_big = _run(big, True)
    got_small = _run(small, True)
    for a, b in zip(got_big + got_small, ref_big + ref_small):
        assert np.array_equal(a, b)
    torch.cuda.synchronize()
    # the field tensors of the runs are freed again; the pushes allocated nothing
    assert torch.cuda.mem_get_info()[0] >= free0 - (64 << 20)


def test_scratch_push_3d_fp64_with_sources():
    w = fixtures.workload(2, shape=(12, 8, 18), steps=2)
    say("push_scratch: 3D FP64 rho form")
    a = _run(w, True, "fp64", "rho", 2)
    b = _run(w, False, "fp64", "rho", 2)
    for x, y in zip(a, b):
        assert np.array_equal(x, y)


def test_scratch_push_rejects_oversized_workspace():
    import torch
    # 4096 x 4096 with sources: 704 MiB of workspace > 256 MiB
    p = pk.Patch(2, (4096, 1, 4096), (0.1, 0.1, 0.1), 0.05)
    plan = pk.Plan([p], precision="fp32", source_mode="vacuum", allocate_workspace=False)
    assert plan.workspace_size > pk._binding.SCRATCH_BYTES
    E = [torch.zeros(plan.total_elements, device="cuda:0") for _ in range(3)]
    B = [torch.zeros(plan.total_elements, device="cuda:0") for _ in range(3)]
    with pytest.raises(pk.PsatdError) as ei:
        plan.push_scratch(E, B)
    assert ei.value.status == -5
    plan.close()
