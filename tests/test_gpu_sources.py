"""The per-step source generator on the GPU (fixtures.DeviceSourceSchedule)
against the host schedule, and a multi-step PSATD run fed by it against the
oracle.

The generator is input synthesis (no part of the field step): J_c = f_c P_c
and rho^{n+1} = -dt sum_c F_c(n+1) D_c in the host schedule's FP64 operation
order, rounded to the storage type, so its values equal the host's bitwise.
"""

import numpy as np
import pytest

import fixtures
from fixtures.device import DeviceSourceSchedule
from gpu_support import compare, fields_to_device, from_device, run_oracle, say

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("index,shape", [(1, (48, 64)), (2, (12, 8, 18))])
@pytest.mark.parametrize("dtype", ["float32", "float64"])
def test_device_sources_equal_host_sources(index, shape, dtype):
    import torch
    w = fixtures.workload(index, shape=shape, steps=4)
    sched = w.schedule[0]
    tdt = getattr(torch, dtype)
    gen = DeviceSourceSchedule(sched, torch, dtype=tdt)
    n = gen.cells
    J = [torch.empty(n, dtype=tdt, device="cuda") for _ in range(3)]
    ro = torch.empty(n, dtype=tdt, device="cuda")
    rn = torch.empty(n, dtype=tdt, device="cuda")
    for step in range(4):
        gen.sources_into(step, J, ro, rn)
        Jh, roh, rnh = sched.sources(step, dtype=np.dtype(dtype))
        for c in range(3):
            assert np.array_equal(J[c].cpu().numpy(), Jh[c].ravel()), (step, c)
        assert np.array_equal(ro.cpu().numpy(), roh.ravel())
        assert np.array_equal(rn.cpu().numpy(), rnh.ravel())


def test_device_source_advance_swaps_rho():
    import torch
    w = fixtures.workload(1, shape=(24, 32), steps=5)
    sched = w.schedule[0]
    gen = DeviceSourceSchedule(sched, torch)
    n = gen.cells
    J = [torch.empty(n, dtype=torch.float32, device="cuda") for _ in range(3)]
    a = torch.empty(n, dtype=torch.float32, device="cuda")
    b = torch.empty(n, dtype=torch.float32, device="cuda")
    for step in range(5):
        gen.advance_into(step, J, a, b)
        _, roh, rnh = sched.sources(step, dtype=np.float32)
        assert np.array_equal(a.cpu().numpy(), roh.ravel()), step
        assert np.array_equal(b.cpu().numpy(), rnh.ravel()), step
        a, b = b, a


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_psatd_run_fed_by_device_sources_matches_oracle(precision):
    import torch
    import paper_1608_05739_amd as pk
    w = fixtures.workload(1, shape=(96, 128), steps=8)
    say(f"device sources 96x128 {precision} 8 steps")
    tdt = torch.float32 if precision == "fp32" else torch.float64
    plan = pk.Plan(w.patches, precision=precision, source_mode="rho", path="fused")
    E = fields_to_device(w.E0, plan, precision)
    B = fields_to_device(w.B0, plan, precision)
    gen = DeviceSourceSchedule(w.schedule[0], torch, dtype=tdt)
    n = plan.total_elements
    J = [torch.zeros(n, dtype=tdt, device="cuda") for _ in range(3)]
    ro = torch.zeros(n, dtype=tdt, device="cuda")
    rn = torch.zeros(n, dtype=tdt, device="cuda")
    for step in range(w.steps):
        gen.advance_into(step, J, ro, rn)
        plan.push(E, B, J, ro, rn, steps=1)
        ro, rn = rn, ro
    torch.cuda.synchronize()
    Eo = [from_device(t, plan) for t in E]
    Bo = [from_device(t, plan) for t in B]
    plan.close()
    got = ([[Eo[c][0] for c in range(3)]], [[Bo[c][0] for c in range(3)]])
    err = compare(got, run_oracle(w, precision, w.steps), precision=precision)
    assert err < {"fp32": 1e-5, "fp64": 1e-12}[precision]
