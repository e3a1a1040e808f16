"""GPU parity at the benchmark's full size (2D 4096 x 4096 with sources), in
the launch configuration bench.py times (FP32 storage, fused path, which
selects the kernels specialized for this shape)."""

import numpy as np
import pytest

import fixtures
import oracle
import paper_1608_05739_amd as pk
from gpu_support import rel_l2, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def w1():
    say("generating 4096x4096 workload ...")
    return fixtures.workload(1)


def _dev(a, dtype=np.float32):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a, dtype=dtype).ravel()).to("cuda:0")


def _host(t, shape):
    return t.detach().cpu().numpy().astype(np.float64).reshape(shape)


def _run(w, steps, generic=False, n0=0):
    import torch
    p = w.patches[0]
    plan = pk.Plan([p], precision="fp32", source_mode="rho", path="fused",
                   generic_kernels=generic)
    E = [_dev(a) for a in w.E0[0]]
    B = [_dev(a) for a in w.B0[0]]
    for n in range(n0, n0 + steps):
        J, ro, rn = w.schedule[0].sources(n, dtype=np.float32)
        plan.push(E, B, [_dev(x) for x in J], _dev(ro), _dev(rn), steps=1)
    torch.cuda.synchronize()
    names = plan.pass_names
    plan.close()
    return [_host(t, p.shape) for t in E + B], names


def test_fullsize_one_step_vs_oracle(w1):
    p = w1.patches[0]
    say("fast path, 1 step at 4096x4096 vs oracle")
    got, names = _run(w1, 1)
    assert names == ["x_r2c_fwd", "z_fused", "x_c2r_inv"]
    E = [np.asarray(a, np.float32).astype(np.float64) for a in w1.E0[0]]
    B = [np.asarray(a, np.float32).astype(np.float64) for a in w1.B0[0]]
    J, ro, rn = w1.schedule[0].sources(0, dtype=np.float32)
    En, Bn = oracle.psatd_step(E, B, [x.astype(np.float64) for x in J], ro.astype(np.float64),
                               rn.astype(np.float64), d=p.d, dt=p.dt)
    err = rel_l2(got, En + Bn)
    say(f"  rel L2 = {err:.3e}")
    assert err < 1e-5


def test_fast_path_matches_generic_kernels(w1):
    say("fast vs generic kernels, 3 steps at 4096x4096")
    a, _ = _run(w1, 3, generic=False)
    b, names = _run(w1, 3, generic=True)
    assert names == ["x_r2c_fwd", "z_fused", "x_c2r_inv"]
    err = rel_l2(a, b)
    say(f"  rel L2 (fast vs generic) = {err:.3e}")
    assert err < 2e-6
