"""psatd_push_profiled: the measured push computes exactly what psatd_push
computes, for eager plans (kernels one after the other) and graph plans (one
captured graph per pass, per-length launches as parallel branches), and
reports a positive time for every pass."""

import numpy as np
import pytest

import fixtures
import paper_1608_05739_amd as pk
from gpu_support import fields_to_device, say, to_device

pytestmark = pytest.mark.gpu


def _fields(plan, w, precision):
    E = fields_to_device(w.E0, plan, precision)
    B = fields_to_device(w.B0, plan, precision)
    if not w.sources:
        return E, B, None, None, None
    srcs = [w.schedule[p].sources(0) for p in range(len(w.patches))]
    J = [to_device([s[0][c] for s in srcs], plan, precision) for c in range(3)]
    return (E, B, J, to_device([s[1] for s in srcs], plan, precision),
            to_device([s[2] for s in srcs], plan, precision))


@pytest.mark.parametrize("graph", [False, True])
@pytest.mark.parametrize("label,index,shape,npatch,mode", [
    ("batched 2D, 20 patches of mixed lengths, vacuum", 3, None, 20, "vacuum"),
    ("3D 32x48x64 with sources", 2, (32, 48, 64), 1, "rho"),
])
def test_profiled_push_equals_push(label, index, shape, npatch, mode, graph):
    import torch
    say(f"profiled push: {label}, graph={graph}")
    w = (fixtures.workload(index, shape=shape, steps=2) if shape else
         fixtures.workload(index, steps=2, npatches=npatch))
    steps = 1 if w.sources else 3
    out = []
    for profiled in (False, True):
        plan = pk.Plan(w.patches, precision="fp32", source_mode=mode, graph=graph)
        E, B, J, ro, rn = _fields(plan, w, "fp32")
        if profiled:
            ms = plan.push_profiled(E, B, J, ro, rn, steps=steps)
            assert len(ms) == plan.npass and all(m > 0.0 for m in ms), ms
        else:
            plan.push(E, B, J, ro, rn, steps=steps)
        torch.cuda.synchronize()
        out.append(np.concatenate([t.cpu().numpy() for t in E + B]))
        plan.close()
    assert np.array_equal(out[0], out[1])
