"""Saved kernel choices: psatd_plan_tuning exports an autotuned plan's
choices and psatd_plan_tuned applies them with no timing launch.  The tuned
plan must describe the same passes, export the same string and compute the
same results bit for bit; a choice the plan does not offer is an error."""

import numpy as np
import pytest

import fixtures
import paper_1608_05739_amd as pk
from gpu_support import fields_to_device, say

pytestmark = pytest.mark.gpu


def _passes(info):
    # pass lines without the tuning marker
    return [ln.replace(" (autotuned)", "").replace(" (tuning applied)", "")
            for ln in info.splitlines()[1:]]


def _run(plan, w, precision, steps):
    import torch
    E = fields_to_device(w.E0, plan, precision)
    B = fields_to_device(w.B0, plan, precision)
    if w.sources:
        from gpu_support import to_device
        srcs = [w.schedule[p].sources(0) for p in range(len(w.patches))]
        J = [to_device([s[0][c] for s in srcs], plan, precision) for c in range(3)]
        ro = to_device([s[1] for s in srcs], plan, precision)
        rn = to_device([s[2] for s in srcs], plan, precision)
        for _ in range(steps):
            plan.push(E, B, J, ro, rn, steps=1)
    else:
        plan.push(E, B, steps=steps)
    torch.cuda.synchronize()
    return np.concatenate([t.cpu().numpy() for t in E + B])


CASES = [
    ("batched 2D, 24 patches of workload 3, vacuum", 3, None, 24, "vacuum", "fp32"),
    ("3D 32x64x48 with sources", 2, (32, 64, 48), 1, "rho", "fp32"),
    ("2D 96x128 with sources, fp64", 1, (96, 128), 1, "rho", "fp64"),
]


@pytest.mark.parametrize("label,index,shape,npatch,mode,precision", CASES)
def test_applied_tuning_equals_autotuned_plan(label, index, shape, npatch, mode, precision):
    say(f"tuning roundtrip: {label}")
    w = (fixtures.workload(index, shape=shape, steps=3) if shape else
         fixtures.workload(index, steps=3, npatches=npatch))
    patches = w.patches
    assert len(patches) == npatch
    auto = pk.Plan(patches, precision=precision, source_mode=mode, path="fused", autotune=True)
    text = auto.tuning
    assert text.startswith("psatd-tuning-1;") and text.count(";") == auto.npass
    again = pk.Plan(patches, precision=precision, source_mode=mode, path="fused", tuning=text)
    assert "(tuning applied)" in again.info
    assert _passes(again.info) == _passes(auto.info)
    assert again.tuning == text
    a = _run(auto, w, precision, 3)
    b = _run(again, w, precision, 3)
    auto.close()
    again.close()
    assert np.array_equal(a, b)


def test_untuned_plan_tuning_applies_its_defaults():
    say("tuning: defaults")
    p = pk.Patch(2, (64, 1, 96), (1.0, 1.0, 1.0), 0.5)
    plain = pk.Plan([p])
    text = plain.tuning
    assert all(c.endswith(",-1") for c in text.split(";")[1:])
    again = pk.Plan([p], tuning=text)
    assert _passes(again.info) == _passes(plain.info)
    plain.close()
    again.close()


def test_tuning_choice_not_offered_is_rejected():
    say("tuning: invalid choices")
    p = pk.Patch(2, (64, 1, 96), (1.0, 1.0, 1.0), 0.5)
    auto = pk.Plan([p], autotune=True)
    text = auto.tuning
    auto.close()
    head, *choices = text.split(";")
    bad = []
    # one choice too few
    bad.append(";".join([head] + choices[:-1]))
    # a tile no candidate has
    f = choices[0].split(",")
    bad.append(";".join([head, ",".join(f[:2] + ["3"] + f[3:])] + choices[1:]))
    # a grid code the pass does not offer
    bad.append(";".join([head, ",".join(f[:5] + ["7"])] + choices[1:]))
    for t in bad:
        with pytest.raises(pk.PsatdError) as ei:
            pk.Plan([p], tuning=t)
        assert ei.value.status == -1 and "tuning" in str(ei.value), t
