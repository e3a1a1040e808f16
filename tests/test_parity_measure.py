"""The GPU tests' parity measure (tests/gpu_support.py) on planted errors.

It must flag an error confined to a component that carries little of the
field energy (a pooled relative L2 over all six components would not), a
single wrong point, and a non-zero output where the reference component is
identically zero."""

import numpy as np

from gpu_support import compare, component_errors


def _ref(rng):
    return [rng.normal(size=(32, 40)) * s for s in (1.0, 1.0, 1.0, 1.0, 1.0, 1e-3)]


def test_small_component_error_is_flagged():
    rng = np.random.default_rng(1)
    ref = _ref(rng)
    got = [r.copy() for r in ref]
    got[5] *= 1.01  # 1 % error on Bz, which holds 1e-3 of the field norm
    assert component_errors(got, ref)["Bz"][0] > 5e-3
    pooled = np.sqrt(sum(np.sum((g - r) ** 2) for g, r in zip(got, ref))
                     / sum(np.sum(r * r) for r in ref))
    assert pooled < 1e-5
    assert compare(([got[:3]], [got[3:]]), ([ref[:3]], [ref[3:]])) > 5e-3


def test_single_wrong_point_is_flagged():
    rng = np.random.default_rng(2)
    ref = _ref(rng)
    got = [r.copy() for r in ref]
    got[1][7, 9] += 1e-3 * np.max(np.abs(ref[1]))
    e = component_errors(got, ref)["Ey"]
    assert e[1] > 9e-4 and e[0] < 1e-4


def test_nonzero_output_over_zero_reference_is_flagged():
    rng = np.random.default_rng(3)
    ref = _ref(rng)
    ref[1] = np.zeros_like(ref[1])
    got = [r.copy() for r in ref]
    assert component_errors(got, ref)["Ey"] == (0.0, 0.0)
    got[1][0, 0] = 1e-3
    assert component_errors(got, ref)["Ey"][0] > 1e-6


def test_worst_patch_decides():
    rng = np.random.default_rng(4)
    refs = [_ref(rng) for _ in range(3)]
    gots = [[r.copy() for r in ref] for ref in refs]
    gots[2][4] *= 1 + 1e-4
    err = compare(([g[:3] for g in gots], [g[3:] for g in gots]),
                  ([r[:3] for r in refs], [r[3:] for r in refs]))
    assert 5e-5 < err < 2e-4
