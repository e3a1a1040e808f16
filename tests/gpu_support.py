"""Helpers shared by the GPU tests: move fixture arrays to the device, run the
HIP path through the binding, run the oracle on the same inputs, compare."""

from __future__ import annotations

import sys

import numpy as np

import oracle
import paper_1608_05739_amd as pk


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def torch_dtype(precision):
    import torch
    return torch.float32 if precision == "fp32" else torch.float64


def np_dtype(precision):
    return np.float32 if precision == "fp32" else np.float64


def to_device(arrays, plan, precision, device="cuda:0"):
    """Pack per-patch arrays (list over patches) into one flat device tensor."""
    import torch
    flat = np.zeros(plan.total_elements, dtype=np_dtype(precision))
    for off, a in zip(plan.offsets, arrays):
        flat[off:off + a.size] = np.asarray(a, dtype=np_dtype(precision)).ravel()
    return torch.from_numpy(flat).to(device)


def from_device(t, plan):
    """Unpack a flat device tensor into per-patch float64 arrays."""
    h = t.detach().cpu().numpy().astype(np.float64)
    return [h[off:off + p.cells].reshape(p.shape) for off, p in zip(plan.offsets, plan.patches)]


def fields_to_device(per_patch_components, plan, precision):
    """per_patch_components[p][c] -> list over c of flat device tensors."""
    ncomp = len(per_patch_components[0])
    return [to_device([pp[c] for pp in per_patch_components], plan, precision) for c in range(ncomp)]


def rounded(a, precision):
    return np.asarray(np.asarray(a, dtype=np_dtype(precision)), dtype=np.float64)


def rel_l2(a, b):
    num = sum(float(np.sum((x - y) ** 2)) for x, y in zip(a, b))
    den = sum(float(np.sum(y * y)) for y in b)
    return float(np.sqrt(num / max(den, 1e-300)))


def run_gpu(w, precision, path, steps, form="rho", order=0, graph=False, patches=None,
            E0=None, B0=None, schedule=None, radix4_lines=False):
    """Run ``steps`` steps of workload ``w`` on the GPU; returns (E, B) per patch (float64)."""
    import torch
    patches = patches if patches is not None else w.patches
    E0 = E0 if E0 is not None else w.E0
    B0 = B0 if B0 is not None else w.B0
    schedule = schedule if schedule is not None else w.schedule
    sources = w.sources
    mode = ("rho" if form == "rho" else "j") if sources else "vacuum"
    plan = pk.Plan(patches, precision=precision, source_mode=mode, path=path, order=order,
                   graph=graph, radix4_lines=radix4_lines)
    E = fields_to_device(E0, plan, precision)
    B = fields_to_device(B0, plan, precision)
    if not sources:
        plan.push(E, B, steps=steps)
    else:
        for n in range(steps):
            srcs = [schedule[p].sources(n, dtype=np_dtype(precision)) for p in range(len(patches))]
            J = fields_to_device([s[0] for s in srcs], plan, precision)
            ro = to_device([s[1] for s in srcs], plan, precision) if mode == "rho" else None
            rn = to_device([s[2] for s in srcs], plan, precision) if mode == "rho" else None
            plan.push(E, B, J, ro, rn, steps=1)
    torch.cuda.synchronize()
    Eo = [from_device(t, plan) for t in E]
    Bo = [from_device(t, plan) for t in B]
    plan.close()
    npch = len(patches)
    return ([[Eo[c][p] for c in range(3)] for p in range(npch)],
            [[Bo[c][p] for c in range(3)] for p in range(npch)])


def run_oracle(w, precision, steps, form="rho", order=0, patches=None, E0=None, B0=None,
               schedule=None):
    """The oracle on the same (precision-rounded) inputs; returns (E, B) per patch."""
    patches = patches if patches is not None else w.patches
    E0 = E0 if E0 is not None else w.E0
    B0 = B0 if B0 is not None else w.B0
    schedule = schedule if schedule is not None else w.schedule
    outE, outB = [], []
    for i, p in enumerate(patches):
        E = [rounded(a, precision) for a in E0[i]]
        B = [rounded(a, precision) for a in B0[i]]
        sched = schedule[i] if w.sources else None
        E, B = oracle.psatd_run(E, B, steps, d=p.d, dt=p.dt, schedule=sched, form=form,
                                order=order, source_dtype=np_dtype(precision))
        outE.append(E)
        outB.append(B)
    return outE, outB


COMPONENTS = ("Ex", "Ey", "Ez", "Bx", "By", "Bz")


def component_errors(got, ref):
    """Per-component errors of one patch: got, ref = six arrays (E then B).

    For a component whose reference is not identically zero: the relative L2
    error against that component's own norm, and the largest pointwise error
    over that component's own largest value.  For an identically zero
    reference: the output's norm over the norm of all six reference
    components (it must stay at rounding).  Returns {name: (rel_l2, max_rel)}.
    """
    total = np.sqrt(sum(float(np.sum(np.asarray(r, np.float64) ** 2)) for r in ref))
    out = {}
    for name, g, r in zip(COMPONENTS, got, ref):
        g = np.asarray(g, np.float64)
        r = np.asarray(r, np.float64)
        nr = float(np.sqrt(np.sum(r * r)))
        if nr == 0.0:
            e = float(np.sqrt(np.sum(g * g))) / max(total, 1e-300)
            out[name] = (e, e)
        else:
            d = g - r
            out[name] = (float(np.sqrt(np.sum(d * d))) / nr,
                         float(np.max(np.abs(d))) / float(np.max(np.abs(r))))
    return out


def compare(gpu, ref, label=None):
    """Worst error over every patch and every component of (E, B).

    Each component of each patch is measured against its own scale
    (``component_errors``): the relative L2 error and the largest pointwise
    error relative to the component's largest value; a component whose
    reference is identically zero is measured against the patch's field norm.
    Returns the largest of all these, so that a wrong low-amplitude component
    cannot hide behind the others.  Prints the per-component worst values.
    """
    (gE, gB), (rE, rB) = gpu, ref
    worst = {c: (0.0, 0.0, -1) for c in COMPONENTS}
    for p, (ge, gb, re_, rb) in enumerate(zip(gE, gB, rE, rB)):
        for name, (e2, em) in component_errors(list(ge) + list(gb), list(re_) + list(rb)).items():
            w2, wm, _ = worst[name]
            if max(e2, em) > max(w2, wm):
                worst[name] = (e2, em, p)
            else:
                worst[name] = (max(w2, e2), max(wm, em), worst[name][2])
    text = ", ".join(f"{c} {v[0]:.2e}/{v[1]:.2e}" for c, v in worst.items())
    say(f"  {label + ': ' if label else ''}per component rel L2 / max rel: {text}")
    return max(max(v[0], v[1]) for v in worst.values())


def compare_global(gpu, ref):
    """Relative L2 of (E, B) pooled over all patches and components (reported
    beside ``compare``, never asserted alone)."""
    (gE, gB), (rE, rB) = gpu, ref
    a = [x for pe, pb in zip(gE, gB) for x in pe + pb]
    b = [x for pe, pb in zip(rE, rB) for x in pe + pb]
    return rel_l2(a, b)


def field_error(got, ref, label=None):
    """``compare`` for one patch given as six arrays (Ex, Ey, Ez, Bx, By, Bz)."""
    return compare(([list(got[:3])], [list(got[3:])]), ([list(ref[:3])], [list(ref[3:])]), label)
