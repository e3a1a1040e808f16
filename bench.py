"""Benchmark of the PSATD field step on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload 3]

A step is one full pass of the hot path (x r2c FFT of every input, fused z
pass with the per-mode update, x c2r FFT of E and B; 3D adds the y passes)
over the workload's synthetic fields, inputs resident in HBM.  Workload 3
(default): 256 independent periodic 2D patches with sides from 64 to 512,
each with its own time step, vacuum, FP32 storage, one launch per pass over
all patches, hipGraph replay, autotuned launch shapes.  Prints ONE JSON line
on stdout; progress goes to stderr.

The line also reports, on the same workload: the plain FP64 path, the
per-pass durations (HIP events on the launch stream), the roofline of the
dominant kernel, and -- in the oracle leg -- the oracle's own throughput on
the host cores (cpu_baseline) and the error of both GPU paths against the
FP64 oracle after the run's step count, per field component.
"""

from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "PSATD cell-steps/s + HBM GB/s (% peak), FP32 batched vs FP64 plain, 1 GPU"
PEAK_HBM_GBS = 8000.0
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic.json")
CSRC = os.path.join(ROOT, "paper_1608_05739_amd", "csrc")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


# Device-code sources of the kernels; a change to any of them makes the stored
# traffic counters stale.
def kernel_sources():
    return sorted(n for n in os.listdir(CSRC) if n.endswith((".hip", ".hpp")))


def kernel_source_hash():
    h = hashlib.sha256()
    for name in kernel_sources():
        with open(os.path.join(CSRC, name), "rb") as f:
            h.update(name.encode())
            h.update(f.read())
    return h.hexdigest()[:16]


def measured_traffic(workload, kernel):
    """HBM bytes per launch from committed rocprofv3 counters, if they still
    describe the current kernel sources; else None."""
    try:
        with open(TRAFFIC_FILE) as f:
            data = json.load(f)
    except (OSError, ValueError):
        return None
    ent = data.get(f"{workload}:{kernel}")
    if not ent or ent.get("source_hash") != kernel_source_hash():
        return None
    return ent.get("bytes_per_launch")


# rocprofv3 kernel names -> pass names: the 4096 x 4096 kernels, the wave
# z pass, and the line kernels whose template argument KIND names the pass
# (line_pass_kernel<S, KIND, PPT>, ct_line_kernel<S, KIND, L>,
# wave_x_kernel<KIND, L>; KIND 0 x fwd, 1 x inv, 2 y fwd, 3 y inv, 4 z fwd,
# 5 z inv)
LINE_KINDS = {"0": "x_r2c_fwd", "1": "x_c2r_inv", "2": "y_c2c_fwd", "3": "y_c2c_inv",
              "4": "z_c2c_fwd", "5": "z_c2c_inv"}


def pass_of_kernel(name):
    import re
    for key, pname in (("x_fwd_kernel", "x_r2c_fwd"), ("z_fused_kernel", "z_fused"),
                       ("x_inv_kernel", "x_c2r_inv"), ("fused_z_kernel", "z_fused"),
                       ("wave_z_fused", "z_fused"), ("wave_z3_fused", "z_fused"),
                       ("wave_z_set", "z_fused"),
                       ("update_kernel", "update")):
        if key in name:
            return pname
    m = (re.search(r"(?:line_pass_kernel|ct_line_kernel)<[^,<>]+, ?(\d)", name)
         or re.search(r"wave_x_kernel<(\d)", name))
    if m:
        return LINE_KINDS[m.group(1)]
    return None


def final_dispatches(rows):
    """The plan's final launches in a list of (kernel, grid, ...) dispatches in
    dispatch order (pass kernels only): the set of (kernel, grid) of the last
    step -- walking back from the end until one repeats -- and the trailing
    run of dispatches drawn from that set (the timed and profiled steps; the
    autotuner's trial launches at plan time come before it)."""
    last = set()
    for r in reversed(rows):
        if (r[0], r[1]) in last:
            break
        last.add((r[0], r[1]))
    out = []
    for r in reversed(rows):
        if (r[0], r[1]) not in last:
            break
        out.append(r)
    return out[::-1]


def ingest_traffic(fetch_csv, write_csv, workload_index, calib_mib):
    """Turn two rocprofv3 --pmc runs of this script (FETCH_SIZE, then
    WRITE_SIZE, both with --copy-calibration-mib) into HBM bytes per launch
    of each pass, scaled by what the counters read for the calibration copy,
    and store them in profiles/traffic.json with the kernel-source hash."""
    import csv
    import fixtures

    def rows(path, counter):
        out = []
        with open(path) as f:
            for r in csv.DictReader(f):
                if r["Counter_Name"] == counter:
                    grid = r.get("Grid_Size") or r.get("Grid_Size_X") or "0"
                    out.append((int(r["Dispatch_Id"]), r["Kernel_Name"], int(grid),
                                float(r["Counter_Value"])))
        out.sort()
        return [(n, g, v) for _, n, g, v in out]

    fetch_all, write_all = rows(fetch_csv, "FETCH_SIZE"), rows(write_csv, "WRITE_SIZE")
    fetch = [(n, v) for n, _, v in fetch_all]
    write = [(n, v) for n, _, v in write_all]
    kib = calib_mib * 1024.0
    # the calibration copy: the first copy kernel whose WRITE_SIZE is the copied size
    wcal = next(v for n, v in write if "copy" in n.lower() and abs(v - kib) < 0.01 * kib)
    fcal = next(v for n, v in fetch if "copy" in n.lower() and 0.3 * kib < v < 1.2 * kib)
    fscale, wscale = kib / fcal, kib / wcal
    name = fixtures.CONFIG_NAMES[workload_index]
    try:
        with open(TRAFFIC_FILE) as f:
            data = json.load(f)
    except (OSError, ValueError):
        data = {}
    h = kernel_source_hash()
    # the plan's final kernels only (not the autotuner's trial launches)
    fetch = [((n, g), v) for n, g, v in final_dispatches([r for r in fetch_all if pass_of_kernel(r[0])])]
    write = [((n, g), v) for n, g, v in final_dispatches([r for r in write_all if pass_of_kernel(r[0])])]
    passes = sorted({pass_of_kernel(k[0]) for k, _ in fetch} - {None})
    for pname in passes:
        # a pass launched per length: one launch (kernel and grid: one kernel
        # may serve several lengths at different grids) per length, each once
        # a step
        f_kib = w_kib = 0.0
        ndisp = 0
        for key in sorted({k for k, _ in fetch if pass_of_kernel(k[0]) == pname}):
            fv = [v for k, v in fetch if k == key]
            wv = [v for k, v in write if k == key]
            if not fv or not wv:
                continue
            f_kib += sum(fv) / len(fv)
            w_kib += sum(wv) / len(wv)
            ndisp += len(fv)
        if ndisp == 0:
            continue
        data[f"{name}:{pname}"] = {
            "bytes_per_launch": (f_kib * fscale + w_kib * wscale) * 1024.0,
            "fetch_kib": f_kib, "write_kib": w_kib, "fetch_scale": fscale, "write_scale": wscale,
            "dispatches": ndisp, "source_hash": h}
    os.makedirs(os.path.dirname(TRAFFIC_FILE), exist_ok=True)
    with open(TRAFFIC_FILE, "w") as f:
        json.dump(data, f, indent=1, sort_keys=True)
        f.write("\n")
    return data


def plan_grids(plan):
    """Launch grid of each pass, as the plan reports it (after autotuning)."""
    out = {}
    for line in plan.info.splitlines()[1:]:
        parts = line.split()
        if parts and any(p.startswith("grid=") for p in parts):
            out[parts[0]] = int(next(p for p in parts if p.startswith("grid="))[5:])
    return out


def build_inputs(index, steps, npatches=None):
    import fixtures

    log(f"[bench] generating workload {index} inputs ...")
    t = time.time()
    w = fixtures.workload(index, steps=steps, npatches=npatches)
    log(f"[bench]   {w.name}: {w.cells} cells, {len(w.patches)} patch(es), {time.time() - t:.1f} s")
    return w


def device_fields(w, plan, dtype):
    import torch

    def pack(arrs):
        flat = np.zeros(plan.total_elements, dtype=dtype)
        for off, a in zip(plan.offsets, arrs):
            flat[off:off + a.size] = np.asarray(a, dtype=dtype).ravel()
        return torch.from_numpy(flat).to("cuda:0")

    E = [pack([w.E0[p][c] for p in range(len(w.patches))]) for c in range(3)]
    B = [pack([w.B0[p][c] for p in range(len(w.patches))]) for c in range(3)]
    J = ro = rn = None
    if w.sources:
        srcs = [w.schedule[p].sources(0, dtype=dtype) for p in range(len(w.patches))]
        J = [pack([s[0][c] for s in srcs]) for c in range(3)]
        ro = pack([s[1] for s in srcs])
        rn = pack([s[2] for s in srcs])
    return E, B, J, ro, rn


def fp32_plan(pk, args, patches, mode):
    """The timed plan: FP32 storage, fused path, graph replay, autotuned --
    or, with --tuning-in, the kernel choices an earlier autotuned run saved
    (no timing launches at plan time; profilers that serialize dispatches
    distort the autotuner's timings, so profiled runs reuse a normal run's
    choices).  --tuning-out saves the plan's choices."""
    if args.tuning_in:
        with open(args.tuning_in) as f:
            text = f.read().strip()
        plan = pk.Plan(patches, precision="fp32", source_mode=mode, path="fused", graph=True,
                       tuning=text)
    else:
        plan = pk.Plan(patches, precision="fp32", source_mode=mode, path="fused", graph=True,
                       autotune=True)
    if args.tuning_out:
        d = os.path.dirname(args.tuning_out)
        if d:
            os.makedirs(d, exist_ok=True)
        with open(args.tuning_out, "w") as f:
            f.write(plan.tuning + "\n")
    return plan


def time_steps(plan, E, B, J, ro, rn, steps, warmup, vacuum_batch):
    """Wall-clock seconds of exactly `steps` steps, synchronized on both sides."""
    import torch

    def run(n):
        if vacuum_batch:
            plan.push(E, B, steps=n)
        else:
            for _ in range(n):
                plan.push(E, B, J, ro, rn, steps=1)

    run(warmup)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    run(steps)
    torch.cuda.synchronize()
    return time.perf_counter() - t0


# ------------------------------------------------------------------ oracle leg
# Everything below that calls the oracle is the cpu_baseline leg: the oracle
# timed on the host cores, and the GPU results of the timed configuration
# checked against it.
def component_errors(got, ref, ndim):
    """Per component (E then B): relative L2 error against the component's own
    norm and against its coupled set's norm (2D: the s set Ey, Bx, Bz and the
    p set Ex, Ez, By never mix; 3D: all six)."""
    groups = ((1, 3, 5), (0, 2, 4)) if ndim == 2 else ((0, 1, 2, 3, 4, 5),)
    names = ("Ex", "Ey", "Ez", "Bx", "By", "Bz")
    out = {}
    for g in groups:
        gn = np.sqrt(sum(float(np.sum(ref[c] ** 2)) for c in g))
        for c in g:
            e = float(np.sqrt(np.sum((got[c] - ref[c]) ** 2)))
            own = float(np.sqrt(np.sum(ref[c] ** 2)))
            out[names[c]] = (e / own if own > 0 else e / max(gn, 1e-300), e / max(gn, 1e-300))
    return out


def summarize(per_patch):
    """Worst own-norm and coupled-set errors per component over the patches,
    and the relative L2 pooled over everything."""
    worst = {}
    num = den = 0.0
    for errs, n2, d2 in per_patch:
        num += n2
        den += d2
        for k, (a, b) in errs.items():
            wa, wb = worst.get(k, (0.0, 0.0))
            worst[k] = (max(wa, a), max(wb, b))
    return {"per_component_own": {k: v[0] for k, v in worst.items()},
            "per_component_coupled_set": {k: v[1] for k, v in worst.items()},
            "max_coupled_set": max(v[1] for v in worst.values()),
            "max_own": max(v[0] for v in worst.values()),
            "pooled": float(np.sqrt(num / max(den, 1e-300)))}


def oracle_leg(w, budget_s, gpu_results, steps, label=None):
    """cpu_baseline: the FP64 oracle unchanged, on the host cores, on a
    bounded sample of the workload: rounds of one step of every patch, the
    first ones, until ``budget_s`` has passed (at most 1000 rounds).  Then
    parity: each GPU result in ``gpu_results``
    ({label: (precision, E, B) per patch as float64 host arrays}) against the
    oracle.  Vacuum: K steps against one oracle step of K dt per patch (the
    exact per-mode flow; the oracle's semigroup pins cover the identity).
    With sources: one step with the step-0 sources."""
    import oracle

    workers = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
    cells = 0
    rounds = 0
    state = [([np.asarray(a, np.float32).astype(np.float64) for a in w.E0[pi]],
              [np.asarray(a, np.float32).astype(np.float64) for a in w.B0[pi]])
             for pi in range(len(w.patches))]
    t0 = time.perf_counter()
    while time.perf_counter() - t0 < budget_s and rounds < 1000:
        for pi, p in enumerate(w.patches):
            J = ro = rn = None
            if w.sources:
                J, ro, rn = w.schedule[pi].sources(rounds, dtype=np.float32)
                J = [np.asarray(a, np.float64) for a in J]
                ro, rn = np.asarray(ro, np.float64), np.asarray(rn, np.float64)
            state[pi] = oracle.psatd_step(*state[pi], J, ro, rn, d=p.d, dt=p.dt, workers=workers)
            cells += p.cells
        rounds += 1
    el = time.perf_counter() - t0
    del state
    label = label or w.name
    sample = (f"{label}: first {rounds} step(s) of its single grid" if len(w.patches) == 1 else
              f"{label}: first {rounds} step(s) of each of its {len(w.patches)} patches")
    cpu = {"value": cells / el, "unit": "cell-steps/s", "cores": workers, "kind": "oracle",
           "sample": sample + f", {el:.1f} s, scipy.fft FP64 + numpy update"}

    parity = {}
    for label, (precision, gE, gB) in gpu_results.items():
        rnd = np.float32 if precision == "fp32" else np.float64
        per_patch = []
        for pi, p in enumerate(w.patches):
            E = [np.asarray(a, rnd).astype(np.float64) for a in w.E0[pi]]
            B = [np.asarray(a, rnd).astype(np.float64) for a in w.B0[pi]]
            if w.sources:
                J, ro, rn = w.schedule[pi].sources(0, dtype=rnd)
                E, B = oracle.psatd_step(E, B, [np.asarray(a, np.float64) for a in J],
                                         np.asarray(ro, np.float64), np.asarray(rn, np.float64),
                                         d=p.d, dt=p.dt, workers=workers)
            else:
                E, B = oracle.psatd_step(E, B, d=p.d, dt=steps * p.dt, workers=workers)
            got = gE[pi] + gB[pi]
            ref = E + B
            per_patch.append((component_errors(got, ref, p.ndim),
                              sum(float(np.sum((a - b) ** 2)) for a, b in zip(got, ref)),
                              sum(float(np.sum(b * b)) for b in ref)))
        parity[label] = summarize(per_patch)
        parity[label]["steps"] = 1 if w.sources else steps
        log(f"[bench]   parity {label}: {parity[label]['max_coupled_set']:.2e} (coupled set), "
            f"{parity[label]['max_own']:.2e} (own norm), pooled {parity[label]['pooled']:.2e}")
    return cpu, parity


def host_fields(plan, tensors, patches):
    """Flat device tensors -> per patch list of float64 host arrays."""
    h = [t.detach().cpu().numpy().astype(np.float64) for t in tensors]
    return [[x[off:off + p.cells].reshape(p.shape) for x in h]
            for off, p in zip(plan.offsets, patches)]


def run_fp64(pk, w, mode, cells, steps, args, vacuum_batch):
    """The plain FP64 path on the same workload (reported beside the FP32
    one); also returns its result after the parity run (see main)."""
    import torch

    plan64 = pk.Plan(w.patches, precision="fp64", source_mode=mode, path="plain", graph=True,
                     autotune=True)
    E64, B64, J64, ro64, rn64 = device_fields(w, plan64, np.float64)
    # parity run: `steps` vacuum steps (one with sources) from the initial fields
    Ep = [t.clone() for t in E64]
    Bp = [t.clone() for t in B64]
    plan64.push(Ep, Bp, J64, ro64, rn64, steps=steps if vacuum_batch else 1)
    torch.cuda.synchronize()
    res = (host_fields(plan64, Ep, w.patches), host_fields(plan64, Bp, w.patches))
    del Ep, Bp
    s64 = min(steps, args.fp64_steps)
    log(f"[bench] timing {s64} fp64 plain steps ...")
    sec64 = time_steps(plan64, E64, B64, J64, ro64, rn64, s64, min(args.warmup, 5), vacuum_batch)
    pass64 = plan64.push_profiled(E64, B64, J64, ro64, rn64, steps=min(s64, 20)) if not vacuum_batch \
        else plan64.push_profiled(E64, B64, steps=min(s64, 20))
    fp64 = {"value": cells * s64 / sec64, "unit": "cell-steps/s", "ms_per_step": 1e3 * sec64 / s64,
            "steps": s64, "passes": {n: round(m, 5) for n, m in zip(plan64.pass_names, pass64)},
            "model_GBps": sum(plan64.pass_bytes) / (sec64 / s64) / 1e9}
    log(f"[bench]   fp64 plain: {fp64['ms_per_step']:.4f} ms/step")
    plan64.close()
    return fp64, res


def bench_decomposition(pk, args, parts=(2, 1, 2), guard=128, order=16):
    """Guard-cell decomposition of the workload's grid: cell-steps/s of the
    global grid (interior cells), beside the undecomposed plan at the same
    order, with the relative difference of the two after the timed steps."""
    import torch

    import fixtures

    steps = args.steps or 100
    w = build_inputs(args.workload, steps)
    p = w.patches[0]
    mode = "rho" if w.sources else "vacuum"
    dom = pk.Domain(len(p.shape), (p.nx, p.ny, p.nz), parts, (guard, guard, guard), p.d, p.dt,
                    precision="fp32", source_mode=mode, order=order, centered_stencil=True,
                    graph=True, autotune=True)
    npatch, local = dom.local_shape
    plan = pk.Plan(w.patches, precision="fp32", source_mode=mode, path="fused", order=order,
                   centered_stencil=True, graph=True, autotune=True)
    E, B, J, ro, rn = device_fields(w, plan, np.float32)
    E2 = [t.clone() for t in E]
    B2 = [t.clone() for t in B]

    def run_dom(n):
        for _ in range(n):
            if w.sources:
                dom.push(E2, B2, J, ro, rn, steps=1)
            else:
                dom.push(E2, B2, steps=1)

    run_dom(min(args.warmup, 5))
    torch.cuda.synchronize()
    log(f"[bench] timing {steps} decomposed steps: {npatch} patches of {local} ...")
    t0 = time.perf_counter()
    run_dom(steps)
    torch.cuda.synchronize()
    sec_dom = time.perf_counter() - t0
    sec_glob = time_steps(plan, E, B, J, ro, rn, steps, min(args.warmup, 5), not w.sources)
    # the same local patches as an ordinary batched plan (no guard exchange):
    # what the local grids cost by themselves, so that the exchange's own cost
    # is the difference
    lp = fixtures.Patch(p.ndim, local[0], local[1], local[2], p.dx, p.dy, p.dz, p.dt)
    lplan = pk.Plan([lp] * npatch, precision="fp32", source_mode=mode, path="fused", order=order,
                    centered_stencil=True, graph=True, autotune=True)
    n = lplan.total_elements
    LE = [torch.zeros(n, dtype=torch.float32, device="cuda") for _ in range(3)]
    LB = [torch.zeros(n, dtype=torch.float32, device="cuda") for _ in range(3)]
    LJ = [torch.zeros(n, dtype=torch.float32, device="cuda") for _ in range(3)] if w.sources else None
    Lro = torch.zeros(n, dtype=torch.float32, device="cuda") if w.sources else None
    Lrn = torch.zeros(n, dtype=torch.float32, device="cuda") if w.sources else None
    sec_loc = time_steps(lplan, LE, LB, LJ, Lro, Lrn, steps, min(args.warmup, 5), not w.sources)
    lplan.close()
    del LE, LB, LJ, Lro, Lrn
    diff = float(np.sqrt(sum(float(torch.sum((a.double() - b.double()) ** 2)) for a, b in zip(E + B, E2 + B2))
                         / sum(float(torch.sum(b.double() ** 2)) for b in E + B)))
    out = {"metric": "PSATD guard-cell decomposition cell-steps/s (global interior cells), 1 GPU",
           "value": w.cells * steps / sec_dom, "unit": "cell-steps/s", "n_gpus": 1, "steps": steps,
           "ms_per_step": 1e3 * sec_dom / steps, "higher_is_better": True, "dtype": "f64",
           "config": {"workload": w.name, "parts": list(parts), "guard": guard, "order": order,
                      "stencil": "centered", "patches": npatch, "local_shape": list(local),
                      "storage": "f32"},
           "undecomposed": {"value": w.cells * steps / sec_glob, "ms_per_step": 1e3 * sec_glob / steps},
           "local_patches_alone": {"ms_per_step": 1e3 * sec_loc / steps,
                                   "note": "the same local patches as a batched plan, no guard exchange"},
           "rel_l2_vs_undecomposed": diff}
    dom.close()
    plan.close()
    print(json.dumps(out), flush=True)


def bench_contrast(pk, args):
    """The contrast solvers of Table 1 beside PSATD on the workload's grid
    (FP32 storage, J sources, each at its Courant-limited time step): ms per
    step, cell-steps/s, the model's HBM bytes, and the cost ratio of PSATD
    to each (the paper's xi, per step at equal resolution, Sec. IV.C)."""
    import torch

    steps = args.steps or 200
    warm = min(args.warmup, 10)
    w = build_inputs(args.workload, steps)
    p = w.patches[0]
    if p.ndim != 2 or not w.sources:
        raise SystemExit("--contrast times the 2D workload with sources (workload 1)")
    cells = w.cells
    dx = p.dx
    out = {"metric": "field-step time of PSATD and the contrast solvers (Table 1), 1 GPU",
           "unit": "ms/step", "n_gpus": 1, "steps": steps, "warmup": warm, "dtype": "f64",
           "config": {"workload": w.name, "storage": "f32", "sources": "J"}, "solvers": {}}

    def record(name, sec, dt, bytes_per_cell, kernels):
        ms = 1e3 * sec / steps
        out["solvers"][name] = {"ms_per_step": ms, "cell_steps_per_s": cells * steps / sec,
                                "dt_over_dx": dt / dx, "model_bytes_per_cell": bytes_per_cell,
                                "model_GBps": bytes_per_cell * cells / (ms * 1e-3) / 1e9,
                                "kernels": kernels}
        log(f"[bench] {name}: {ms:.3f} ms/step")

    def psatd_like(name, mode, dt, **kw):
        pp = fixtures_patch(p, dt)
        plan = pk.Plan([pp], precision="fp32", source_mode=mode, path="fused", graph=True,
                       autotune=True, **kw)
        E, B, J, ro, rn = device_fields(w, plan, np.float32)
        if mode == "j":
            ro = rn = None
        sec = time_steps(plan, E, B, J, ro, rn, steps, warm, False)
        nin = 11 if mode == "rho" else 9
        record(name, sec, dt, 4 * (2 * nin + (nin + 6) + 2 * 6), plan.pass_names)
        plan.close()
        del E, B, J, ro, rn

    def fdtd(name, scheme, dt):
        pp = fixtures_patch(p, dt)
        f = pk.Fdtd(scheme, pp, precision="fp32", source_mode="j")
        plan_like = type("P", (), {"total_elements": cells, "offsets": [0]})
        E, B, J, _, _ = device_fields(w, plan_like, np.float32)

        def run(n):
            for _ in range(n):
                f.push(E, B, J)
        run(warm)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        run(steps)
        torch.cuda.synchronize()
        sec = time.perf_counter() - t0
        # Faraday: E, B in, B out; Ampere: B, E, J in, E out
        record(name, sec, dt, 4 * ((6 + 3) + (9 + 3)), ["faraday", "ampere"])
        f.close()
        del E, B, J

    psatd_like("psatd_rho", "rho", p.dt)
    psatd_like("psatd_j", "j", p.dt)
    psatd_like("psatd_j_generic", "j", p.dt, generic_kernels=True)
    psatd_like("pstd", "j", np.sqrt(2.0) / np.pi * dx, pstd=True)
    fdtd("yee", "yee", dx / np.sqrt(2.0))
    fdtd("ckc", "ckc", dx)
    t = {k: v["ms_per_step"] for k, v in out["solvers"].items()}
    out["xi_psatd_over_yee"] = t["psatd_rho"] / t["yee"]
    out["xi_psatd_over_ckc"] = t["psatd_rho"] / t["ckc"]
    out["pstd_over_psatd_j_generic"] = t["pstd"] / t["psatd_j_generic"]
    # cost per unit of simulated time, each at its own Courant-limited dt
    out["cost_per_sim_time_vs_psatd"] = {
        k: (v["ms_per_step"] / v["dt_over_dx"]) / (t["psatd_rho"] / out["solvers"]["psatd_rho"]["dt_over_dx"])
        for k, v in out["solvers"].items()}
    print(json.dumps(out), flush=True)


def fixtures_patch(p, dt):
    import fixtures
    return fixtures.workloads.Patch(p.ndim, p.nx, p.ny, p.nz, p.dx, p.dy, p.dz, float(dt))


def reap_children():
    """End any child process this run left behind (e.g. library worker pools),
    so that the benchmark leaves nothing running when it returns."""
    try:
        import psutil
    except ImportError:
        return
    kids = psutil.Process().children(recursive=True)
    for c in kids:
        log(f"[bench] ending leftover child process {c.pid} ({c.name()})")
        c.terminate()
    _gone, alive = psutil.wait_procs(kids, timeout=5)
    for c in alive:
        c.kill()


def pass_report(plan, pass_ms):
    names, pbytes = plan.pass_names, plan.pass_bytes
    grids = plan_grids(plan)
    passes = {n: {"ms": round(m, 5), "model_GBps": round(b / (m * 1e-3) / 1e9, 1),
                  "model_bytes": b, "grid": grids.get(n)} for n, m, b in zip(names, pass_ms, pbytes)}
    dom = int(np.argmax(pass_ms))
    return passes, names[dom], pbytes[dom] / (pass_ms[dom] * 1e-3) / 1e9, sum(pbytes)


def time_source_generator(w, steps):
    """ms per step of the fixture's GPU source generator (J^{n+1/2} and
    rho^{n+1} of one patch formed on the device, rho^n kept from the step
    before), timed on its own: the timed field steps reuse one resident set
    of sources, whose values do not change the cost of the step."""
    import torch
    from fixtures.device import DeviceSourceSchedule
    gen = DeviceSourceSchedule(w.schedule[0], torch)
    n = gen.cells
    J = [torch.empty(n, dtype=torch.float32, device="cuda") for _ in range(3)]
    a = torch.empty(n, dtype=torch.float32, device="cuda")
    b = torch.empty(n, dtype=torch.float32, device="cuda")
    gen.advance_into(0, J, a, b)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(1, steps + 1):
        gen.advance_into(k, J, a, b)
        a, b = b, a
    torch.cuda.synchronize()
    ms = 1e3 * (time.perf_counter() - t0) / steps
    del gen, J, a, b
    return {"kind": "fixture (torch elementwise kernels on the GPU, FP64 then rounded)",
            "ms_per_step": ms, "steps": steps}


def result_line(w_name, cells, steps, args, ms_step, value, cfg, dom_name, achieved, step_bytes,
                passes, fp64, parity, cpu, sources=None):
    traffic = measured_traffic(w_name, dom_name)
    return {
        "metric": METRIC,
        "value": value,
        "unit": "cell-steps/s",
        "n_gpus": 1,
        "steps": steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic (seeded laser and harmonic combs; current sheet with continuity-consistent rho)",
        "config": cfg,
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": PEAK_HBM_GBS, "unit": "GB/s",
                     "frac": achieved / PEAK_HBM_GBS, "traffic": traffic, "kernel": dom_name},
        "step_model_GBps": step_bytes / (ms_step * 1e-3) / 1e9,
        "step_model_frac": step_bytes / (ms_step * 1e-3) / 1e9 / PEAK_HBM_GBS,
        "passes": passes,
        "fp64_plain": fp64,
        "parity": parity,
        "cpu_baseline": cpu,
        "source_generator": sources,
    }


def bench_large_3d(pk, args, steps):
    """Workload 4 (1024 x 1024 x 512 with sources): inputs built on the GPU
    from the workload's seeded parameters (fixtures.device); parity and the
    cpu_baseline on the same-seed 64^3 run."""
    import torch

    import fixtures
    from fixtures.device import workload4_device

    log("[bench] building workload 4 inputs on the GPU ...")
    t = time.time()
    p, E, B, J, ro, rn = workload4_device(torch)
    torch.cuda.synchronize()
    cells = p.cells
    log(f"[bench]   {fixtures.CONFIG_NAMES[4]}: {cells} cells, {time.time() - t:.1f} s")
    plan = fp32_plan(pk, args, [p], "rho")
    log("[bench] fp32 fused plan:\n" + plan.info)
    log(f"[bench] timing {steps} fp32 steps (+{args.warmup} warmup) ...")
    sec = time_steps(plan, E, B, J, ro, rn, steps, args.warmup, False)
    ms_step = 1e3 * sec / steps
    value = cells * steps / sec
    log(f"[bench]   {ms_step:.4f} ms/step, {value:.4e} cell-steps/s")
    pass_ms = plan.push_profiled(E, B, J, ro, rn, steps=min(steps, 20))
    passes, dom_name, achieved, step_bytes = pass_report(plan, pass_ms)
    plan.close()
    del E, B, J, ro, rn
    torch.cuda.empty_cache()
    fp64 = None
    if not args.skip_fp64:
        p, E, B, J, ro, rn = workload4_device(torch, dtype=torch.float64)
        plan64 = pk.Plan([p], precision="fp64", source_mode="rho", path="plain", graph=True,
                         autotune=True)
        s64 = min(steps, args.fp64_steps)
        log(f"[bench] timing {s64} fp64 plain steps ...")
        sec64 = time_steps(plan64, E, B, J, ro, rn, s64, min(args.warmup, 5), False)
        pass64 = plan64.push_profiled(E, B, J, ro, rn, steps=min(s64, 10))
        fp64 = {"value": cells * s64 / sec64, "unit": "cell-steps/s", "ms_per_step": 1e3 * sec64 / s64,
                "steps": s64, "passes": {n: round(m, 5) for n, m in zip(plan64.pass_names, pass64)},
                "model_GBps": sum(plan64.pass_bytes) / (sec64 / s64) / 1e9}
        log(f"[bench]   fp64 plain: {fp64['ms_per_step']:.4f} ms/step")
        plan64.close()
        del E, B, J, ro, rn
        torch.cuda.empty_cache()
    cpu, parity = None, {}
    if not args.no_cpu_baseline:
        ws = fixtures.workload(4, shape=(64, 64, 64))
        res = {}
        for precision, path, dt in (("fp32", "fused", np.float32), ("fp64", "plain", np.float64)):
            pl = pk.Plan(ws.patches, precision=precision, source_mode="rho", path=path)
            Es, Bs, Js, ros, rns = device_fields(ws, pl, dt)
            pl.push(Es, Bs, Js, ros, rns, steps=1)
            torch.cuda.synchronize()
            res[f"{precision}_{path}_64cubed_same_seed"] = (precision, host_fields(pl, Es, ws.patches),
                                                             host_fields(pl, Bs, ws.patches))
            pl.close()
        log(f"[bench] oracle on host cores (~{args.cpu_budget:.0f} s budget), 64^3 same-seed run ...")
        cpu, parity = oracle_leg(ws, args.cpu_budget, res, 1,
                                 label=f"{fixtures.CONFIG_NAMES[4]} recipe and seed on a 64x64x64 grid")
    cfg = {"workload": fixtures.CONFIG_NAMES[4], "cells": cells, "patches": 1,
           "steps_per_config": 100, "source_form": "rho", "storage": "f32", "arithmetic": "f64",
           "path": "fused", "graph": True,
           "autotune": "saved choices" if args.tuning_in else True, "inputs": "built on the GPU"}
    out = result_line(fixtures.CONFIG_NAMES[4], cells, steps, args, ms_step, value, cfg, dom_name,
                      achieved, step_bytes, passes, fp64, parity, cpu)
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--workload", type=int, default=None,
                    help="workload index (default: 3, the batched patches; 1, the 4096 x 4096 grid, "
                         "for --decomposition and --contrast)")
    ap.add_argument("--fp64-steps", type=int, default=100)
    ap.add_argument("--cpu-budget", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-calibration-mib", type=int, default=0,
                    help="first run one device-to-device copy of this many MiB (a kernel of "
                         "known traffic, to scale rocprofv3 FETCH_SIZE / WRITE_SIZE)")
    ap.add_argument("--skip-fp64", action="store_true")
    ap.add_argument("--tuning-out", metavar="PATH",
                    help="save the timed plan's kernel choices (psatd_plan_tuning) to PATH")
    ap.add_argument("--tuning-in", metavar="PATH",
                    help="build the timed plan from kernel choices saved by --tuning-out "
                         "instead of autotuning it")
    ap.add_argument("--decomposition", action="store_true",
                    help="instead of the default line: time the guard-cell domain decomposition "
                         "(2 x 2 boxes, 128 guard cells, centered order 16) on the same workload")
    ap.add_argument("--contrast", action="store_true",
                    help="instead of the default line: time PSATD beside the contrast solvers "
                         "(PSTD, Yee, CKC) on the workload's grid")
    ap.add_argument("--ingest-traffic", nargs=2, metavar=("FETCH_CSV", "WRITE_CSV"),
                    help="no run: store HBM bytes per pass from two rocprofv3 --pmc counter "
                         "files (FETCH_SIZE, WRITE_SIZE) of this script, scaled by its "
                         "calibration copy (--copy-calibration-mib, default 1024)")
    args = ap.parse_args()
    if args.workload is None:
        args.workload = 1 if (args.decomposition or args.contrast) else 3
    if (args.decomposition or args.contrast) and args.workload not in (0, 1, 2):
        print("--decomposition and --contrast take a single-grid workload (0, 1 or 2)", file=sys.stderr)
        sys.exit(2)
    if args.ingest_traffic:
        data = ingest_traffic(*args.ingest_traffic, args.workload, args.copy_calibration_mib or 1024)
        print(json.dumps(data, indent=1, sort_keys=True))
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only: the library has no multi-GPU path "
              f"(asked for --gpus {args.gpus}); use --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_1608_05739_amd as pk

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    if args.copy_calibration_mib > 0:
        n = args.copy_calibration_mib * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.float32, device="cuda:0")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        log(f"[bench] calibration copy: {args.copy_calibration_mib} MiB read + written")
        del src, dst
    index = args.workload
    if args.decomposition:
        return bench_decomposition(pk, args)
    if args.contrast:
        return bench_contrast(pk, args)
    default_steps = {0: 100, 1: 1000, 2: 200, 3: 500, 4: 100}[index]
    steps = args.steps if args.steps is not None else default_steps
    if index == 4:
        return bench_large_3d(pk, args, steps)
    w = build_inputs(index, steps)
    mode = "rho" if w.sources else "vacuum"
    vacuum_batch = not w.sources
    cells = w.cells

    # ------------------------------------------------ FP32 storage, fused path
    plan = fp32_plan(pk, args, w.patches, mode)
    log("[bench] fp32 fused plan:\n" + plan.info)
    E, B, J, ro, rn = device_fields(w, plan, np.float32)
    # parity run of the timed configuration (the oracle leg checks it): the
    # run's step count in vacuum, one step with sources
    Ep = [t.clone() for t in E]
    Bp = [t.clone() for t in B]
    plan.push(Ep, Bp, J, ro, rn, steps=steps if vacuum_batch else 1)
    torch.cuda.synchronize()
    res32 = (host_fields(plan, Ep, w.patches), host_fields(plan, Bp, w.patches))
    del Ep, Bp
    log(f"[bench] timing {steps} fp32 steps (+{args.warmup} warmup) ...")
    sec = time_steps(plan, E, B, J, ro, rn, steps, args.warmup, vacuum_batch)
    ms_step = 1e3 * sec / steps
    value = cells * steps / sec
    log(f"[bench]   {ms_step:.4f} ms/step, {value:.4e} cell-steps/s")
    prof_steps = min(steps, 200)
    pass_ms = plan.push_profiled(E, B, J, ro, rn, steps=prof_steps) if not vacuum_batch else \
        plan.push_profiled(E, B, steps=prof_steps)
    passes, dom_name, achieved, step_bytes = pass_report(plan, pass_ms)
    log(f"[bench]   passes: {passes}")
    plan.close()
    del E, B, J, ro, rn

    sources = None
    if w.sources and len(w.patches) == 1:
        sources = time_source_generator(w, min(steps, 100))
        log(f"[bench]   source generator (fixture, GPU): {sources['ms_per_step']:.4f} ms/step")

    # ------------------------------------------------ FP64 storage, plain path
    fp64, res64 = None, None
    if not args.skip_fp64:
        fp64, res64 = run_fp64(pk, w, mode, cells, steps, args, vacuum_batch)

    # ------------------------------------------------ oracle leg: cpu_baseline + parity
    cpu, parity = None, {}
    if not args.no_cpu_baseline:
        log(f"[bench] oracle on host cores (~{args.cpu_budget:.0f} s budget) ...")
        results = {"fp32_fused": ("fp32",) + res32}
        if res64 is not None:
            results["fp64_plain"] = ("fp64",) + res64
        cpu, parity = oracle_leg(w, args.cpu_budget, results, steps)
        log(f"[bench]   cpu {cpu['value']:.4e} cell-steps/s on {cpu['cores']} threads")

    nin = 11 if w.sources else 6
    ws_bytes = sum(p.cells * 4 * nin * (3 if p.ndim == 3 else 2) for p in w.patches)
    cfg = {"workload": w.name, "cells": cells, "patches": len(w.patches),
           "steps_per_config": default_steps, "source_form": mode, "storage": "f32",
           "arithmetic": "f64", "path": "fused", "graph": True,
           "autotune": "saved choices" if args.tuning_in else True,
           "working_set_bytes": ws_bytes}
    out = result_line(w.name, cells, steps, args, ms_step, value, cfg, dom_name, achieved,
                      step_bytes, passes, fp64, parity, cpu, sources)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    try:
        main()
    finally:
        reap_children()
