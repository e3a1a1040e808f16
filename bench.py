"""Benchmark of the PSATD field step on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload 1]

A step is one full pass of the hot path (x r2c FFT of every input, fused z
pass with the per-mode update, x c2r FFT of E and B) over the workload's
synthetic fields, inputs resident in HBM.  Workload 1 (default): 2D 4096 x
4096, J and rho sources (rho form), FP32 storage.  Prints ONE JSON line on
stdout; progress goes to stderr.

The line also reports, on the same workload: the plain FP64 path, the
per-pass durations (HIP events on the launch stream), the roofline of the
dominant kernel, a one-step parity check against the FP64 oracle, and the
oracle's own throughput on the host cores (cpu_baseline).
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


# Device-code sources of the kernels the stored traffic describes (the 4096 x
# 4096 passes); a change to any of them makes the stored counters stale.
KERNEL_SOURCES = ("fast2d.hip", "fast2d.hpp", "fft.hpp", "groups.hpp", "update.hpp", "internal.hpp")


def kernel_source_hash():
    h = hashlib.sha256()
    for name in KERNEL_SOURCES:
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


PASS_OF_KERNEL = (("x_fwd_kernel", "x_r2c_fwd"), ("z_fused_kernel", "z_fused"),
                  ("x_inv_kernel", "x_c2r_inv"))


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
                    out.append((r["Kernel_Name"], float(r["Counter_Value"])))
        return out

    fetch, write = rows(fetch_csv, "FETCH_SIZE"), rows(write_csv, "WRITE_SIZE")
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
    for key, pname in PASS_OF_KERNEL:
        fv = [v for n, v in fetch if key in n]
        wv = [v for n, v in write if key in n]
        if not fv or not wv:
            continue
        f_kib, w_kib = sum(fv) / len(fv), sum(wv) / len(wv)
        data[f"{name}:{pname}"] = {
            "bytes_per_launch": (f_kib * fscale + w_kib * wscale) * 1024.0,
            "fetch_kib": f_kib, "write_kib": w_kib, "fetch_scale": fscale, "write_scale": wscale,
            "dispatches": len(fv), "source_hash": h}
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


def cpu_baseline(w, budget_s, rounded_dtype):
    """The FP64 oracle on the host cores, on the first steps of the same workload."""
    import oracle

    workers = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
    cells = 0
    steps_done = 0
    t0 = time.perf_counter()
    first = None
    for pi, p in enumerate(w.patches):
        E = [np.asarray(a, rounded_dtype).astype(np.float64) for a in w.E0[pi]]
        B = [np.asarray(a, rounded_dtype).astype(np.float64) for a in w.B0[pi]]
        n = 0
        while True:
            if w.sources:
                J, ro, rn = w.schedule[pi].sources(0, dtype=rounded_dtype)
                J = [np.asarray(a, np.float64) for a in J]
                ro, rn = np.asarray(ro, np.float64), np.asarray(rn, np.float64)
            else:
                J = ro = rn = None
            E, B = oracle.psatd_step(E, B, J, ro, rn, d=p.d, dt=p.dt, workers=workers)
            n += 1
            cells += p.cells
            if pi == 0 and n == 1:
                first = (E, B)
            if time.perf_counter() - t0 > budget_s or n >= 1000:
                break
            if len(w.patches) > 1 and n >= 1:
                break
        steps_done = max(steps_done, n)
        if time.perf_counter() - t0 > budget_s:
            break
    el = time.perf_counter() - t0
    return cells / el, el, workers, steps_done, first


def run_fp64(pk, w, mode, cells, steps, args, vacuum_batch):
    """The plain FP64 path on the same workload (reported beside the FP32 one)."""
    import torch

    plan64 = pk.Plan(w.patches, precision="fp64", source_mode=mode, path="plain", graph=True,
                     autotune=True)
    E64, B64, J64, ro64, rn64 = device_fields(w, plan64, np.float64)
    E64_1 = [t.clone() for t in E64]
    B64_1 = [t.clone() for t in B64]
    plan64.push(E64_1, B64_1, J64, ro64, rn64, steps=1)
    torch.cuda.synchronize()
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
    return fp64


def bench_decomposition(pk, args, parts=(2, 1, 2), guard=128, order=16):
    """Guard-cell decomposition of the workload's grid: cell-steps/s of the
    global grid (interior cells), beside the undecomposed plan at the same
    order, with the relative difference of the two after the timed steps."""
    import torch

    steps = args.steps or 100
    w = build_inputs(args.workload, steps)
    p = w.patches[0]
    mode = "rho" if w.sources else "vacuum"
    dom = pk.Domain(len(p.shape), (p.nx, p.ny, p.nz), parts, (guard, guard, guard), p.d, p.dt,
                    precision="fp32", source_mode=mode, order=order, centered_stencil=True,
                    graph=True)
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
    diff = float(np.sqrt(sum(float(torch.sum((a.double() - b.double()) ** 2)) for a, b in zip(E + B, E2 + B2))
                         / sum(float(torch.sum(b.double() ** 2)) for b in E + B)))
    out = {"metric": "PSATD guard-cell decomposition cell-steps/s (global interior cells), 1 GPU",
           "value": w.cells * steps / sec_dom, "unit": "cell-steps/s", "n_gpus": 1, "steps": steps,
           "ms_per_step": 1e3 * sec_dom / steps, "higher_is_better": True, "dtype": "f64",
           "config": {"workload": w.name, "parts": list(parts), "guard": guard, "order": order,
                      "stencil": "centered", "patches": npatch, "local_shape": list(local),
                      "storage": "f32"},
           "undecomposed": {"value": w.cells * steps / sec_glob, "ms_per_step": 1e3 * sec_glob / steps},
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


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--workload", type=int, default=1)
    ap.add_argument("--fp64-steps", type=int, default=100)
    ap.add_argument("--cpu-budget", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-calibration-mib", type=int, default=0,
                    help="first run one device-to-device copy of this many MiB (a kernel of "
                         "known traffic, to scale rocprofv3 FETCH_SIZE / WRITE_SIZE)")
    ap.add_argument("--skip-fp64", action="store_true")
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
    w = build_inputs(index, steps)
    mode = "rho" if w.sources else "vacuum"
    vacuum_batch = not w.sources
    cells = w.cells

    # ------------------------------------------------ FP32 storage, fused path
    # radix-4 generic line passes where every generic line is short (<= 256)
    radix4 = max(max(p.nx // 2, p.ny) for p in w.patches) <= 256
    plan = pk.Plan(w.patches, precision="fp32", source_mode=mode, path="fused", graph=True,
                   autotune=True, radix4_lines=radix4)
    log("[bench] fp32 fused plan:\n" + plan.info)
    E, B, J, ro, rn = device_fields(w, plan, np.float32)
    # one-step parity spot check on the same inputs (before timing mutates E, B)
    E1 = [t.clone() for t in E]
    B1 = [t.clone() for t in B]
    plan.push(E1, B1, J, ro, rn, steps=1)
    torch.cuda.synchronize()
    log(f"[bench] timing {steps} fp32 steps (+{args.warmup} warmup) ...")
    sec = time_steps(plan, E, B, J, ro, rn, steps, args.warmup, vacuum_batch)
    ms_step = 1e3 * sec / steps
    value = cells * steps / sec
    log(f"[bench]   {ms_step:.4f} ms/step, {value:.4e} cell-steps/s")
    prof_steps = min(steps, 200)
    pass_ms = plan.push_profiled(E, B, J, ro, rn, steps=prof_steps) if not vacuum_batch else \
        plan.push_profiled(E, B, steps=prof_steps)
    names, pbytes = plan.pass_names, plan.pass_bytes
    grids = plan_grids(plan)
    passes = {n: {"ms": round(m, 5), "model_GBps": round(b / (m * 1e-3) / 1e9, 1),
                  "model_bytes": b, "grid": grids.get(n)} for n, m, b in zip(names, pass_ms, pbytes)}
    dom = int(np.argmax(pass_ms))
    achieved = pbytes[dom] / (pass_ms[dom] * 1e-3) / 1e9
    step_bytes = sum(pbytes)
    log(f"[bench]   passes: {passes}")
    traffic = measured_traffic(w.name, names[dom])

    # ------------------------------------------------ FP64 storage, plain path
    fp64 = None
    if not args.skip_fp64:
        fp64 = run_fp64(pk, w, mode, cells, steps, args, vacuum_batch)

    # ------------------------------------------------ oracle: CPU baseline + parity
    cpu = None
    parity = {}
    if not args.no_cpu_baseline:
        log(f"[bench] oracle on host cores (~{args.cpu_budget:.0f} s budget) ...")
        v, el, workers, nst, first = cpu_baseline(w, args.cpu_budget, np.float32)
        sample = (f"{w.name}: first {nst} step(s) of patch 0" if len(w.patches) == 1 else
                  f"{w.name}: 1 step of the first patches within the budget")
        cpu = {"value": v, "unit": "cell-steps/s", "cores": workers, "kind": "oracle",
               "sample": sample + f", {el:.1f} s, scipy.fft FP64 + numpy update"}
        if first is not None:
            p0 = w.patches[0]

            def rel(gpuE, gpuB, plan_):
                got = [t.detach().cpu().numpy().astype(np.float64)[:p0.cells].reshape(p0.shape)
                       for t in gpuE + gpuB]
                ref = first[0] + first[1]
                return float(np.sqrt(sum(np.sum((g - r) ** 2) for g, r in zip(got, ref))
                                     / sum(np.sum(r * r) for r in ref)))
            parity["fp32_fused_1step_rel_l2"] = rel(E1, B1, plan)
        log(f"[bench]   cpu {v:.4e} cell-steps/s on {workers} threads; parity {parity}")

    cfg = {"workload": w.name, "cells": cells, "patches": len(w.patches), "steps_per_config": default_steps,
           "source_form": mode, "storage": "f32", "arithmetic": "f64", "path": "fused",
           "graph": True, "autotune": True, "radix4_lines": radix4}
    out = {
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
        "data": "synthetic (seeded laser + harmonic comb, current sheet with continuity-consistent rho)",
        "config": cfg,
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": PEAK_HBM_GBS, "unit": "GB/s",
                     "frac": achieved / PEAK_HBM_GBS, "traffic": traffic, "kernel": names[dom]},
        "step_model_GBps": step_bytes / (ms_step * 1e-3) / 1e9,
        "step_model_frac": step_bytes / (ms_step * 1e-3) / 1e9 / PEAK_HBM_GBS,
        "passes": passes,
        "fp64_plain": fp64,
        "parity": parity,
        "cpu_baseline": cpu,
    }
    plan.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
