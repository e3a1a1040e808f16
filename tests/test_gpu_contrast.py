"""GPU contrast solvers against the oracle: Yee and order-p FDTD, CKC
(psatd_fdtd_*) and PSTD (psatd_plan with PSATD_FLAG_PSTD), Sec. III.A and
Table 1.  Element-by-element relative L2 on the same seeded inputs: FP64 to
1e-12, FP32 to 1e-5; ragged sizes (rows that end inside a workgroup, lengths
that are not powers of two for FDTD); full 4096 x 4096 runs; and the GPU
reproducing Table 1's dispersion directly (a Yee lattice mode advances by
the Yee phase, CKC moves an axis-aligned pulse by exactly one cell per step).
"""

import numpy as np
import pytest

import fixtures
import paper_1608_05739_amd as pk
from gpu_support import field_error, rounded, say
from oracle import contrast as C
from oracle import dispersion as D

pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-12, "fp32": 1e-5}


def _dev(a, precision):
    import torch
    dt = np.float32 if precision == "fp32" else np.float64
    return torch.from_numpy(np.ascontiguousarray(a, dtype=dt).ravel()).to("cuda:0")


def _host(t, shape):
    return t.detach().cpu().numpy().astype(np.float64).reshape(shape)


def _inputs(index, shape, frac, seed_sources=True):
    """Seeded fields and sources of a workload at ``shape``, with dt = frac * dx."""
    w = fixtures.workload(index, shape=shape, steps=4)
    p0 = w.patches[0]
    p = fixtures.workloads.Patch(p0.ndim, p0.nx, p0.ny, p0.nz, p0.dx, p0.dy, p0.dz,
                                 frac * p0.dx)
    sched = w.schedule[0] if (seed_sources and w.sources) else None
    return p, w.E0[0], w.B0[0], sched


def _sources(sched, n, precision):
    J, _, _ = sched.sources(n, dtype=np.float32 if precision == "fp32" else np.float64)
    return J


def _gpu_fdtd(scheme, order, p, E0, B0, sched, steps, precision):
    import torch
    f = pk.Fdtd(scheme, p, precision=precision, source_mode="j" if sched else "vacuum",
                order=order)
    E = [_dev(a, precision) for a in E0]
    B = [_dev(a, precision) for a in B0]
    for n in range(steps):
        if sched is not None:
            f.push(E, B, [_dev(x, precision) for x in _sources(sched, n, precision)])
        else:
            f.push(E, B)
    torch.cuda.synchronize()
    f.close()
    return [_host(t, p.shape) for t in E + B]


def _oracle_fdtd(scheme, order, p, E0, B0, sched, steps, precision):
    E = [rounded(a, precision) for a in E0]
    B = [rounded(a, precision) for a in B0]
    for n in range(steps):
        J = None
        if sched is not None:
            J = [np.asarray(x, np.float64) for x in _sources(sched, n, precision)]
        E, B = C.fdtd_step(E, B, J, d=p.d, dt=p.dt, scheme=scheme, order=order)
    return E + B


FDTD_CASES = [
    # scheme, order, workload, shape, dt / dx, precision
    ("yee", 2, 1, (80, 300), 0.5, "fp64"),
    ("yee", 2, 1, (80, 300), 0.5, "fp32"),
    ("ckc", 2, 1, (72, 260), 0.9, "fp64"),
    ("ckc", 2, 1, (72, 260), 1.0, "fp32"),
    ("yee", 8, 1, (64, 96), 0.3, "fp64"),
    ("yee", 2, 2, (20, 12, 36), 0.4, "fp64"),
    ("yee", 2, 2, (20, 12, 36), 0.4, "fp32"),
    ("yee", 4, 2, (24, 18, 30), 0.3, "fp64"),
]


@pytest.mark.parametrize("scheme,order,index,shape,frac,precision", FDTD_CASES)
@pytest.mark.parametrize("sources", [False, True])
def test_fdtd_matches_oracle(scheme, order, index, shape, frac, precision, sources):
    p, E0, B0, sched = _inputs(index, shape, frac, sources)
    steps = 4
    say(f"fdtd {scheme} p={order} {shape} dt={frac}dx {precision} sources={sources}")
    got = _gpu_fdtd(scheme, order, p, E0, B0, sched, steps, precision)
    ref = _oracle_fdtd(scheme, order, p, E0, B0, sched, steps, precision)
    err = field_error(got, ref, precision=precision)
    assert err < TOL[precision]


def test_fdtd_offset_and_neighbours_untouched():
    # a patch at an element offset: nothing outside [offset, offset + cells) changes
    import torch
    p, E0, B0, _ = _inputs(1, (40, 50), 0.5, False)
    off = 7
    f = pk.Fdtd("yee", p, precision="fp64", offset=off)
    pad = 13
    E, B = [], []
    for a in E0 + B0:
        buf = np.full(off + a.size + pad, -3.25)
        buf[off:off + a.size] = a.ravel()
        (E if len(E) < 3 else B).append(torch.from_numpy(buf).to("cuda:0"))
    f.push(E, B, steps=2)
    torch.cuda.synchronize()
    ref = _oracle_fdtd("yee", 2, p, E0, B0, None, 2, "fp64")
    got = []
    for t in E + B:
        h = t.cpu().numpy()
        assert np.all(h[:off] == -3.25) and np.all(h[off + p.cells:] == -3.25)
        got.append(h[off:off + p.cells].reshape(p.shape))
    err = field_error(got, ref, precision="fp64")
    assert err < 1e-12


def _gpu_pstd(p, E0, B0, sched, steps, precision, path, order=0):
    import torch
    plan = pk.Plan([p], precision=precision, source_mode="j" if sched else "vacuum", path=path,
                   order=order, pstd=True)
    assert "solver=pstd" in plan.info
    E = [_dev(a, precision) for a in E0]
    B = [_dev(a, precision) for a in B0]
    for n in range(steps):
        if sched is not None:
            plan.push(E, B, [_dev(x, precision) for x in _sources(sched, n, precision)])
        else:
            plan.push(E, B)
    torch.cuda.synchronize()
    plan.close()
    return [_host(t, p.shape) for t in E + B]


def _oracle_pstd(p, E0, B0, sched, steps, precision, order=0):
    E = [rounded(a, precision) for a in E0]
    B = [rounded(a, precision) for a in B0]
    for n in range(steps):
        J = None
        if sched is not None:
            J = [np.asarray(x, np.float64) for x in _sources(sched, n, precision)]
        E, B = C.pstd_step(E, B, J, d=p.d, dt=p.dt, order=order)
    return E + B


PSTD_CASES = [
    # workload, shape, dt / dx, precision, path, order
    (1, (96, 128), 0.4, "fp64", "fused", 0),
    (1, (96, 128), 0.4, "fp32", "fused", 0),
    (1, (96, 128), 0.4, "fp64", "plain", 0),
    (1, (64, 72), 0.3, "fp64", "fused", 8),
    (2, (24, 18, 32), 0.25, "fp64", "fused", 0),
    (2, (24, 18, 32), 0.25, "fp32", "plain", 0),
]


@pytest.mark.parametrize("index,shape,frac,precision,path,order", PSTD_CASES)
@pytest.mark.parametrize("sources", [False, True])
def test_pstd_matches_oracle(index, shape, frac, precision, path, order, sources):
    p, E0, B0, sched = _inputs(index, shape, frac, sources)
    steps = 3
    say(f"pstd {shape} dt={frac}dx {precision} {path} p={order} sources={sources}")
    got = _gpu_pstd(p, E0, B0, sched, steps, precision, path, order)
    ref = _oracle_pstd(p, E0, B0, sched, steps, precision, order)
    err = field_error(got, ref, precision=precision)
    assert err < TOL[precision]


def test_pstd_courant_condition_is_enforced():
    p, _, _, _ = _inputs(1, (64, 64), 0.5, False)   # above sqrt(2)/pi
    with pytest.raises(pk.PsatdError, match="Courant"):
        pk.Plan([p], precision="fp64", pstd=True)


def test_gpu_yee_lattice_mode_advances_by_the_table1_phase():
    # s-pol Yee eigenmode; after n steps it is the initial mode times exp(-i w n dt)
    import torch
    nx, nz, dx, dz = 64, 48, 0.1, 0.1
    dt = 0.6 * dx
    Ey, Bx, Bz, w = D.yee_lattice_mode(nx, nz, 5, -3, dx, dz, dt)
    p = fixtures.workloads.Patch(2, nx, 1, nz, dx, 1.0, dz, dt)
    zero = np.zeros((nz, nx))
    E = [_dev(a, "fp64") for a in (zero, Ey.real, zero)]
    B = [_dev(a, "fp64") for a in (Bx.real, zero, Bz.real)]
    f = pk.Fdtd("yee", p, precision="fp64")
    n = 40
    f.push(E, B, steps=n)
    torch.cuda.synchronize()
    ph = np.exp(-1j * w * n * dt)
    assert np.max(np.abs(_host(E[1], (nz, nx)) - (Ey * ph).real)) < 1e-11
    assert np.max(np.abs(_host(B[0], (nz, nx)) - (Bx * ph).real)) < 1e-11
    assert np.max(np.abs(_host(B[2], (nz, nx)) - (Bz * ph).real)) < 1e-11
    f.close()


def test_gpu_ckc_is_exact_along_x_at_courant_one():
    # Sec. III.A: dispersion-free along the axes at c dt = dx = dz
    import torch
    n = 300
    rng = np.random.default_rng(4)
    f1 = np.convolve(rng.normal(size=n), np.ones(7) / 7, mode="same")
    dx = 0.05
    p = fixtures.workloads.Patch(2, n, 1, 16, dx, 1.0, dx, dx)
    zero = np.zeros((16, n))
    E = [_dev(a, "fp64") for a in (zero, zero, np.tile(f1[None, :], (16, 1)))]
    B = [_dev(a, "fp64") for a in (zero, -np.tile(np.roll(f1, -1)[None, :], (16, 1)), zero)]
    f = pk.Fdtd("ckc", p, precision="fp64")
    f.push(E, B, steps=25)
    torch.cuda.synchronize()
    assert np.max(np.abs(_host(E[2], (16, n)) - np.tile(np.roll(f1, 25)[None, :], (16, 1)))) < 1e-13
    f.close()


@pytest.mark.parametrize("scheme,frac", [("yee", 0.7), ("ckc", 1.0)])
def test_fdtd_fullsize_4096_fp32_vs_oracle(scheme, frac):
    # the contrast at the headline size: 2 steps with sources
    p, E0, B0, sched = _inputs(1, None, frac, True)
    say(f"fdtd {scheme} full size {p.shape} fp32, 2 steps")
    got = _gpu_fdtd(scheme, 2, p, E0, B0, sched, 2, "fp32")
    ref = _oracle_fdtd(scheme, 2, p, E0, B0, sched, 2, "fp32")
    err = field_error(got, ref)
    assert err < 1e-5


def test_pstd_fullsize_4096_fp32_vs_oracle():
    p, E0, B0, sched = _inputs(1, None, 0.4, True)
    say(f"pstd full size {p.shape} fp32 fused, 1 step")
    got = _gpu_pstd(p, E0, B0, sched, 1, "fp32", "fused")
    ref = _oracle_pstd(p, E0, B0, sched, 1, "fp32")
    err = field_error(got, ref)
    assert err < 1e-5
