"""Invariants and closed forms the PSATD step must satisfy (oracle side).

* Dispersion-free vacuum with no Courant limit (Sec. III.B item 2; Table 1,
  PSATD row: index 1, Courant condition "None"): a lattice plane wave at any
  angle advances by exactly c|k| dt per step for any dt.
* Vacuum energy is conserved (the per-mode transverse update is unitary).
* div B = 0 and Gauss's law are kept when J and rho obey continuity.
* The rho-form and the J-form agree under continuity; r2c and c2c agree.
* Sources held constant over a step (Sec. III.B item 2) make the step exact,
  so k steps of dt equal one step of k*dt for constant J and linear rho.
* A brute-force step (explicit DFT sums, matrix exponential per mode,
  explicit inverse sums) equals the oracle step on tiny grids.
"""

import itertools

import numpy as np
import pytest
from scipy.linalg import expm

import fixtures
import oracle
from conftest import rel_l2


def _div(F, d):
    return fixtures.spectral_div(F, d)


# ------------------------------------------------------------------ plane waves
ANGLES_2D = [(1, 0), (1, 1), (2, 1), (3, 2), (5, 3), (0, 4), (-3, 2)]
DTS = [0.5, 1.0, 5.0, 20.0]


@pytest.mark.parametrize("m", ANGLES_2D)
@pytest.mark.parametrize("dt_factor", DTS)
def test_plane_wave_phase_2d(m, dt_factor):
    nz, nx = 24, 32
    dx = dz = 1.0 / 16
    d = (dx, dx, dz)
    k = np.array([2 * np.pi * m[0] / (nx * dx), 0.0, 2 * np.pi * m[1] / (nz * dz)])
    e = np.cross(k, [0.0, 1.0, 0.0])
    e = 0.6 * e / np.linalg.norm(e) + 0.8 * np.array([0.0, 1.0, 0.0])  # mixed polarization
    E, B, _ = fixtures.lattice_plane_wave((nz, nx), d, (m[0], 0, m[1]), e, phase=0.3)
    dt = dt_factor * dx
    steps = 7
    En, Bn = oracle.psatd_run(E, B, steps, d=d, dt=dt)
    Ex, Bx, _ = fixtures.lattice_plane_wave((nz, nx), d, (m[0], 0, m[1]), e, phase=0.3, t=steps * dt)
    assert rel_l2(En + Bn, Ex + Bx) < 1e-12


@pytest.mark.parametrize("m", [(1, 2, 3), (3, -1, 2), (2, 2, 2), (0, 3, 1)])
def test_plane_wave_phase_3d(m):
    shape = (12, 16, 18)
    d = (0.1, 0.07, 0.13)
    k = np.array([2 * np.pi * m[0] / (shape[2] * d[0]), 2 * np.pi * m[1] / (shape[1] * d[1]),
                  2 * np.pi * m[2] / (shape[0] * d[2])])
    e = np.cross(k, [0.3, 0.5, -0.2])
    e /= np.linalg.norm(e)
    E, B, _ = fixtures.lattice_plane_wave(shape, d, m, e, phase=1.1)
    dt = 3.7 * min(d)
    En, Bn = oracle.psatd_run(E, B, 5, d=d, dt=dt)
    Ex, Bx, _ = fixtures.lattice_plane_wave(shape, d, m, e, phase=1.1, t=5 * dt)
    assert rel_l2(En + Bn, Ex + Bx) < 1e-12


def test_phase_per_step_is_exactly_ck_dt_not_yee():
    # One step shifts the wave by c|k|dt; the Yee frequency (Sec. III.A) would
    # give a visibly different field -- the contrast the paper draws.
    from oracle.dispersion import omega_fdtd
    nz, nx, dx = 16, 16, 1.0 / 16
    d = (dx, dx, dx)
    m = (3, 0, 2)
    e = np.array([0.0, 1.0, 0.0])
    E, B, k = fixtures.lattice_plane_wave((nz, nx), d, m, e)
    dt = 0.7 * dx
    En, Bn = oracle.psatd_step(E, B, d=d, dt=dt)
    Ex, Bx, _ = fixtures.lattice_plane_wave((nz, nx), d, m, e, t=dt)
    assert rel_l2(En + Bn, Ex + Bx) < 1e-13
    w_yee = float(omega_fdtd(k[0], k[2], dx, dx, dt))
    Ey_, By_, _ = fixtures.lattice_plane_wave((nz, nx), d, m, e, t=w_yee * dt / np.linalg.norm(k))
    assert rel_l2(En + Bn, Ey_ + By_) > 1e-3


# ------------------------------------------------------------------ invariants
def _vacuum_fields(shape, d, seed=3):
    rng = np.random.default_rng(seed)
    E = fixtures.project_transverse([rng.standard_normal(shape) for _ in range(3)], d)
    B = fixtures.project_transverse([rng.standard_normal(shape) for _ in range(3)], d)
    return E, B


@pytest.mark.parametrize("shape", [(32, 48), (12, 16, 10)])
def test_vacuum_energy_conserved(shape):
    d = (0.05, 0.06, 0.04)
    E, B = _vacuum_fields(shape, d)
    W0 = oracle.field_energy(E, B)
    En, Bn = oracle.psatd_run(E, B, 40, d=d, dt=0.9 * 0.05)
    assert abs(oracle.field_energy(En, Bn) / W0 - 1.0) < 1e-13


def _sourced_workload(shape=(48, 64)):
    return fixtures.workload(1, shape=shape, steps=12)


@pytest.mark.parametrize("form", ["rho", "J"])
def test_gauss_and_divb_preserved(form):
    w = _sourced_workload()
    p = w.patches[0]
    sched = w.schedule[0]
    E, B = w.E0[0], w.B0[0]
    norm_e = np.sqrt(sum(np.sum(f * f) for f in E))
    for n in range(w.steps):
        J, ro, rn = sched.sources(n)
        E, B = oracle.psatd_step(E, B, J, ro, rn, d=p.d, dt=p.dt, form=form)
        gauss = _div(E, p.d) - rn
        assert np.sqrt(np.sum(gauss ** 2)) < 1e-12 * norm_e / p.dx
        assert np.sqrt(np.sum(_div(B, p.d) ** 2)) < 1e-12 * norm_e / p.dx


def test_rho_form_equals_j_form_under_continuity():
    w = _sourced_workload()
    p = w.patches[0]
    a = oracle.psatd_run(w.E0[0], w.B0[0], 10, d=p.d, dt=p.dt, schedule=w.schedule[0], form="rho")
    b = oracle.psatd_run(w.E0[0], w.B0[0], 10, d=p.d, dt=p.dt, schedule=w.schedule[0], form="J")
    assert rel_l2(a[0] + a[1], b[0] + b[1]) < 1e-13


@pytest.mark.parametrize("shape", [(24, 32), (8, 12, 10)])
def test_r2c_equals_c2c(shape):
    d = (0.1, 0.1, 0.1)
    rng = np.random.default_rng(7)
    E = [rng.standard_normal(shape) for _ in range(3)]   # arbitrary (non-physical) fields
    B = [rng.standard_normal(shape) for _ in range(3)]
    J = [rng.standard_normal(shape) for _ in range(3)]
    ro, rn = rng.standard_normal(shape), rng.standard_normal(shape)
    a = oracle.psatd_step(E, B, J, ro, rn, d=d, dt=0.13, transform="r2c")
    b = oracle.psatd_step(E, B, J, ro, rn, d=d, dt=0.13, transform="c2c")  # asserts a real result
    assert rel_l2(a[0] + a[1], b[0] + b[1]) < 1e-14


def test_semigroup_vacuum():
    d = (0.05, 0.05, 0.05)
    E, B = _vacuum_fields((32, 40), d, seed=11)
    a = oracle.psatd_run(E, B, 16, d=d, dt=0.3 * 0.05)
    b = oracle.psatd_step(E, B, d=d, dt=16 * 0.3 * 0.05)
    assert rel_l2(a[0] + a[1], b[0] + b[1]) < 1e-13


def test_semigroup_constant_current_linear_charge():
    # J constant in time and rho^n = rho^0 - n dt div J: the exact integration
    # over k steps equals one step of k*dt.
    w = _sourced_workload((32, 48))
    p = w.patches[0]
    P, D = w.schedule[0].P, w.schedule[0].D
    J = [1.7 * P[c] for c in range(3)]
    divJ = 1.7 * (D[0] + D[1] + D[2])
    rho0 = np.zeros(p.shape)
    E, B = w.E0[0], w.B0[0]
    k = 9
    for n in range(k):
        E, B = oracle.psatd_step(E, B, J, rho0 - n * p.dt * divJ, rho0 - (n + 1) * p.dt * divJ,
                                 d=p.d, dt=p.dt)
    E1, B1 = oracle.psatd_step(w.E0[0], w.B0[0], J, rho0, rho0 - k * p.dt * divJ, d=p.d, dt=k * p.dt)
    assert rel_l2(E + B, E1 + B1) < 1e-12


# ------------------------------------------------------------------ brute force
def _crossmat(k):
    kx, ky, kz = k
    return np.array([[0, -kz, ky], [kz, 0, -kx], [-ky, kx, 0]], dtype=np.complex128)


def _bruteforce_step(E, B, J, d, dt):
    """Explicit DFT -> per-mode matrix exponential (J constant) -> explicit inverse DFT."""
    shape = E[0].shape
    N = int(np.prod(shape))
    axes_k = []
    for ax, n in enumerate(shape):
        dd = d[2] if ax == 0 else (d[0] if ax == len(shape) - 1 else d[1])
        m = np.array([j if j < (n + 1) // 2 else j - n for j in range(n)], float)
        if n % 2 == 0:
            m[n // 2] = 0.0       # Nyquist reading
        axes_k.append(2 * np.pi * m / (n * dd))
    grids = np.meshgrid(*[np.arange(n) for n in shape], indexing="ij")
    inputs = list(E) + list(B) + list(J)
    outE = [np.zeros(shape, complex) for _ in range(3)]
    outB = [np.zeros(shape, complex) for _ in range(3)]
    for kidx in itertools.product(*[range(n) for n in shape]):
        ph = np.exp(-2j * np.pi * sum(kk * g / n for kk, g, n in zip(kidx, grids, shape)))
        spec = np.array([np.sum(f * ph) for f in inputs])
        if len(shape) == 2:
            kv = (axes_k[1][kidx[1]], 0.0, axes_k[0][kidx[0]])
        else:
            kv = (axes_k[2][kidx[2]], axes_k[1][kidx[1]], axes_k[0][kidx[0]])
        A = np.zeros((7, 7), complex)
        A[0:3, 3:6] = 1j * _crossmat(kv)
        A[3:6, 0:3] = -1j * _crossmat(kv)
        A[0:3, 6] = -spec[6:9]
        y = expm(dt * A) @ np.concatenate([spec[0:6], [1.0]])
        back = np.conj(ph) / N
        for i in range(3):
            outE[i] += y[i] * back
            outB[i] += y[3 + i] * back
    return [f.real for f in outE], [f.real for f in outB]


@pytest.mark.parametrize("shape", [(6, 8), (8, 6), (4, 6, 6)])
def test_full_step_equals_bruteforce(shape):
    d = (0.2, 0.3, 0.25)
    rng = np.random.default_rng(5)
    E = [rng.standard_normal(shape) for _ in range(3)]
    B = fixtures.project_transverse([rng.standard_normal(shape) for _ in range(3)], d)
    J = [rng.standard_normal(shape) for _ in range(3)]
    dt = 0.37
    Eb, Bb = _bruteforce_step(E, B, J, d, dt)
    Eo, Bo = oracle.psatd_step(E, B, J, d=d, dt=dt, form="J")
    assert rel_l2(Eo + Bo, Eb + Bb) < 1e-12
    # rho-form with Gauss-consistent E and continuity-consistent rho gives the same step
    rho_o = _div(E, d)
    rho_n = rho_o - dt * _div(J, d)
    Er, Br = oracle.psatd_step(E, B, J, rho_o, rho_n, d=d, dt=dt, form="rho")
    assert rel_l2(Er + Br, Eb + Bb) < 1e-12
