"""Planted mistakes in the oracle must be caught by its pins (CPU only).

Each case patches one plausible error into ``oracle.psatd`` (a dropped term, a
wrong sign, a transposed operand, a missed convention) and checks that at
least one independent pin -- the matrix exponential of the per-mode system,
the exact plane-wave phase, or r2c == c2c -- sees it.
"""

import numpy as np
import pytest

import fixtures
import oracle
import oracle.psatd as ops
from conftest import rel_l2
from test_oracle_update import exact_step, rand_c, transverse, oracle_update


def expm_error(form):
    rng = np.random.default_rng(99)
    worst = 0.0
    for _ in range(10):
        k = rng.standard_normal(3) * 2
        B = transverse(rand_c(rng, 3), k)
        ro = complex(rng.standard_normal())
        E = transverse(rand_c(rng, 3), k) - 1j * k * ro / (k @ k)
        J = rand_c(rng, 3)
        rn = ro - 1j * 0.4 * (k @ J)
        Er, Br = exact_step(E, B, J, k, 0.4, 1.0, 1.0)
        En, Bn = oracle_update(E, B, J, ro, rn, k, 0.4, 1.0, 1.0, form)
        worst = max(worst, np.abs(En - Er).max(), np.abs(Bn - Br).max())
    return worst


def plane_wave_error():
    d = (1 / 16, 1 / 16, 1 / 16)
    k_m = (3, 0, 2)
    kv = np.array([2 * np.pi * 3 / (32 / 16), 0.0, 2 * np.pi * 2 / (24 / 16)])
    e = np.cross(kv, [0.2, 1.0, 0.1])
    e /= np.linalg.norm(e)
    E, B, _ = fixtures.lattice_plane_wave((24, 32), d, k_m, e, phase=0.4)
    En, Bn = oracle.psatd_run(E, B, 3, d=d, dt=0.9 / 16)
    Ex, Bx, _ = fixtures.lattice_plane_wave((24, 32), d, k_m, e, phase=0.4, t=3 * 0.9 / 16)
    return rel_l2(En + Bn, Ex + Bx)


def r2c_c2c_error():
    rng = np.random.default_rng(3)
    shape = (8, 12)
    E = [rng.standard_normal(shape) for _ in range(3)]
    B = [rng.standard_normal(shape) for _ in range(3)]
    try:
        a = oracle.psatd_step(E, B, d=(0.1, 0.1, 0.1), dt=0.2, transform="r2c")
        b = oracle.psatd_step(E, B, d=(0.1, 0.1, 0.1), dt=0.2, transform="c2c")
    except AssertionError:
        return np.inf
    return rel_l2(a[0] + a[1], b[0] + b[1])


def all_pins_pass():
    return (expm_error("rho") < 1e-12 and expm_error("J") < 1e-12
            and plane_wave_error() < 1e-12 and r2c_c2c_error() < 1e-13)


def test_unmutated_oracle_passes_all_pins():
    assert all_pins_pass()


def _coeff_mutant(key, fn):
    orig = ops.psatd_coefficients

    def mutant(K, dt, c=1.0, eps0=1.0):
        co = orig(K, dt, c, eps0)
        co[key] = fn(co, K, dt, c, eps0)
        return co
    return mutant


MUTANTS = {
    "X3 sign": ("psatd_coefficients", _coeff_mutant("X3", lambda co, K, dt, c, e: -co["X3"])),
    "X2 dropped": ("psatd_coefficients", _coeff_mutant("X2", lambda co, K, dt, c, e: 0 * co["X2"])),
    "X1 halved": ("psatd_coefficients", _coeff_mutant("X1", lambda co, K, dt, c, e: 0.5 * co["X1"])),
    "C at half angle": ("psatd_coefficients",
                        _coeff_mutant("C", lambda co, K, dt, c, e: np.cos(0.5 * c * K * dt))),
    "S without 1/(cK)": ("psatd_coefficients",
                         _coeff_mutant("S", lambda co, K, dt, c, e: np.sin(c * K * dt))),
    "cross transposed": ("_cross", lambda a, b: (b[1] * a[2] - b[2] * a[1],
                                                 b[2] * a[0] - b[0] * a[2],
                                                 b[0] * a[1] - b[1] * a[0])),
    "cross index slip": ("_cross", lambda a, b: (a[1] * b[2] - a[2] * b[1],
                                                 a[2] * b[0] - a[0] * b[2],
                                                 a[0] * b[2] - a[1] * b[0])),
    "Nyquist kept": ("ktable", lambda n, d, order=0, stencil="staggered": 2 * np.pi * np.fft.fftfreq(n, d=d)),
}


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_planted_mistake_is_caught(name, monkeypatch):
    attr, fn = MUTANTS[name]
    monkeypatch.setattr(ops, attr, fn)
    assert not all_pins_pass(), f"mutant '{name}' slipped past every pin"
