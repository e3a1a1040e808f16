"""Pins of the centered order-p stencil and of the guard-cell decomposition
(oracle/decomposition.py, Sec. II.A), against closed forms, exact special
cases and brute force."""

from fractions import Fraction
from math import factorial

import numpy as np
import pytest

import fixtures
import oracle
from oracle.decomposition import decomposed_step, local_index
from oracle.dispersion import fornberg_centered, modified_k


# ---------------------------------------------------------------- centered stencil
def test_centered_weights_closed_form():
    # textbook central differences, then the closed form for every order
    assert fornberg_centered(2) == [Fraction(1, 2)]
    assert fornberg_centered(4) == [Fraction(2, 3), Fraction(-1, 12)]
    for p in range(2, 33, 2):
        m = p // 2
        ref = [Fraction((-1) ** (l + 1) * factorial(m) ** 2, factorial(m - l) * factorial(m + l) * l)
               for l in range(1, m + 1)]
        assert fornberg_centered(p) == ref


def test_centered_stencil_is_exact_on_polynomials():
    # f'(0) from sum_l a_l (f(l) - f(-l)) is exact for polynomials of degree <= p
    for p in (2, 4, 8, 12):
        w = fornberg_centered(p)
        for deg in range(0, p + 1):
            approx = sum(a * (Fraction(l) ** deg - Fraction(-l) ** deg) for l, a in enumerate(w, 1))
            assert approx == (1 if deg == 1 else 0)


def test_centered_symbol_vanishes_at_nyquist_and_converges():
    dx = 0.3
    kn = np.pi / dx
    for p in (2, 8, 32):
        assert abs(modified_k(np.array([kn]), dx, p, "centered")[0]) < 1e-12 / dx
    k = np.linspace(0.05, 0.5, 7) * np.pi / dx
    errs = [np.max(np.abs(modified_k(k, dx, p, "centered") - k) / k) for p in (4, 8, 16, 32, 64)]
    assert all(b < a for a, b in zip(errs, errs[1:]))
    assert errs[-1] < 1e-9


# ---------------------------------------------------------------- decomposition
def _rel(a, b):
    num = sum(np.sum((x - y) ** 2) for x, y in zip(a, b))
    return np.sqrt(num / sum(np.sum(y * y) for y in b))


def test_local_index_against_brute_force():
    shape = (12, 10, 8)  # [z][y][x]
    parts, guard = (2, 1, 3), (3, 5, 2)
    for s in [(0, 0, 0), (1, 0, 2), (1, 0, 1)]:
        idx = local_index(shape, parts, guard, s)
        # x: box 4, guard 3 (split); y: unsplit, no guard; z: box 4, guard 2
        ex = [(s[0] * 4 - 3 + i) % 8 for i in range(4 + 6)]
        ey = list(range(10))
        ez = [(s[2] * 4 - 2 + i) % 12 for i in range(4 + 4)]
        assert list(idx[2]) == ex and list(idx[1]) == ey and list(idx[0]) == ez


def test_single_box_without_guards_is_the_global_step():
    w = fixtures.workload(0, shape=(24, 32))
    p = w.patches[0]
    ref = oracle.psatd_step(w.E0[0], w.B0[0], d=p.d, dt=p.dt)
    got = decomposed_step(w.E0[0], w.B0[0], parts=(1, 1, 1), guard=(0, 0, 0), d=p.d, dt=p.dt)
    assert _rel(got[0] + got[1], ref[0] + ref[1]) < 1e-15


@pytest.mark.parametrize("order,stencil", [(0, "staggered"), (16, "staggered"), (16, "centered")])
def test_wave_periodic_on_the_local_grid_is_exact(order, stencil):
    # period 32 cells in x divides the global 128 and the local 64 + 2*16;
    # period 48 in z divides the global 96 and the local 48 + 2*24
    shape, d = (96, 128), (1 / 32, 1.0, 1 / 32)
    kx, kz = 2 * np.pi / (32 * d[0]), 2 * np.pi / (48 * d[2])
    a = np.arctan2(kz, kx)
    E, B, _ = fixtures.lattice_plane_wave(shape, d, (4, 0, 2), (-np.sin(a), 0.0, np.cos(a)))
    ref = oracle.psatd_step(E, B, d=d, dt=d[0], order=order, stencil=stencil)
    got = decomposed_step(E, B, parts=(2, 1, 2), guard=(16, 0, 24), d=d, dt=d[0], order=order,
                          stencil=stencil)
    assert _rel(got[0] + got[1], ref[0] + ref[1]) < 1e-14


def _laser():
    rng = np.random.default_rng(3)
    d = (1 / 32, 1.0, 1 / 32)
    E, B = fixtures.fields.laser_2d(128, 128, d[0], d[2], angle_deg=30, waist=1.5, tau=1.0,
                                    nharm=8, rng=rng)
    return E, B, d


def _decomposition_error(order, stencil, guard, steps=4, cfl=0.5):
    E, B, d = _laser()
    dt = cfl * d[0]
    ref = oracle.psatd_run(E, B, steps, d=d, dt=dt, order=order, stencil=stencil)
    Ed, Bd = E, B
    for _ in range(steps):
        Ed, Bd = decomposed_step(Ed, Bd, parts=(2, 1, 2), guard=(guard, 0, guard), d=d, dt=dt,
                                 order=order, stencil=stencil)
    return _rel(Ed + Bd, ref[0] + ref[1])


def test_truncation_error_falls_with_guards_for_centered_order_p():
    e16 = _decomposition_error(16, "centered", 16)
    e40 = _decomposition_error(16, "centered", 40)
    assert e40 < 1e-12 < e16 < 1e-5


def test_infinite_order_is_not_local():
    # exact k: the wrap of every local grid reaches the interior (Sec. II.A
    # contrasts this with finite order p)
    assert _decomposition_error(0, "staggered", 16) > 1e-3
    assert _decomposition_error(0, "staggered", 40) > 1e-3
