"""Pins of the dispersion contrast (Yee, CKC, PSTD) against numbers the paper prints."""

import json
import os

import numpy as np
import pytest

from oracle import dispersion as dz

GOLDEN = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_values.json")))


def test_pstd_index_and_limit_angle_match_paper():
    g = GOLDEN["pstd_index_at_kdx_pi_over_2"]
    eta = GOLDEN["courant_limits"]["pstd"]          # c dt / dx at the PSTD Courant limit
    n_r = float(dz.index_pstd(np.pi / 2, eta))       # k dx = pi/2, dx = 1
    assert round(n_r, g["decimals"]) == g["value"]
    assert n_r < 1.0                                 # supraluminal (Sec. III.B item 1)
    ga = GOLDEN["pstd_limit_angle_deg"]
    assert round(float(dz.limit_angle_deg(g["value"])), ga["decimals"]) == ga["value"]


def test_courant_limits_of_table1():
    cl = GOLDEN["courant_limits"]
    dx = 1.0
    # Yee: the Nyquist mode kx = kz = pi/dx is marginal exactly at eta = 1/sqrt(2)
    w = dz.omega_fdtd(np.pi, np.pi, dx, dx, cl["yee"] * (1 - 1e-12) * dx)
    assert np.isfinite(w) and np.isnan(dz.omega_fdtd(np.pi, np.pi, dx, dx, cl["yee"] * 1.0001))
    # CKC allows c dt = dx
    assert np.isfinite(dz.omega_fdtd(np.pi, np.pi, dx, dx, cl["ckc"] * (1 - 1e-12) * dx, beta=dz.BETA_CKC))
    assert cl["pstd"] == pytest.approx(np.sqrt(2) / np.pi)
    assert cl["yee"] == pytest.approx(1 / np.sqrt(2))


def test_ckc_is_dispersion_free_along_axes_only():
    # Sec. III.A: CKC with beta = 1/4 and c dt = dx is dispersion-free along x and z
    k = np.linspace(0.05, 3.0, 30)
    np.testing.assert_allclose(dz.index_ckc(k, 0 * k, 1.0, 1.0, 1.0), 1.0, rtol=1e-12)
    np.testing.assert_allclose(dz.index_ckc(0 * k, k, 1.0, 1.0, 1.0), 1.0, rtol=1e-12)
    diag = dz.index_ckc(k / np.sqrt(2), k / np.sqrt(2), 1.0, 1.0, 1.0)
    assert np.all(diag[5:] > 1.0 + 1e-4)
    # Yee is dispersive along the axes (index > 1)
    assert np.all(dz.index_yee(k, 0 * k, 1.0, 1.0, 0.7) > 1.0)


def test_ckc_matches_appendix_beta_prime():
    # Appendix A eq. (A1): the CKC relation equals the beta' form with beta' = -4 beta = -1
    g = GOLDEN["ckc_beta_prime"]
    rng = np.random.default_rng(0)
    for _ in range(50):
        kt, th, eta = rng.uniform(0.01, 3.0), rng.uniform(0, np.pi / 2), rng.uniform(0.1, 1.0)
        kx, kz = kt * np.cos(th), kt * np.sin(th)
        w = dz.omega_fdtd(kx, kz, 1.0, 1.0, eta, beta=g["beta"])
        sx2, sz2 = np.sin(kx / 2) ** 2, np.sin(kz / 2) ** 2
        rhs = eta ** 2 * (sx2 + sz2 + g["beta_prime"] * sx2 * sz2)
        if np.isfinite(w):
            assert np.sin(w * eta / 2) ** 2 == pytest.approx(rhs, rel=1e-12)


def test_appendix_a_reduces_to_yee_at_pi_over_4():
    g = GOLDEN["appendix_a_pi_over_4"]
    eta, beta = dz.appendix_eta_beta(np.pi / 4)
    assert eta == pytest.approx(g["eta"], rel=1e-14)
    assert beta == pytest.approx(g["beta_prime"], abs=1e-14)
    # elsewhere the tuned scheme violates the Nyquist stability ansatz (Appendix A)
    for th in np.linspace(0.1, 1.4, 12):
        if abs(th - np.pi / 4) < 0.05:
            continue
        e, b = dz.appendix_eta_beta(th)
        assert e > dz.appendix_eta_stable(b)


def test_appendix_a_solution_satisfies_its_two_conditions():
    for th in np.linspace(0.1, 1.4, 9):
        e, b = dz.appendix_eta_beta(th)
        cs2 = np.cos(th) ** 2 * np.sin(th) ** 2
        assert e ** 2 == pytest.approx(1 - (2 + 3 * b) * cs2, rel=1e-12)
        assert e ** 4 == pytest.approx(1 - (3 + 7.5 * b) * cs2, rel=1e-12)


@pytest.mark.parametrize("m,eta", [((1, 0), 0.5), ((3, 2), 0.7), ((5, 5), 0.7071), ((7, 1), 0.3)])
def test_yee_stepper_reproduces_its_dispersion_relation(m, eta):
    nx, nz, dx = 32, 24, 1.0
    dt = eta * dx
    Ey, Bx, Bz, w = dz.yee_lattice_mode(nx, nz, m[0], m[1], dx, dx, dt)
    E0 = Ey.copy()
    steps = 25
    for _ in range(steps):
        Ey, Bx, Bz = dz.yee_step_s_pol(Ey, Bx, Bz, dx, dx, dt)
    measured = -np.angle(np.vdot(E0, Ey) / np.vdot(E0, E0))
    expect = (w * dt * steps + np.pi) % (2 * np.pi) - np.pi
    assert measured == pytest.approx(expect, abs=1e-11)
    # and it is not c|k|dt: Yee's vacuum is dispersive
    kk = 2 * np.pi * np.hypot(m[0] / (nx * dx), m[1] / (nz * dx))
    assert abs(w - kk) > 1e-6


def test_psatd_p_index_tends_to_one():
    k = np.linspace(0.05, np.pi / 2, 20)
    n128 = dz.index_psatd_p(k * np.cos(0.4), k * np.sin(0.4), 1.0, 1.0, 128)
    np.testing.assert_allclose(n128, 1.0, atol=1e-12)
    n2 = dz.index_psatd_p(k * np.cos(0.4), k * np.sin(0.4), 1.0, 1.0, 2)
    assert np.all(n2[3:] > 1.0 + 1e-4)
