"""Pins of the per-mode PSATD update against the exact solution of Maxwell's equations.

Per mode, with constant J, d/dt (E^, B^) = A (E^, B^) + (-J^/eps0, 0) where
A = [[0, i c^2 [k]x], [-i [k]x, 0]].  The exact solution over dt is the matrix
exponential of the 7x7 augmented system (scipy.linalg.expm), which is
independent of the closed-form coefficients the oracle uses.
"""

import numpy as np
import pytest
from scipy.integrate import quad
from scipy.linalg import expm

import oracle


def crossmat(k):
    kx, ky, kz = k
    return np.array([[0, -kz, ky], [kz, 0, -kx], [-ky, kx, 0]], dtype=np.complex128)


def exact_step(E, B, J, k, dt, c, eps0):
    A = np.zeros((7, 7), dtype=np.complex128)
    K = crossmat(k)
    A[0:3, 3:6] = 1j * c * c * K
    A[3:6, 0:3] = -1j * K
    A[0:3, 6] = -J / eps0
    y = expm(dt * A) @ np.concatenate([E, B, [1.0]])
    return y[0:3], y[3:6]


def rand_c(rng, n):
    return rng.standard_normal(n) + 1j * rng.standard_normal(n)


def transverse(v, k):
    k = np.asarray(k, float)
    return v - k * (k @ v) / (k @ k)


def oracle_update(E, B, J, ro, rn, k, dt, c, eps0, form):
    Ek = [np.array([e]) for e in E]
    Bk = [np.array([b]) for b in B]
    Jk = [np.array([j]) for j in J] if J is not None else None
    kk = tuple(np.array([x]) for x in k)
    En, Bn = oracle.update_modes(Ek, Bk, kk, dt, c=c, eps0=eps0, Jk=Jk,
                                 rho_old_k=None if ro is None else np.array([ro]),
                                 rho_new_k=None if rn is None else np.array([rn]), form=form)
    return np.array([x[0] for x in En]), np.array([x[0] for x in Bn])


CASES = [
    # (c, eps0, dt, |k| scale)  -- theta = c|k|dt spans the series branch, O(1) and >> 1
    (1.0, 1.0, 0.37, 1.0),
    (1.3, 0.7, 0.37, 2.5),
    (1.0, 1.0, 1e-3, 1.0),
    (2.0, 3.0, 5.0, 4.0),
    (1.0, 1.0, 20.0, 0.3),
]


@pytest.mark.parametrize("c,eps0,dt,ks", CASES)
def test_rho_form_equals_matrix_exponential(c, eps0, dt, ks, rng):
    for _ in range(20):
        k = rng.standard_normal(3) * ks
        K2 = k @ k
        B = transverse(rand_c(rng, 3), k)
        ro = complex(rng.standard_normal() + 1j * rng.standard_normal())
        E = transverse(rand_c(rng, 3), k) - 1j * k * ro / (eps0 * K2)   # Gauss at t^n
        J = rand_c(rng, 3)
        rn = ro - 1j * dt * (k @ J)                                   # continuity
        Eref, Bref = exact_step(E, B, J, k, dt, c, eps0)
        En, Bn = oracle_update(E, B, J, ro, rn, k, dt, c, eps0, "rho")
        scale = max(np.abs(Eref).max(), np.abs(Bref).max() * c)
        assert np.abs(En - Eref).max() <= 1e-12 * scale
        assert np.abs(Bn - Bref).max() * c <= 1e-12 * scale


@pytest.mark.parametrize("c,eps0,dt,ks", CASES)
def test_j_form_equals_matrix_exponential(c, eps0, dt, ks, rng):
    for _ in range(20):
        k = rng.standard_normal(3) * ks
        B = transverse(rand_c(rng, 3), k)
        E = rand_c(rng, 3)            # any longitudinal part
        J = rand_c(rng, 3)
        Eref, Bref = exact_step(E, B, J, k, dt, c, eps0)
        En, Bn = oracle_update(E, B, J, None, None, k, dt, c, eps0, "J")
        scale = max(np.abs(Eref).max(), np.abs(Bref).max() * c)
        assert np.abs(En - Eref).max() <= 1e-12 * scale
        assert np.abs(Bn - Bref).max() * c <= 1e-12 * scale


def test_vacuum_equals_matrix_exponential(rng):
    for _ in range(20):
        k = rng.standard_normal(3) * 3
        B = transverse(rand_c(rng, 3), k)
        E = transverse(rand_c(rng, 3), k)
        Eref, Bref = exact_step(E, B, np.zeros(3), k, 0.8, 1.0, 1.0)
        En, Bn = oracle_update(E, B, None, None, None, k, 0.8, 1.0, 1.0, "rho")
        assert np.abs(En - Eref).max() < 1e-12 and np.abs(Bn - Bref).max() < 1e-12


def test_k_zero_mode(rng):
    E, B, J = rand_c(rng, 3), rand_c(rng, 3), rand_c(rng, 3)
    for form in ("rho", "J"):
        En, Bn = oracle_update(E, B, J, 0.3 + 0.1j, 0.2j, (0.0, 0.0, 0.0), 0.5, 1.2, 0.8, form)
        np.testing.assert_allclose(En, E - 0.5 * J / 0.8, rtol=0, atol=1e-15)
        np.testing.assert_allclose(Bn, B, rtol=0, atol=1e-15)


def test_coefficients_at_k_zero():
    co = oracle.psatd_coefficients(np.array([0.0]), 0.7, c=1.5, eps0=0.9)
    assert co["C"][0] == 1.0
    assert co["S"][0] == pytest.approx(0.7, rel=1e-15)
    assert co["X1"][0] == pytest.approx(0.7 ** 2 / (2 * 0.9), rel=1e-15)
    assert co["X2"][0] == pytest.approx(1.5 ** 2 * 0.7 ** 2 / (6 * 0.9), rel=1e-15)
    assert co["X3"][0] == pytest.approx(-1.5 ** 2 * 0.7 ** 2 / (3 * 0.9), rel=1e-15)


def test_g_against_quadrature():
    # g(theta) = (1 - sin theta / theta) / theta^2 = int_0^1 (t^2/2) sinc^2(theta t/2) dt,
    # an integral with no cancellation at small theta.
    import warnings

    def g_quad(th):
        f = lambda t: 0.5 * t * t * (np.sinc(th * t / (2 * np.pi))) ** 2
        with warnings.catch_warnings():
            warnings.simplefilter("ignore")
            return quad(f, 0.0, 1.0, epsabs=1e-300, epsrel=1e-14, limit=200)[0]

    thetas = np.array([0.0, 1e-8, 1e-5, 1e-3, 0.1, 0.2499999, 0.25, 0.2500001, 0.5, 1.0, 3.0, 10.0])
    g = oracle.g_series(thetas)
    for th, gv in zip(thetas, g):
        assert gv == pytest.approx(g_quad(th), rel=2e-14), th


def test_coefficients_against_direct_forms_away_from_zero():
    # Where no cancellation occurs (theta >= 1) the textbook forms are accurate.
    K = np.linspace(2.0, 40.0, 50)
    dt, c, e = 0.9, 1.1, 0.8
    th = c * K * dt
    co = oracle.psatd_coefficients(K, dt, c, e)
    np.testing.assert_allclose(co["C"], np.cos(th), rtol=1e-14, atol=1e-15)
    np.testing.assert_allclose(co["S"], np.sin(th) / (c * K), rtol=1e-13, atol=1e-15)
    np.testing.assert_allclose(co["X1"], (1 - np.cos(th)) / (e * c * c * K * K), rtol=1e-12)
    np.testing.assert_allclose(co["X2"], (1 - np.sin(th) / th) / (e * K * K), rtol=1e-12)
    np.testing.assert_allclose(co["X3"], (np.cos(th) - np.sin(th) / th) / (e * K * K), rtol=1e-12, atol=1e-15)
