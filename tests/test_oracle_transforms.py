"""Pins of the oracle's transforms and k tables against brute-force definitions."""

import itertools

import numpy as np
import pytest

import oracle


def dft_bruteforce(f, half_last=False):
    """Direct O(N^2) sum  F(k) = sum_x f(x) exp(-2 pi i k.x / N), all axes."""
    shape = f.shape
    out_shape = list(shape)
    if half_last:
        out_shape[-1] = shape[-1] // 2 + 1
    F = np.zeros(out_shape, dtype=np.complex128)
    grids = np.meshgrid(*[np.arange(n) for n in shape], indexing="ij")
    for kidx in itertools.product(*[range(n) for n in out_shape]):
        phase = sum(kk * g / n for kk, g, n in zip(kidx, grids, shape))
        F[kidx] = np.sum(f * np.exp(-2j * np.pi * phase))
    return F


def idft_bruteforce(F, shape):
    """Direct inverse sum with 1/N over the full (c2c) spectrum."""
    N = int(np.prod(shape))
    f = np.zeros(shape, dtype=np.complex128)
    grids = np.meshgrid(*[np.arange(n) for n in shape], indexing="ij")
    for kidx in itertools.product(*[range(n) for n in shape]):
        phase = sum(kk * g / n for kk, g, n in zip(kidx, grids, shape))
        f += F[kidx] * np.exp(2j * np.pi * phase)
    return f / N


@pytest.mark.parametrize("shape", [(4, 6), (6, 8), (8, 12), (6, 4, 6), (4, 6, 8)])
def test_forward_matches_bruteforce_dft(shape, rng):
    f = rng.standard_normal(shape)
    ref_c2c = dft_bruteforce(f)
    ref_r2c = dft_bruteforce(f, half_last=True)
    np.testing.assert_allclose(oracle.forward(f, "c2c"), ref_c2c, rtol=0, atol=1e-12 * np.abs(ref_c2c).max())
    np.testing.assert_allclose(oracle.forward(f, "r2c"), ref_r2c, rtol=0, atol=1e-12 * np.abs(ref_r2c).max())


@pytest.mark.parametrize("shape", [(4, 6), (6, 4, 6)])
def test_inverse_matches_bruteforce(shape, rng):
    f = rng.standard_normal(shape)
    F = dft_bruteforce(f)
    back = idft_bruteforce(F, shape)
    np.testing.assert_allclose(back.imag, 0, atol=1e-12)
    np.testing.assert_allclose(oracle.inverse(F, shape, "c2c"), back.real, atol=1e-12)
    Fh = dft_bruteforce(f, half_last=True)
    np.testing.assert_allclose(oracle.inverse(Fh, shape, "r2c"), f, atol=1e-12)


def test_ktable_definition():
    # k_j = 2 pi m_j / (N d): m = 0, 1, .., N/2 - 1, [Nyquist -> 0], -N/2 + 1, .., -1
    k = oracle.ktable(8, 0.5)
    expect = 2 * np.pi / (8 * 0.5) * np.array([0, 1, 2, 3, 0, -3, -2, -1])
    np.testing.assert_allclose(k, expect, rtol=0, atol=1e-15)
    np.testing.assert_allclose(oracle.rktable(8, 0.5), expect[:5], rtol=0, atol=1e-15)
    k6 = oracle.ktable(6, 1.0)
    np.testing.assert_allclose(k6, 2 * np.pi / 6 * np.array([0, 1, 2, 0, -2, -1]), atol=1e-15)
    k9 = oracle.ktable(9, 1.0)  # odd: no Nyquist index
    np.testing.assert_allclose(k9, 2 * np.pi / 9 * np.array([0, 1, 2, 3, 4, -4, -3, -2, -1]), atol=1e-15)


def test_order_p_tables_limits():
    from oracle.dispersion import fornberg_staggered, modified_k
    # p = 2 is the Yee stencil: k_2 = 2 sin(k dx / 2) / dx
    k = np.linspace(0.01, 3.0, 50)
    np.testing.assert_allclose(modified_k(k, 1.0, 2), 2 * np.sin(k / 2), rtol=1e-14)
    # staggered 4th order weights 9/8, -1/24 (a textbook stencil)
    w = fornberg_staggered(4)
    assert w[0] == pytest.approx(9 / 8) and w[1] == pytest.approx(-1 / 24)
    # consistency: sum_l C_l (2l - 1) = 1 for every p (exact on linear functions)
    for p in (2, 4, 8, 16, 32, 64, 128):
        assert float(sum(c * (2 * l - 1) for l, c in enumerate(fornberg_staggered(p), 1))) == pytest.approx(1.0, abs=1e-14)
    # p -> infinity converges to k where k dx < pi / 2 (Sec. III.B)
    kk = np.linspace(0.01, np.pi / 2, 40)
    err = [np.max(np.abs(modified_k(kk, 1.0, p) - kk) / kk) for p in (8, 32, 128)]
    assert err[0] > err[1] > err[2] and err[2] < 1e-13
