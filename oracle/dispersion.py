"""Numerical dispersion of the solvers the paper compares -- TEST INFRASTRUCTURE.

These are the contrast the paper draws against PSATD: refractive-index
formulas of Table 1, the order-p modified wavevector (Sec. III.B and the
Table 1 caption), the angle-tuned CK analysis of Appendix A and a plain CPU
Yee FDTD stepper (Sec. III.A).  None of it is on the GPU path.

Readings of garbled or inconsistent printed formulas:
  * Yee / CKC rows of Table 1: the factor 1/2 inside the arcsin contradicts
    the Courant column; the standard relation
    sin(w dt/2) = c dt sqrt(sum_X A_X S_X^2 / dX^2), S_X = sin(k_X dX/2),
    is used (A_X = 1 for Yee).  It gives the Courant limit 1/sqrt(2) for Yee.
  * CKC: A_X = (1 - beta) + beta cos(k_Y dY) with beta = 1/4.  This is the
    form that matches Appendix A's beta' = -4 beta, and the one that makes
    CKC dispersion-free along x and z at c dt = dx (Sec. III.A).
  * PSATD order-p row: the index is (|k|/2) / sqrt(Sigma_px^2 + Sigma_pz^2),
    i.e. |k| / |k_p| (the stray c dt is dropped).
  * Order-p wavevector: k_p = sum_{l=1}^{p/2} C_l^p (2/dx) sin((2l-1) k dx/2)
    with the staggered-grid Fornberg weights C_l^p.
  * Appendix A: eta is the Courant number c dt / dx.
"""

from __future__ import annotations

import functools
from fractions import Fraction

import numpy as np

BETA_CKC = 0.25


# ---------------------------------------------------------------- dispersion relations
def omega_fdtd(kx, kz, dx, dz, dt, c=1.0, beta=0.0):
    """Frequency of a lattice mode under Yee (beta = 0) or CKC (beta = 1/4), 2D.

    Returns NaN where the scheme is unstable for that mode (argument > 1).
    """
    sx, sz = np.sin(0.5 * kx * dx), np.sin(0.5 * kz * dz)
    ax = (1.0 - beta) + beta * np.cos(kz * dz)
    az = (1.0 - beta) + beta * np.cos(kx * dx)
    arg = c * dt * np.sqrt(ax * sx * sx / dx ** 2 + az * sz * sz / dz ** 2)
    with np.errstate(invalid="ignore"):
        return np.where(arg <= 1.0, 2.0 / dt * np.arcsin(np.minimum(arg, 1.0)), np.nan)


def index_yee(kx, kz, dx, dz, dt, c=1.0):
    """n = c|k| / omega for the Yee scheme (Table 1, Yee row)."""
    return c * np.hypot(kx, kz) / omega_fdtd(kx, kz, dx, dz, dt, c, 0.0)


def index_ckc(kx, kz, dx, dz, dt, c=1.0):
    """n = c|k| / omega for the CKC scheme with beta = 1/4 (Table 1, CKC row)."""
    return c * np.hypot(kx, kz) / omega_fdtd(kx, kz, dx, dz, dt, c, BETA_CKC)


def index_pstd(k, dt, c=1.0):
    """PSTD row of Table 1: n = (|k| c dt/2) / arcsin(c dt |k|/2)."""
    a = 0.5 * c * dt * np.asarray(k, dtype=np.float64)
    return a / np.arcsin(a)


def index_psatd(k):
    """PSATD row of Table 1: n = 1 for every k."""
    return np.ones_like(np.asarray(k, dtype=np.float64))


def limit_angle_deg(n_r, n_i=1.0):
    """Total-reflection limit angle of Sec. IV.B.2: n_i sin(theta_l) = n_r."""
    return np.rad2deg(np.arcsin(n_r / n_i))


# ---------------------------------------------------------------- order p
def fornberg_staggered(p: int):
    """Staggered-grid first-derivative weights C_1..C_{p/2} (exact rationals).

    f'(0) ~ sum_l C_l [f((l - 1/2) h) - f(-(l - 1/2) h)] / h.  C_l is the
    derivative at 0 of the Lagrange basis polynomial on the nodes
    +-1/2, +-3/2, ..., +-(p-1)/2; because the nodes are symmetric,
    L_j'(0) = L_j(0) / x_j.
    """
    if p < 2 or p % 2:
        raise ValueError("p must be even and >= 2")
    half = p // 2
    nodes = [Fraction(2 * j - p + 1, 2) for j in range(p)]
    weights = []
    for l in range(1, half + 1):
        xj = Fraction(2 * l - 1, 2)
        L0 = Fraction(1)
        for xn in nodes:
            if xn != xj:
                L0 *= (0 - xn) / (xj - xn)
        weights.append(L0 / xj)
    return weights


def fornberg_centered(p: int):
    """Centered (collocated) first-derivative weights a_1..a_{p/2} (exact rationals).

    f'(0) ~ sum_l a_l [f(l h) - f(-l h)] / h on the integer nodes -p/2..p/2.
    a_l is the derivative at 0 of the Lagrange basis polynomial of node l;
    one factor of that polynomial is x / l, so L_l'(0) is the product of the
    remaining factors at 0, divided by l.
    """
    if p < 2 or p % 2:
        raise ValueError("p must be even and >= 2")
    half = p // 2
    nodes = [Fraction(j) for j in range(-half, half + 1)]
    weights = []
    for l in range(1, half + 1):
        xj = Fraction(l)
        prod = Fraction(1)
        for xn in nodes:
            if xn != xj and xn != 0:
                prod *= (0 - xn) / (xj - xn)
        weights.append(prod / xj)
    return weights


@functools.lru_cache(maxsize=None)
def _float_weights(p: int, stencil: str):
    """The order-p weights as floats (computed once per order and stencil)."""
    w = fornberg_staggered(p) if stencil == "staggered" else fornberg_centered(p)
    return tuple(float(x) for x in w)


def modified_k(k, dx, p: int, stencil: str = "staggered"):
    """Wavenumber of the order-p first-derivative stencil; p = 0 returns k.

    staggered (Table 1 caption):  k_p = sum_l C_l (2/dx) sin((2l-1) k dx/2)
    centered (collocated nodes):  k_p = sum_l a_l (2/dx) sin(l k dx), which
                                  vanishes smoothly at the Nyquist wavenumber.
    """
    k = np.asarray(k, dtype=np.float64)
    if p == 0:
        return k.copy()
    if stencil not in ("staggered", "centered"):
        raise ValueError(f"unknown stencil {stencil!r}")
    out = np.zeros_like(k)
    for l, wl in enumerate(_float_weights(p, stencil), start=1):
        arg = (2 * l - 1) * k * dx / 2.0 if stencil == "staggered" else l * k * dx
        out += wl * (2.0 / dx) * np.sin(arg)
    return out


def index_psatd_p(kx, kz, dx, dz, p):
    """PSATD order-p row of Table 1 (read as |k| / |k_p|)."""
    return np.hypot(kx, kz) / np.hypot(modified_k(kx, dx, p), modified_k(kz, dz, p))


# ---------------------------------------------------------------- Appendix A
def appendix_eta_beta(theta):
    """Courant number and beta' that cancel the k^4 and k^6 dispersion at angle theta."""
    cs2 = np.cos(theta) ** 2 * np.sin(theta) ** 2
    eta = 0.5 * np.sqrt(5.0 - np.sqrt(1.0 + 32.0 * cs2))
    with np.errstate(invalid="ignore", divide="ignore"):
        beta = (1.0 - eta ** 2 - 2.0 * cs2) / (3.0 * cs2)
    return eta, beta


def appendix_eta_stable(beta_prime):
    """Nyquist-mode stability bound of Appendix A: eta_stable^2 = 1/(2 + beta')."""
    return np.sqrt(1.0 / (2.0 + beta_prime))


# ---------------------------------------------------------------- Yee stepper
def yee_step_s_pol(Ey, Bx, Bz, dx, dz, dt, c=1.0):
    """One leapfrog step of the 2D Yee scheme for (Ey, Bx, Bz) on a periodic grid.

    Arrays are [z][x].  Ey lives at nodes (i, k) and integer times; Bx at
    (i, k+1/2) and Bz at (i+1/2, k), both at half-integer times:
      Bx += dt dEy/dz,  Bz -= dt dEy/dx,  Ey += c^2 dt (dBx/dz - dBz/dx).
    """
    Bx = Bx + dt * (np.roll(Ey, -1, axis=0) - Ey) / dz
    Bz = Bz - dt * (np.roll(Ey, -1, axis=1) - Ey) / dx
    Ey = Ey + c * c * dt * ((Bx - np.roll(Bx, 1, axis=0)) / dz
                            - (Bz - np.roll(Bz, 1, axis=1)) / dx)
    return Ey, Bx, Bz


def yee_lattice_mode(nx, nz, mx, mz, dx, dz, dt, c=1.0):
    """Complex Yee eigenmode exp(i(k.x - w t)) at t = 0 with B at t = -dt/2.

    Returns (Ey, Bx, Bz, omega) with omega from :func:`omega_fdtd`.
    """
    kx = 2 * np.pi * mx / (nx * dx)
    kz = 2 * np.pi * mz / (nz * dz)
    w = float(omega_fdtd(kx, kz, dx, dz, dt, c))
    x = np.arange(nx) * dx
    z = np.arange(nz) * dz
    s = np.sin(0.5 * w * dt)
    Ey = np.exp(1j * (kx * x[None, :] + kz * z[:, None]))
    phase_b = np.exp(1j * w * dt / 2)  # B^{-1/2}
    Bx = -(dt / dz) * np.sin(kz * dz / 2) / s * np.exp(
        1j * (kx * x[None, :] + kz * (z[:, None] + dz / 2))) * phase_b
    Bz = (dt / dx) * np.sin(kx * dx / 2) / s * np.exp(
        1j * (kx * (x[None, :] + dx / 2) + kz * z[:, None])) * phase_b
    return Ey, Bx, Bz, w
