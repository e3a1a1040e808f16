"""The refraction model of Sec. IV (eq. 1) -- TEST INFRASTRUCTURE.

Harmonics leave the plasma surface as if from a non-dispersive medium of index
n_i = 1 at the incidence angle theta_i, and enter the numerical vacuum of the
solver, whose refractive index n_r depends on the frequency and on the
propagation angle.  The Snell-Descartes law

    n_i sin(theta_i) = n_r(omega, theta_r) sin(theta_r)

has theta_r(omega) as its unknown; the paper solves it by an iterative method
(Newton-Raphson).  Here:

- ``omega_num(solver, kx, kz, ...)``: the solver's numerical frequency of the
  lattice mode k (Table 1 rows: Yee, CKC, PSTD(-p), PSATD(-p)).
- ``index_at(solver, omega, theta, ...)``: n_r(omega, theta) = c |k| / omega,
  where |k| along the direction theta solves omega_num(k) = omega (bisection
  on the monotonic branch inside the first Brillouin zone, then Newton).
  NaN when no propagating mode of that frequency exists along theta.
- ``refraction_angle(solver, omega, theta_i, ...)``: theta_r by Newton-Raphson
  on f(theta) = n_r(omega, theta) sin(theta) - n_i sin(theta_i) from
  theta = theta_i, the derivative by a central difference.  NaN beyond total
  reflection (no theta_r in [0, pi/2) satisfies eq. 1).

Readings (the paper does not fix them): theta is measured from the normal of
the plasma surface, taken along the grid's x axis, in the (x, z) plane of the
2D simulations, so the direction of propagation is (cos theta, sin theta);
omega and k in the normalized units of the rest of the oracle (c = 1).
"""

from __future__ import annotations

import numpy as np

from .dispersion import BETA_CKC, modified_k, omega_fdtd


def omega_num(solver, kx, kz, dx, dz, dt, c=1.0, order=0, stencil="staggered"):
    """Numerical frequency of the lattice mode (kx, kz) (2D).

    yee, ckc: sin(w dt/2) = c dt sqrt(sum_X A_X sin^2(k_X dX/2) / dX^2)
    pstd:     sin(w dt/2) = c dt |k_p| / 2      (k_p = k for order 0)
    psatd:    w = c |k_p|                        (exact time integration)
    """
    if solver in ("yee", "ckc"):
        return omega_fdtd(kx, kz, dx, dz, dt, c, BETA_CKC if solver == "ckc" else 0.0)
    kp = np.hypot(modified_k(kx, dx, order, stencil), modified_k(kz, dz, order, stencil))
    if solver == "pstd":
        a = 0.5 * c * dt * kp
        with np.errstate(invalid="ignore"):
            return np.where(a <= 1.0, 2.0 / dt * np.arcsin(np.minimum(a, 1.0)), np.nan)
    if solver == "psatd":
        return c * kp
    raise ValueError(f"unknown solver {solver!r}")


def _k_edge(theta, dx, dz):
    """|k| at which the direction theta leaves the first Brillouin zone."""
    cx, sz = abs(np.cos(theta)), abs(np.sin(theta))
    edges = []
    if cx > 0:
        edges.append(np.pi / dx / cx)
    if sz > 0:
        edges.append(np.pi / dz / sz)
    return min(edges)


def index_at(solver, omega, theta, dx, dz, dt, c=1.0, order=0, stencil="staggered"):
    """n_r(omega, theta) = c |k| / omega for the mode of frequency omega
    propagating along theta (NaN if there is none)."""
    if not np.isfinite(theta):
        return np.nan
    ct, st = np.cos(theta), np.sin(theta)
    hi = _k_edge(theta, dx, dz)
    # the dispersion branch rises from 0 along the direction; keep the part
    # where it still rises (and is defined), so the root is bracketed and unique
    ks = np.linspace(0.0, hi, 513)
    w = np.asarray(omega_num(solver, ks * ct, ks * st, dx, dz, dt, c, order, stencil), float)
    stop = np.nonzero(~np.isfinite(w[1:]) | (np.diff(w) < 0.0))[0]
    top = int(stop[0]) if stop.size else len(ks) - 1
    if not w[top] >= omega:
        return np.nan
    i = max(int(np.searchsorted(w[: top + 1], omega)), 1)
    lo, hi = ks[i - 1], ks[i]

    def f(k):
        return float(omega_num(solver, k * ct, k * st, dx, dz, dt, c, order, stencil)) - omega

    for _ in range(80):  # bisection within the bracket
        mid = 0.5 * (lo + hi)
        if f(mid) < 0.0:
            lo = mid
        else:
            hi = mid
        if hi - lo <= 4e-16 * hi:
            break
    return c * 0.5 * (lo + hi) / omega


def refraction_angle(solver, omega, theta_i, dx, dz, dt, c=1.0, n_i=1.0, order=0,
                     stencil="staggered", tol=1e-15, maxiter=100):
    """theta_r solving n_i sin(theta_i) = n_r(omega, theta_r) sin(theta_r)
    (eq. 1) by Newton-Raphson; NaN when no solution exists in [0, pi/2)."""
    target = n_i * np.sin(theta_i)

    def g(th):
        return index_at(solver, omega, th, dx, dz, dt, c, order, stencil) * np.sin(th) - target

    th = float(theta_i)
    h = 1e-6
    for _ in range(maxiter):
        gv = g(th)
        if not np.isfinite(gv):
            return np.nan
        if abs(gv) <= tol:
            return th
        d = (g(min(th + h, np.pi / 2 - 1e-12)) - g(max(th - h, 0.0))) / (
            min(th + h, np.pi / 2 - 1e-12) - max(th - h, 0.0))
        if not np.isfinite(d) or d == 0.0:
            return np.nan
        step = gv / d
        new = th - step
        if new >= np.pi / 2:  # past grazing: no refracted wave (total reflection)
            new = 0.5 * (th + np.pi / 2)
            if np.pi / 2 - new < 1e-9:
                return np.nan
        th = max(new, 0.0)
        if abs(step) <= 1e-16:
            return th if abs(g(th)) <= 1e-12 else np.nan
    return th if abs(g(th)) <= 1e-12 else np.nan


def index_map(solver, eta, kdx, theta, dx=1.0, c=1.0, order=0, stencil="staggered"):
    """Refractive-index map of Fig. 2: n = c |k| / omega_num(k) on the grid of
    wavenumbers |k| dx = ``kdx`` (1D array) and directions ``theta`` (1D
    array, radians from the x axis), at Courant number eta = c dt / dx (square
    cells).  Returns an array [len(theta), len(kdx)]; NaN where the scheme has
    no stable mode."""
    K, T = np.meshgrid(np.asarray(kdx, float) / dx, np.asarray(theta, float))
    w = omega_num(solver, K * np.cos(T), K * np.sin(T), dx, dx, eta * dx / c, c, order, stencil)
    with np.errstate(invalid="ignore", divide="ignore"):
        return np.where(K > 0, c * K / w, 1.0)
