"""PSATD field step in FP64: forward FFT, per-mode analytic update, inverse FFT.

TEST INFRASTRUCTURE (see the package docstring): nothing in the product path
imports this module.

What the method computes (Sec. III.B, item 2; Table 1, PSATD row): in
(k, t) space Maxwell's equations are integrated analytically over one time
step with the sources held constant during the step, which makes the vacuum
dispersion-free (refractive index exactly 1) with no Courant condition.  The
paper cites the update without printing it, so it is derived here from

    dE/dt = c^2 curl B - J/eps0,   dB/dt = -curl E,
    div E = rho/eps0,              div B = 0,

with the forward transform  f^(k) = sum_x f(x) exp(-i k.x),  so curl -> i k x.
Write K = |k|, w = cK, theta = w dt.  Split E^ into its transverse part and
its longitudinal part k_hat (k_hat . E^).

* Transverse E^ and B^ form a driven oscillator: d2E_T/dt2 = -w^2 E_T for
  constant J, so over one step
      E_T' = C E_T + i c^2 S (k x B^) - (S/eps0) J_T,
      B'   = C B^  - i S (k x E^) + i X1 (k x J^),
  with C = cos theta, S = sin(theta)/w, X1 = (1 - C)/(eps0 c^2 K^2).
  (B^ is transverse because div B = 0.)
* Longitudinal E: dE_L/dt = -J_L/eps0.  Two equivalent closures:
  - J-form: E_L' = E_L - (dt/eps0) J_L.
  - rho-form: Gauss's law gives E_L = -i k rho^/(eps0 K^2) at both ends of
    the step, with rho varying linearly in time (continuity
    rho^_new = rho^_old - i dt k.J^).
  Adding the closure to the transverse update gives, for every k,

  rho-form  E^' = C E^ + i c^2 S (k x B^) - (S/eps0) J^ + i k (X3 rho^_old - X2 rho^_new)
  J-form    E^' = C E^ + i c^2 S (k x B^) - (S/eps0) J^
                  + eps0 c^2 X1 k (k.E^) - dt X2 k (k.J^)
            B^' = C B^ - i S (k x E^) + i X1 (k x J^)

  with X2 = (1 - sin(theta)/theta)/(eps0 K^2), X3 = (C - sin(theta)/theta)/(eps0 K^2).
  At k = 0: E^' = E^ - (dt/eps0) J^, B^' = B^.

Readings where the paper is silent:
  * grid: collocated, all components at the cell nodes;
  * Nyquist: the wavenumber of the Nyquist index of an even axis is 0 in both
    the curl and |k|, so real fields stay real and r2c == c2c;
  * wavevector: exact k (infinite order) by default; order p > 0 replaces
    every 1-D k table by k_p, the Fourier transform of the order-p staggered
    stencil (Sec. III.B; Table 1 caption), before the Nyquist rule;
  * sources: J = J^{n+1/2} constant over the step, rho_old = rho^n,
    rho_new = rho^{n+1}.
"""

from __future__ import annotations

import os

import numpy as np
import scipy.fft as sfft

from .dispersion import modified_k

_WORKERS = os.cpu_count() or 1


# ---------------------------------------------------------------- k tables
def ktable(n: int, d: float, order: int = 0, stencil: str = "staggered") -> np.ndarray:
    """Lattice wavenumbers of a full (c2c) axis in fftfreq order, Nyquist -> 0.

    ``order`` = p > 0 replaces k by the order-p modified wavevector k_p
    (Sec. III.B; Table 1 caption) of the ``stencil`` ("staggered", the
    default, or "centered"); 0 keeps the exact k.
    """
    m = np.arange(n)
    m = np.where(m < (n + 1) // 2, m, m - n).astype(np.float64)
    k = 2.0 * np.pi * m / (n * d)
    if order:
        k = modified_k(k, d, order, stencil)
    if n % 2 == 0:
        k[n // 2] = 0.0
    return k


def rktable(n: int, d: float, order: int = 0, stencil: str = "staggered") -> np.ndarray:
    """Wavenumbers of the halved r2c axis (indices 0..n/2), Nyquist -> 0."""
    return ktable(n, d, order, stencil)[: n // 2 + 1]


def _kvectors(shape, d, transform, order=0, stencil="staggered"):
    """Broadcastable (kx, ky, kz) for spectra of arrays shaped [z][x] or [z][y][x]."""
    kx_fn = rktable if transform == "r2c" else ktable
    if len(shape) == 2:
        nz, nx = shape
        kx = kx_fn(nx, d[0], order, stencil)[None, :]
        kz = ktable(nz, d[2], order, stencil)[:, None]
        ky = np.zeros((1, 1))
    else:
        nz, ny, nx = shape
        kx = kx_fn(nx, d[0], order, stencil)[None, None, :]
        ky = ktable(ny, d[1], order, stencil)[None, :, None]
        kz = ktable(nz, d[2], order, stencil)[:, None, None]
    return kx, ky, kz


# ---------------------------------------------------------------- coefficients
def _sinc(t):
    """sin(t)/t with the value 1 at t = 0."""
    out = np.ones_like(t)
    nz = t != 0.0
    out[nz] = np.sin(t[nz]) / t[nz]
    return out


def g_series(theta):
    """g(theta) = (1 - sin(theta)/theta) / theta^2 without cancellation.

    For theta < 0.25 the Taylor series sum_n (-1)^n theta^(2n) / (2n+3)! is
    summed to theta^10 (truncation below 1e-19 relative); above, the direct
    form loses at most ~1e-14 relative.
    """
    theta = np.asarray(theta, dtype=np.float64)
    t2 = theta * theta
    series = (1.0 / 6.0 - t2 * (1.0 / 120.0 - t2 * (1.0 / 5040.0 - t2 * (
        1.0 / 362880.0 - t2 * (1.0 / 39916800.0 - t2 / 6227020800.0)))))
    small = theta < 0.25
    safe = np.where(small, 1.0, theta)
    direct = (1.0 - np.sin(safe) / safe) / (safe * safe)
    return np.where(small, series, direct)


def psatd_coefficients(K, dt, c=1.0, eps0=1.0):
    """C, S, X1, X2, X3 of the update for |k| = K, in forms finite at K = 0.

    C  = cos(theta)
    S  = sin(theta)/(cK)                    = dt sinc(theta)           -> dt
    X1 = (1 - C)/(eps0 c^2 K^2)             = dt^2 sinc(theta/2)^2/(2 eps0)
    X2 = (1 - sinc theta)/(eps0 K^2)        = c^2 dt^2 g(theta)/eps0   -> c^2 dt^2/(6 eps0)
    X3 = (C - sinc theta)/(eps0 K^2)        = c^2 dt^2 (g - sinc(theta/2)^2/2)/eps0
                                                                       -> -c^2 dt^2/(3 eps0)
    None of 1 - cos(theta) or 1 - sin(theta)/theta is formed by subtraction
    near theta = 0.
    """
    K = np.asarray(K, dtype=np.float64)
    theta = c * K * dt
    half = _sinc(0.5 * theta)
    g = g_series(theta)
    C = np.cos(theta)
    S = dt * _sinc(theta)
    X1 = dt * dt * half * half / (2.0 * eps0)
    X2 = c * c * dt * dt * g / eps0
    X3 = c * c * dt * dt * (g - 0.5 * half * half) / eps0
    return {"C": C, "S": S, "X1": X1, "X2": X2, "X3": X3}


def _cross(a, b):
    return (a[1] * b[2] - a[2] * b[1],
            a[2] * b[0] - a[0] * b[2],
            a[0] * b[1] - a[1] * b[0])


def update_modes(Ek, Bk, k, dt, *, c=1.0, eps0=1.0, Jk=None, rho_old_k=None,
                 rho_new_k=None, form="rho"):
    """Advance spectra (E^, B^) by one step at wavevectors k = (kx, ky, kz).

    ``form``: "rho" (rho_old and rho_new enter through Gauss's law) or "J"
    (continuity implied; rho is not used).  Sources may be None (vacuum).
    Returns (E^', B^') as lists of three complex arrays.
    """
    kx, ky, kz = k
    K = np.sqrt(kx * kx + ky * ky + kz * kz)
    co = psatd_coefficients(K, dt, c, eps0)
    C, S, X1, X2, X3 = co["C"], co["S"], co["X1"], co["X2"], co["X3"]
    kv = (kx, ky, kz)
    kxB = _cross(kv, Bk)
    kxE = _cross(kv, Ek)
    Enew = [C * Ek[i] + 1j * c * c * S * kxB[i] for i in range(3)]
    Bnew = [C * Bk[i] - 1j * S * kxE[i] for i in range(3)]
    if form == "J":
        kdotE = kx * Ek[0] + ky * Ek[1] + kz * Ek[2]
        for i in range(3):
            Enew[i] = Enew[i] + eps0 * c * c * X1 * kv[i] * kdotE
    if Jk is not None:
        kxJ = _cross(kv, Jk)
        for i in range(3):
            Enew[i] = Enew[i] - (S / eps0) * Jk[i]
            Bnew[i] = Bnew[i] + 1j * X1 * kxJ[i]
        if form == "J":
            kdotJ = kx * Jk[0] + ky * Jk[1] + kz * Jk[2]
            for i in range(3):
                Enew[i] = Enew[i] - dt * X2 * kv[i] * kdotJ
    if form == "rho" and (rho_old_k is not None or rho_new_k is not None):
        ro = rho_old_k if rho_old_k is not None else 0.0
        rn = rho_new_k if rho_new_k is not None else 0.0
        lam = X3 * ro - X2 * rn
        for i in range(3):
            Enew[i] = Enew[i] + 1j * kv[i] * lam
    return Enew, Bnew


# ---------------------------------------------------------------- transforms
def forward(f, transform="r2c", workers=None):
    """Unnormalized forward DFT over all axes (r2c halves the last, x, axis)."""
    w = workers or _WORKERS
    if transform == "r2c":
        return sfft.rfftn(np.asarray(f, dtype=np.float64), workers=w)
    return sfft.fftn(np.asarray(f, dtype=np.complex128), workers=w)


def inverse(F, shape, transform="r2c", workers=None):
    """Inverse of :func:`forward`, with the 1/N normalization; returns real arrays."""
    w = workers or _WORKERS
    if transform == "r2c":
        return sfft.irfftn(F, s=shape, workers=w)
    out = sfft.ifftn(F, workers=w)
    scale = max(np.max(np.abs(out.real)), 1e-300)
    imag = np.max(np.abs(out.imag))
    if imag > 1e-12 * scale:
        raise AssertionError(f"c2c step left an imaginary part {imag:.3e} (scale {scale:.3e})")
    return out.real


# ---------------------------------------------------------------- the step
def psatd_step(E, B, J=None, rho_old=None, rho_new=None, *, d, dt, c=1.0, eps0=1.0,
               form="rho", transform="r2c", order=0, stencil="staggered", workers=None):
    """One PSATD step on a periodic grid.

    E, B: three real arrays each ([z][x] or [z][y][x]); J: three arrays or None;
    rho_old, rho_new: arrays or None.  ``d`` = (dx, dy, dz) (dy unused in 2D).
    ``order`` selects the order-p wavevector (0: exact k) of ``stencil``.
    Steps, in the method's order: forward FFT of every input, the per-mode
    update of :func:`update_modes`, inverse FFT of E and B.
    """
    shape = E[0].shape
    k = _kvectors(shape, d, transform, order, stencil)
    Ek = [forward(f, transform, workers) for f in E]
    Bk = [forward(f, transform, workers) for f in B]
    Jk = [forward(f, transform, workers) for f in J] if J is not None else None
    ro = forward(rho_old, transform, workers) if rho_old is not None else None
    rn = forward(rho_new, transform, workers) if rho_new is not None else None
    En, Bn = update_modes(Ek, Bk, k, dt, c=c, eps0=eps0, Jk=Jk, rho_old_k=ro,
                          rho_new_k=rn, form=form)
    return ([inverse(f, shape, transform, workers) for f in En],
            [inverse(f, shape, transform, workers) for f in Bn])


def psatd_run(E, B, steps, *, d, dt, schedule=None, c=1.0, eps0=1.0, form="rho",
              transform="r2c", order=0, stencil="staggered", source_dtype=np.float64,
              workers=None, callback=None):
    """``steps`` successive steps; sources of step n come from ``schedule.sources(n)``.

    ``source_dtype`` rounds the sources before use (float32 reproduces what an
    FP32 caller hands over).  ``callback(n, E, B)`` runs after each step.
    """
    E = [np.asarray(f, dtype=np.float64) for f in E]
    B = [np.asarray(f, dtype=np.float64) for f in B]
    for n in range(steps):
        if schedule is not None:
            J, ro, rn = schedule.sources(n, dtype=source_dtype)
            J = [np.asarray(f, dtype=np.float64) for f in J]
            ro = np.asarray(ro, dtype=np.float64)
            rn = np.asarray(rn, dtype=np.float64)
        else:
            J = ro = rn = None
        E, B = psatd_step(E, B, J, ro, rn, d=d, dt=dt, c=c, eps0=eps0, form=form,
                          transform=transform, order=order, stencil=stencil, workers=workers)
        if callback is not None:
            callback(n, E, B)
    return E, B


def field_energy(E, B, c=1.0, eps0=1.0):
    """sum over cells of (eps0/2)(|E|^2 + c^2 |B|^2) (cell volume omitted)."""
    return 0.5 * eps0 * (sum(np.sum(f * f) for f in E) + c * c * sum(np.sum(f * f) for f in B))
