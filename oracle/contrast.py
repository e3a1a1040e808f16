"""FDTD (Yee, order-p, CKC) and PSTD field steps, FP64 -- TEST INFRASTRUCTURE.

These are the solvers the paper contrasts with PSATD (Sec. III.A and
Table 1): finite differences in time for all of them, finite differences in
space for FDTD and spectral derivatives for PSTD.  Each is a leapfrog: E at
integer times, B at half-integer times.  One step takes E^n, B^{n-1/2} and
J^{n+1/2} to
    B^{n+1/2} = B^{n-1/2} - dt curl E^n                       (Faraday)
    E^{n+1}   = E^n + dt (c^2 curl B^{n+1/2} - J^{n+1/2} / eps0)  (Ampere)

FDTD on the Yee grid (Sec. III.A).  Components sit at staggered positions:
    Ex (i+1/2, j, k)      Ey (i, j+1/2, k)      Ez (i, j, k+1/2)
    Bx (i, j+1/2, k+1/2)  By (i+1/2, j, k+1/2)  Bz (i+1/2, j+1/2, k)
and J with E.  Array element [k][j][i] ([k][i] in 2D, where y-derivatives
vanish) holds a component at its own position.  The curl of E uses forward
differences, the curl of B backward ones; at order p (Table 1, FDTD p-order
row) with the staggered weights C_l of Sec. III.B:
    D+ f[i] = sum_l C_l (f[i+l] - f[i-l+1]) / d      (p = 2: f[i+1] - f[i])
    D- f[i] = sum_l C_l (f[i+l-1] - f[i-l]) / d      (p = 2: f[i] - f[i-1])
Both have the symbol i k_p, k_p = sum_l C_l (2/d) sin((2l-1) k d/2), taken
at each component's own position.
CKC (2D, dx = dz, beta = 1/4; Table 1, CKC row): in the curl of E only, each
x-difference is averaged over z and each z-difference over x with weights
(1 - beta, beta/2, beta/2), which multiplies its symbol by
A = (1 - beta) + beta cos(k_other d_other).

PSTD (Table 1, PSTD row): collocated grid, spectral derivatives with the
k tables of the PSATD oracle (Nyquist -> 0; order p optional), so the curl
of a mode is i k x (.).

Grids are periodic.  Arrays are real ([z][x] or [z][y][x]); the steppers
also accept complex arrays (lattice eigenmode pins).
"""

from __future__ import annotations

import numpy as np
import scipy.fft as sfft

from .dispersion import BETA_CKC, fornberg_staggered
from .psatd import _kvectors, forward, inverse

SCHEMES = ("yee", "ckc")


def _axis(shape, a):
    """Array axis of spatial axis a (0 = x, 1 = y, 2 = z), or None (y in 2D)."""
    if len(shape) == 2:
        return {0: 1, 1: None, 2: 0}[a]
    return {0: 2, 1: 1, 2: 0}[a]


def _dplus(f, a, d, weights):
    ax = _axis(f.shape, a)
    if ax is None:
        return np.zeros_like(f)
    out = np.zeros_like(f)
    for l, cl in enumerate(weights, start=1):
        out = out + cl * (np.roll(f, -l, axis=ax) - np.roll(f, l - 1, axis=ax))
    return out / d[a]


def _dminus(f, a, d, weights):
    ax = _axis(f.shape, a)
    if ax is None:
        return np.zeros_like(f)
    out = np.zeros_like(f)
    for l, cl in enumerate(weights, start=1):
        out = out + cl * (np.roll(f, -(l - 1), axis=ax) - np.roll(f, l, axis=ax))
    return out / d[a]


def _smooth(g, a, beta):
    """CKC transverse average of g along spatial axis a."""
    ax = _axis(g.shape, a)
    return (1.0 - beta) * g + 0.5 * beta * (np.roll(g, -1, axis=ax) + np.roll(g, 1, axis=ax))


def fdtd_weights(order):
    """Staggered weights C_1..C_{p/2} as floats (order 0 or 2: Yee)."""
    p = 2 if order in (0, 2) else order
    return [float(w) for w in fornberg_staggered(p)]


def fdtd_step(E, B, J=None, *, d, dt, c=1.0, eps0=1.0, scheme="yee", order=2):
    """One leapfrog step of the Yee (order p) or CKC scheme; returns (E', B')."""
    if scheme not in SCHEMES:
        raise ValueError(f"unknown scheme {scheme!r}")
    w = fdtd_weights(order)
    if scheme == "ckc":
        if len(E[0].shape) != 2 or order not in (0, 2):
            raise ValueError("CKC is the 2D second-order scheme")
        beta = BETA_CKC

        def dp(f, a):  # x-differences averaged along z, z-differences along x
            return _smooth(_dplus(f, a, d, w), 2 if a == 0 else 0, beta)
    else:
        def dp(f, a):
            return _dplus(f, a, d, w)

    def dm(f, a):
        return _dminus(f, a, d, w)

    Ex, Ey, Ez = E
    Bx = B[0] - dt * (dp(Ez, 1) - dp(Ey, 2))
    By = B[1] - dt * (dp(Ex, 2) - dp(Ez, 0))
    Bz = B[2] - dt * (dp(Ey, 0) - dp(Ex, 1))
    c2 = c * c
    curl = (dm(Bz, 1) - dm(By, 2), dm(Bx, 2) - dm(Bz, 0), dm(By, 0) - dm(Bx, 1))
    En = []
    for i in range(3):
        e = E[i] + dt * c2 * curl[i]
        if J is not None:
            e = e - (dt / eps0) * J[i]
        En.append(e)
    return En, [Bx, By, Bz]


def pstd_step(E, B, J=None, *, d, dt, c=1.0, eps0=1.0, order=0, stencil="staggered",
              workers=None):
    """One PSTD leapfrog step on the collocated grid; returns (E', B').

    Real inputs use r2c transforms; complex inputs (lattice-mode pins) use
    c2c transforms and stay complex.
    """
    shape = E[0].shape
    cplx = np.iscomplexobj(E[0]) or np.iscomplexobj(B[0])
    if cplx:
        kx, ky, kz = _kvectors(shape, d, "c2c", order, stencil)
        fwd = lambda f: sfft.fftn(np.asarray(f, dtype=np.complex128))  # noqa: E731
        inv = lambda F: sfft.ifftn(F)  # noqa: E731
    else:
        kx, ky, kz = _kvectors(shape, d, "r2c", order, stencil)
        fwd = lambda f: forward(f, "r2c", workers)  # noqa: E731
        inv = lambda F: inverse(F, shape, "r2c", workers)  # noqa: E731
    Ek = [fwd(f) for f in E]
    Bk = [fwd(f) for f in B]
    # B^{n+1/2} = B^{n-1/2} - i dt k x E^n
    kxE = (ky * Ek[2] - kz * Ek[1], kz * Ek[0] - kx * Ek[2], kx * Ek[1] - ky * Ek[0])
    Bn = [Bk[i] - 1j * dt * kxE[i] for i in range(3)]
    # E^{n+1} = E^n + i c^2 dt k x B^{n+1/2} - dt J / eps0
    kxB = (ky * Bn[2] - kz * Bn[1], kz * Bn[0] - kx * Bn[2], kx * Bn[1] - ky * Bn[0])
    En = [Ek[i] + 1j * c * c * dt * kxB[i] for i in range(3)]
    if J is not None:
        for i in range(3):
            En[i] = En[i] - (dt / eps0) * fwd(J[i])
    return [inv(f) for f in En], [inv(f) for f in Bn]


def courant_limit(scheme, d, ndim, c=1.0, order=0):
    """Largest stable dt (Table 1, Courant column, for any spacings).

    yee / order p: c dt sqrt(sum_a (sum_l |C_l| / d_a)^2) <= 1
    ckc:           c dt <= dx (= dz)
    pstd:          c dt |k|max / 2 <= 1 with |k|max the corner of the exact
                   (order 0) or order-p table, bounded by pi / d_a per axis
                   (sum_l 2 |C_l| / d_a at order p).
    """
    axes = (0, 2) if ndim == 2 else (0, 1, 2)
    if scheme == "ckc":
        return d[0] / c
    if scheme == "pstd":
        per = (lambda a: np.pi / d[a]) if order == 0 else (
            lambda a: 2.0 * sum(abs(x) for x in fdtd_weights(order)) / d[a])
        return 2.0 / (c * np.sqrt(sum(per(a) ** 2 for a in axes)))
    s = sum(abs(x) for x in fdtd_weights(order))
    return 1.0 / (c * np.sqrt(sum((s / d[a]) ** 2 for a in axes)))


# ---------------------------------------------------------------- lattice modes
def yee_positions(shape, d):
    """Staggered positions (x, y, z) of the six components, as broadcastable grids.

    Order: Ex, Ey, Ez, Bx, By, Bz.  Offsets in cells per axis.
    """
    offs = [(0.5, 0, 0), (0, 0.5, 0), (0, 0, 0.5), (0, 0.5, 0.5), (0.5, 0, 0.5), (0.5, 0.5, 0)]
    if len(shape) == 2:
        nz, nx = shape
        grids = [(np.arange(nx)[None, :], None, np.arange(nz)[:, None])]
    else:
        nz, ny, nx = shape
        grids = [(np.arange(nx)[None, None, :], np.arange(ny)[None, :, None],
                  np.arange(nz)[:, None, None])]
    gx, gy, gz = grids[0]
    out = []
    for o in offs:
        x = (gx + o[0]) * d[0]
        y = 0.0 if gy is None else (gy + o[1]) * d[1]
        z = (gz + o[2]) * d[2]
        out.append((x, y, z))
    return out


def amplification_matrix(step, shape, m, d, staggered):
    """6 x 6 one-step matrix of a linear vacuum stepper on lattice mode m.

    Each component j is set to exp(i k . x_j) (x_j its own position on the
    Yee grid when ``staggered``, the grid node otherwise), the others to
    zero; one step is taken and the amplitude of every component at its own
    position is read back.  The eigenvalues are exp(-+ i omega dt) of the
    waves and 1 of the static modes.
    """
    if len(shape) == 2:
        n = (shape[1], 1, shape[0])
    else:
        n = (shape[2], shape[1], shape[0])
    k = [2 * np.pi * m[a] / (n[a] * d[a]) for a in range(3)]
    pos = yee_positions(shape, d) if staggered else [_nodes(shape, d)] * 6
    phases = [np.exp(1j * (k[0] * x + k[1] * y + k[2] * z)) * np.ones(shape) for x, y, z in pos]
    M = np.zeros((6, 6), dtype=complex)
    for j in range(6):
        F = [np.zeros(shape, dtype=complex) for _ in range(6)]
        F[j] = phases[j].copy()
        En, Bn = step(F[:3], F[3:])
        out = list(En) + list(Bn)
        for i in range(6):
            M[i, j] = np.mean(out[i] / phases[i])
    return M


def _nodes(shape, d):
    if len(shape) == 2:
        nz, nx = shape
        return np.arange(nx)[None, :] * d[0], 0.0, np.arange(nz)[:, None] * d[2]
    nz, ny, nx = shape
    return (np.arange(nx)[None, None, :] * d[0], np.arange(ny)[None, :, None] * d[1],
            np.arange(nz)[:, None, None] * d[2])
