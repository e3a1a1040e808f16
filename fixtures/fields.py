"""Field and source generators (numpy, FP64).

Every generator takes a ``numpy.random.Generator`` (PCG64) so that the same
seed gives the same arrays on every machine.  Spectral helpers use the
lattice wavevector k_j = 2*pi*m_j / (N*d) (numpy ``fftfreq`` order) with the
Nyquist index of an even axis set to k = 0, so that derivatives of real
fields stay real.
"""

from __future__ import annotations

import os

import numpy as np
import scipy.fft as sfft

_WORKERS = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else (os.cpu_count() or 1)


def _fftn(a):
    return sfft.fftn(a, workers=_WORKERS)


def _ifftn(a):
    return sfft.ifftn(a, workers=_WORKERS)


LAMBDA0 = 1.0
C_LIGHT = 1.0
OMEGA0 = 2.0 * np.pi * C_LIGHT / LAMBDA0


# ---------------------------------------------------------------- k-space helpers
def lattice_k(n: int, d: float) -> np.ndarray:
    """Full-length lattice wavenumbers of an axis of n points and spacing d."""
    k = 2.0 * np.pi * np.fft.fftfreq(n, d=d)
    if n % 2 == 0:
        k[n // 2] = 0.0
    return k


def _kgrid(shape, d):
    """Broadcastable (kx, ky, kz) for arrays shaped [z][x] or [z][y][x].

    ``d`` is (dx, dy, dz); dy is ignored in 2D.
    """
    if len(shape) == 2:
        nz, nx = shape
        kx = lattice_k(nx, d[0])[None, :]
        kz = lattice_k(nz, d[2])[:, None]
        ky = np.zeros((1, 1))
    else:
        nz, ny, nx = shape
        kx = lattice_k(nx, d[0])[None, None, :]
        ky = lattice_k(ny, d[1])[None, :, None]
        kz = lattice_k(nz, d[2])[:, None, None]
    return kx, ky, kz


def spectral_grad(f, d):
    """(d/dx, d/dy, d/dz) of a real periodic array, evaluated spectrally."""
    fh = _fftn(f)
    return tuple(np.real(_ifftn(1j * k * fh)) for k in _kgrid(f.shape, d))


def spectral_div(F, d):
    """div of a real periodic vector field (3 arrays), evaluated spectrally."""
    kx, ky, kz = _kgrid(F[0].shape, d)
    acc = 1j * (kx * _fftn(F[0]) + ky * _fftn(F[1]) + kz * _fftn(F[2]))
    return np.real(_ifftn(acc))


def project_transverse(F, d):
    """Remove the longitudinal (curl-free) part of a vector field; the mean is kept."""
    kx, ky, kz = _kgrid(F[0].shape, d)
    Fh = [_fftn(f) for f in F]
    k2 = kx * kx + ky * ky + kz * kz
    inv = np.zeros_like(k2)
    np.divide(1.0, k2, out=inv, where=k2 > 0)
    kdot = (kx * Fh[0] + ky * Fh[1] + kz * Fh[2]) * inv
    out = []
    for f, k in zip(Fh, (kx, ky, kz)):
        out.append(np.real(_ifftn(f - k * kdot)))
    return out


# ---------------------------------------------------------------- laser fields
def _harmonic_comb(xi, nharm, rng, first_phase_zero=True):
    """sum_n a_n cos(n k0 xi + phi_n), a_n = n^(-4/3); phases drawn in order."""
    k0 = 2.0 * np.pi / LAMBDA0
    phases = rng.uniform(0.0, 2.0 * np.pi, size=nharm)
    if first_phase_zero:
        phases[0] = 0.0
    s = np.zeros_like(xi)
    for n in range(1, nharm + 1):
        s += n ** (-4.0 / 3.0) * np.cos(n * k0 * xi + phases[n - 1])
    return s


def laser_2d(nx, nz, dx, dz, *, angle_deg, waist, tau, nharm, rng, amplitude=1.0):
    """p-polarized Gaussian-envelope pulse with a harmonic comb, in the (x, z) plane.

    Propagation direction (cos a, 0, sin a) with a = angle_deg; E lies in the
    (x, z) plane, B = k_hat x E / c along y.  Envelope
    exp(-r_perp^2/w^2) * exp(-xi^2/(c tau)^2), centred in the box.  Both E and B
    are projected onto their transverse (divergence-free) parts.
    """
    a = np.deg2rad(angle_deg)
    x = (np.arange(nx) - nx / 2) * dx
    z = (np.arange(nz) - nz / 2) * dz
    Z, X = np.meshgrid(z, x, indexing="ij")
    xi = X * np.cos(a) + Z * np.sin(a)
    rp = -X * np.sin(a) + Z * np.cos(a)
    env = np.exp(-(rp / waist) ** 2) * np.exp(-(xi / (C_LIGHT * tau)) ** 2)
    s = amplitude * env * _harmonic_comb(xi, nharm, rng)
    khat = np.array([np.cos(a), 0.0, np.sin(a)])
    ehat = np.array([-np.sin(a), 0.0, np.cos(a)])
    bhat = np.cross(khat, ehat) / C_LIGHT
    d = (dx, 1.0, dz)
    E = project_transverse([ehat[i] * s for i in range(3)], d)
    B = project_transverse([bhat[i] * s for i in range(3)], d)
    return E, B


def laser_3d(nx, ny, nz, d, *, angle_deg, waist, tau, nharm, rng, amplitude=1.0):
    """3D version of :func:`laser_2d`: Gaussian beam in the (x, z) plane at angle_deg.

    The pulse s(x, y, z) = A(x, z) g(y) separates: the phase coordinate xi and
    the in-plane transverse offset do not depend on y, and the envelope factor
    exp(-r_perp^2/w^2) splits into exp(-(in-plane offset)^2/w^2) exp(-y^2/w^2).
    Its spectrum is therefore one 2D transform times one 1D transform, and the
    transverse projections of e_hat s and b_hat s (both constant directions
    times s) share it: one inverse transform per output component.
    """
    a = np.deg2rad(angle_deg)
    x = (np.arange(nx) - nx / 2) * d[0]
    y = (np.arange(ny) - ny / 2) * d[1]
    z = (np.arange(nz) - nz / 2) * d[2]
    Z, X = np.meshgrid(z, x, indexing="ij")
    xi = X * np.cos(a) + Z * np.sin(a)
    rp = -X * np.sin(a) + Z * np.cos(a)
    A = amplitude * np.exp(-(rp / waist) ** 2) * np.exp(-(xi / (C_LIGHT * tau)) ** 2) \
        * _harmonic_comb(xi, nharm, rng)
    g = np.exp(-(y / waist) ** 2)
    khat = np.array([np.cos(a), 0.0, np.sin(a)])
    ehat = np.array([-np.sin(a), 0.0, np.cos(a)])
    bhat = np.cross(khat, ehat) / C_LIGHT
    # half spectrum of s: rfft over x of A, full transforms over z (of A) and y (of g)
    Ah = sfft.fft(sfft.rfft(A, axis=1, workers=_WORKERS), axis=0, workers=_WORKERS)
    gh = sfft.fft(g)
    return _project_separable((Ah, gh), (nz, ny, nx), d, (ehat, bhat))


def _project_separable(spec, shape, d, directions):
    """Transverse parts of v s for constant vectors v, with s given by its
    half spectrum s^(kz, ky, kx) = Ah(kz, kx) gh(ky) (r2c along x):
    F^_i = v_i s^ - k_i (k.v) s^ / |k|^2 (the mean is kept)."""
    Ah, gh = spec
    nz, ny, nx = shape
    KX = lattice_k(nx, d[0])[: nx // 2 + 1][None, None, :]
    KY = lattice_k(ny, d[1])[None, :, None]
    KZ = lattice_k(nz, d[2])[:, None, None]
    sh = Ah[:, None, :] * gh[None, :, None]
    k2 = KX * KX + KY * KY + KZ * KZ
    inv = np.zeros_like(k2)
    np.divide(1.0, k2, out=inv, where=k2 > 0)
    del k2
    out = []
    for v in directions:
        kv = (KX * v[0] + KY * v[1] + KZ * v[2]) * inv
        comps = []
        for i, ki in enumerate((KX, KY, KZ)):
            f = sh * (v[i] - ki * kv)
            comps.append(sfft.irfftn(f, s=shape, workers=_WORKERS))
            del f
        out.append(comps)
    return tuple(out)


def plane_wave_list(shape, d, *, nharm, max_angle_deg, rng):
    """Parameters of the lattice plane waves of :func:`plane_wave_packets_3d`.

    Returns a list of (m, e, b, phase): integer mode numbers (m_x, m_y, m_z),
    the amplitude-scaled E and B vectors, and the phase, so that each wave is
    E = e cos(2 pi m.x / N + phase), B = b cos(...).  Draws from ``rng`` in the
    same order as :func:`plane_wave_packets_3d`.
    """
    nz, ny, nx = shape
    L = (nx * d[0], ny * d[1], nz * d[2])
    k0 = 2.0 * np.pi / LAMBDA0
    lim = np.deg2rad(max_angle_deg)
    out = []
    for n in range(1, nharm + 1):
        t, p = rng.uniform(-lim, lim, size=2)
        khat = np.array([np.cos(t) * np.cos(p), np.sin(p), np.sin(t) * np.cos(p)])
        m = [int(round(n * k0 * khat[i] * L[i] / (2.0 * np.pi))) for i in range(3)]
        n_ax = (nx, ny, nz)
        for i in range(3):  # stay strictly below Nyquist
            m[i] = int(np.clip(m[i], -(n_ax[i] // 2 - 1), n_ax[i] // 2 - 1))
        kvec = np.array([2.0 * np.pi * m[i] / L[i] for i in range(3)])
        kn = np.linalg.norm(kvec)
        if kn == 0.0:
            continue
        kh = kvec / kn
        r = rng.normal(size=3)
        e = r - kh * (kh @ r)
        e /= np.linalg.norm(e)
        phase = rng.uniform(0.0, 2.0 * np.pi)
        amp = n ** (-4.0 / 3.0)
        b = np.cross(kh, e) / C_LIGHT
        out.append((tuple(m), e * amp, b * amp, phase))
    return out


def plane_wave_packets_3d(shape, d, *, nharm, max_angle_deg, rng):
    """Lattice plane waves n = 1..nharm, amplitude n^(-4/3), random directions.

    Direction k_hat = (cos t cos p, sin p, sin t cos p) with t, p uniform in
    [-max_angle, max_angle]; the wavevector n*k0*k_hat is snapped to the
    nearest lattice vector, so every wave is an exact discrete Fourier mode and
    E, B are exactly transverse without projection.  Returns (E, B, waves),
    where ``waves`` lists (m_x, m_y, m_z, e_vec, phase) for analytic checks.
    """
    nz, ny, nx = shape
    x = np.arange(nx) * d[0]
    y = np.arange(ny) * d[1]
    z = np.arange(nz) * d[2]
    L = (nx * d[0], ny * d[1], nz * d[2])
    E = [np.zeros(shape) for _ in range(3)]
    B = [np.zeros(shape) for _ in range(3)]
    waves = []
    for m, e, b, phase in plane_wave_list(shape, d, nharm=nharm, max_angle_deg=max_angle_deg,
                                          rng=rng):
        kvec = [2.0 * np.pi * m[i] / L[i] for i in range(3)]
        arg = (kvec[0] * x[None, None, :] + kvec[1] * y[None, :, None]
               + kvec[2] * z[:, None, None] + phase)
        cs = np.cos(arg)
        for i in range(3):
            E[i] += e[i] * cs
            B[i] += b[i] * cs
        waves.append((m[0], m[1], m[2], e, phase))
    return E, B, waves


# ---------------------------------------------------------------- sources
def current_factors(shape, d, *, width, nmodes, min_wavelength, rng):
    """Separable factors of the current-sheet profiles of :func:`current_profile`.

    Returns (Q, G, Gx, Qy, Qz): Q[c] of shape (nz, ny) (ny = 1 in 2D), G and
    its spectral x derivative Gx of shape (nx,), and the spectral y derivative
    of Q[1] and z derivative of Q[2] (Qy is zero in 2D), so that
    P_c = Q_c G and D = (Q_0 Gx, Qy G, Qz G).  Draws from ``rng`` in the same
    order as :func:`current_profile`.
    """
    if len(shape) == 2:
        nz, nx = shape
        ny = 1
    else:
        nz, ny, nx = shape
    x = (np.arange(nx) - nx / 2) * d[0]
    G = np.exp(-(x / width) ** 2)
    Lz = nz * d[2]
    Ly = ny * d[1]
    z = np.arange(nz) * d[2]
    y = np.arange(ny) * d[1]
    mz_max = max(1, int(np.floor(Lz / min_wavelength)))
    my_max = max(0, int(np.floor(Ly / min_wavelength))) if len(shape) == 3 else 0
    Qs = []
    for _c in range(3):
        Q = np.zeros((nz, ny))
        for _m in range(nmodes):
            mz = rng.integers(0, mz_max + 1)
            my = rng.integers(-my_max, my_max + 1) if my_max > 0 else 0
            amp = rng.normal() / np.sqrt(nmodes)
            ph = rng.uniform(0.0, 2.0 * np.pi)
            Q += amp * np.cos(2.0 * np.pi * (mz * z[:, None] / Lz + my * y[None, :] / Ly) + ph)
        Qs.append(Q)

    def deriv(f, axis, n, dd):
        # spectral derivative along one axis (lattice k, Nyquist -> 0)
        k = lattice_k(n, dd).reshape([-1 if a == axis else 1 for a in range(f.ndim)])
        return np.real(sfft.ifft(1j * k * sfft.fft(f, axis=axis), axis=axis))

    Gx = deriv(G, 0, nx, d[0])
    Qy = deriv(Qs[1], 1, ny, d[1]) if len(shape) == 3 else np.zeros_like(Qs[1])
    Qz = deriv(Qs[2], 0, nz, d[2])
    return Qs, G, Gx, Qy, Qz


def current_profile(shape, d, *, width, nmodes, min_wavelength, rng):
    """Seeded smooth current-sheet profiles P_c = G(x) Q_c(.) and their derivatives.

    G(x) = exp(-(x - x_c)^2 / width^2) (Gaussian in x, centred in the box);
    Q_c is a sum of ``nmodes`` random lattice Fourier modes along the other
    axes with wavelength >= min_wavelength.  Returns (P, D) where
    D_c = d P_c / d x_c (spectral), so that div J = sum_c f_c(t) D_c.  P_c is
    separable, so its spectral derivative along one axis is the 1D (or 2D)
    derivative of the factor that depends on that axis.
    """
    Qs, G, Gx, Qy, Qz = current_factors(shape, d, width=width, nmodes=nmodes,
                                        min_wavelength=min_wavelength, rng=rng)

    def outer(q, g):
        return q[:, 0][:, None] * g[None, :] if len(shape) == 2 else q[:, :, None] * g[None, None, :]

    P = [outer(Qs[c], G) for c in range(3)]
    D = [outer(Qs[0], Gx), outer(Qy, G) if len(shape) == 3 else np.zeros(shape), outer(Qz, G)]
    return P, D


def source_time_factors(t, phases):
    """f_c(t) = sum_n n^(-4/3) cos(n omega0 t + phi_{n,c}) for c = x, y, z.

    ``phases`` has shape (3, nharm).
    """
    nh = phases.shape[1]
    n = np.arange(1, nh + 1)
    return np.array([np.sum(n ** (-4.0 / 3.0) * np.cos(n * OMEGA0 * t + phases[c]))
                     for c in range(3)])


class SourceSchedule:
    """Per-step sources J^{n+1/2}, rho^n, rho^{n+1} with exact discrete continuity.

    J_c(x, t) = P_c(x) f_c(t).  Starting from rho^0 = 0,
    rho^{n+1} = rho^n - dt * div J^{n+1/2}, with the spectral divergence, so
    rho^n = -dt * sum_c F_c(n) D_c where F_c(n) = sum_{m<n} f_c((m + 1/2) dt).
    """

    def __init__(self, P, D, phases, dt):
        self.P = P
        self.D = D
        self.phases = phases
        self.dt = dt
        self._F = [np.zeros(3)]

    def _cum(self, n):
        while len(self._F) <= n:
            m = len(self._F) - 1
            self._F.append(self._F[-1] + source_time_factors((m + 0.5) * self.dt, self.phases))
        return self._F[n]

    def coefficients(self, n):
        """Scalars (f_c(t^{n+1/2}), F_c(n), F_c(n+1)) that define step n's sources."""
        f = source_time_factors((n + 0.5) * self.dt, self.phases)
        return f, self._cum(n), self._cum(n + 1)

    def sources(self, n, dtype=np.float64):
        f, F0, F1 = self.coefficients(n)
        J = [(self.P[c] * f[c]).astype(dtype) for c in range(3)]
        rho_old = (-self.dt * sum(F0[c] * self.D[c] for c in range(3))).astype(dtype)
        rho_new = (-self.dt * sum(F1[c] * self.D[c] for c in range(3))).astype(dtype)
        return J, rho_old, rho_new
