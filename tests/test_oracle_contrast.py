"""Pins of the contrast solvers of the oracle (oracle/contrast.py): Yee and
order-p FDTD, CKC and PSTD (Sec. III.A, Table 1).

Each stepper is pinned by what Table 1 and the mathematics fix, not by its
own formulas: the eigenvalues of its one-step matrix on a lattice mode
against the refractive-index rows (Yee, CKC, FDTD p-order, PSTD), the
Courant column (stable just below the limit, unstable just above), the
exact one-cell shift of CKC along the axes at c dt = dx (Sec. III.A), the
discrete divergence and Gauss invariants of the Yee grid, an independent s-pol
Yee stepper, the k = 0 mode, and second-order convergence of PSTD to PSATD.
"""

import numpy as np
import pytest

import oracle
from oracle import contrast as C
from oracle import dispersion as D


def _phases(M):
    ev = np.linalg.eigvals(M)
    return np.sort(np.abs(np.angle(ev))), np.abs(ev)


def _fdtd(scheme, d, dt, order=2):
    return lambda E, B: C.fdtd_step(E, B, d=d, dt=dt, scheme=scheme, order=order)


@pytest.mark.parametrize("scheme,beta", [("yee", 0.0), ("ckc", D.BETA_CKC)])
@pytest.mark.parametrize("eta", [0.3, 0.65])
def test_fdtd_2d_eigenvalues_follow_table1(scheme, beta, eta):
    d = (1.0, 1.0, 1.0)
    shape = (16, 24)
    dt = eta * d[0]
    for m in [(1, 0, 0), (3, 0, 2), (7, 0, -5), (0, 0, 8), (12, 0, 8), (11, 0, 1)]:
        ph, mag = _phases(C.amplification_matrix(_fdtd(scheme, d, dt), shape, m, d, True))
        kx, kz = 2 * np.pi * m[0] / 24, 2 * np.pi * m[2] / 16
        w = D.omega_fdtd(kx, kz, d[0], d[2], dt, beta=beta)
        assert np.allclose(ph[:2], 0.0, atol=1e-12)       # the two static modes
        assert np.allclose(ph[2:], w * dt, atol=1e-12)     # both polarizations
        assert np.allclose(mag, 1.0, atol=1e-12)


@pytest.mark.parametrize("order", [2, 4, 8])
def test_fdtd_order_p_3d_eigenvalues_follow_table1(order):
    # FDTD p-order row: sin(w dt/2) = c dt |k_p| / 2 with the staggered k_p
    d = (1.0, 0.7, 1.3)
    shape = (8, 6, 10)
    dt = 0.9 * C.courant_limit("yee", d, 3, order=order)
    for m in [(1, 2, 3), (4, -2, 1), (5, 3, -4)]:
        ph, mag = _phases(C.amplification_matrix(_fdtd("yee", d, dt, order), shape, m, d, True))
        n = (10, 6, 8)
        kp = np.sqrt(sum(D.modified_k(2 * np.pi * m[a] / (n[a] * d[a]), d[a], order) ** 2
                         for a in range(3)))
        assert np.allclose(ph[2:], 2 * np.arcsin(0.5 * dt * kp), atol=1e-12)
        assert np.allclose(mag, 1.0, atol=1e-12)


@pytest.mark.parametrize("order", [0, 4])
def test_pstd_eigenvalues_follow_table1(order):
    d = (1.0, 0.7, 1.3)
    shape = (8, 6, 10)
    dt = 0.9 * C.courant_limit("pstd", d, 3, order=order)
    n = (10, 6, 8)
    for m in [(1, 2, 3), (4, -2, 1), (3, 3, -3)]:
        M = C.amplification_matrix(lambda E, B: C.pstd_step(E, B, d=d, dt=dt, order=order),
                                   shape, m, d, False)
        ph, mag = _phases(M)
        K = np.sqrt(sum(oracle.ktable(n[a], d[a], order)[m[a] % n[a]] ** 2 for a in range(3)))
        # PSTD row: n_r = (|k| c dt/2) / arcsin(c dt |k| / 2), i.e. w = c |k| / n_r
        w = K / D.index_pstd(K, dt)
        assert np.allclose(ph[2:], w * dt, atol=1e-12)
        assert np.allclose(mag, 1.0, atol=1e-12)


def _corner_growth(scheme, d, dt, ndim, order=2):
    """Largest |eigenvalue| over the highest lattice modes (the Nyquist corner region)."""
    if ndim == 2:
        shape, modes = (8, 8), [(4, 0, 4), (4, 0, 3), (3, 0, 4), (4, 0, 0), (0, 0, 4)]
    else:
        shape, modes = (4, 4, 4), [(2, 2, 2), (2, 2, 1), (2, 1, 2), (1, 2, 2)]
    g = 0.0
    for m in modes:
        if scheme == "pstd":
            step = lambda E, B: C.pstd_step(E, B, d=d, dt=dt, order=order if order != 2 else 0)
            M = C.amplification_matrix(step, shape, m, d, False)
        else:
            M = C.amplification_matrix(_fdtd(scheme, d, dt, order), shape, m, d, True)
        g = max(g, np.max(np.abs(np.linalg.eigvals(M))))
    return g


@pytest.mark.parametrize("scheme,order,printed", [
    ("yee", 2, 1 / np.sqrt(2)),                                            # Yee
    ("ckc", 2, 1.0),                                                       # CKC
    ("yee", 4, 1 / (np.sqrt(2) * sum(abs(float(c)) for c in D.fornberg_staggered(4)))),
])
def test_courant_limits_match_table1_and_bound_stability(scheme, order, printed):
    d = (1.0, 1.0, 1.0)
    lim = C.courant_limit(scheme, d, 2, order=order)
    assert lim == pytest.approx(printed, rel=1e-14)
    assert _corner_growth(scheme, d, 0.999 * lim, 2, order) < 1 + 1e-12
    assert _corner_growth(scheme, d, 1.01 * lim, 2, order) > 1 + 1e-3


def test_pstd_courant_limit():
    # Table 1 prints sqrt(2)/pi for dx = dz; the Nyquist -> 0 convention keeps
    # the corner mode static, so the limit is reached at the highest kept modes
    d = (1.0, 1.0, 1.0)
    lim = C.courant_limit("pstd", d, 2)
    assert lim == pytest.approx(np.sqrt(2) / np.pi, rel=1e-14)
    # at 16 points the largest kept |k| is 2 pi 7/16 per axis
    kmax = np.sqrt(2) * 2 * np.pi * 7 / 16
    shape = (16, 16)
    M = C.amplification_matrix(lambda E, B: C.pstd_step(E, B, d=d, dt=2 / kmax * 0.999),
                               shape, (7, 0, 7), d, False)
    assert np.max(np.abs(np.linalg.eigvals(M))) < 1 + 1e-12
    M = C.amplification_matrix(lambda E, B: C.pstd_step(E, B, d=d, dt=2 / kmax * 1.01),
                               shape, (7, 0, 7), d, False)
    assert np.max(np.abs(np.linalg.eigvals(M))) > 1 + 1e-3


@pytest.mark.parametrize("axis", ["x", "z"])
def test_ckc_is_exact_along_the_axes_at_courant_one(axis):
    # Sec. III.A: CKC with c dt = dx = dz is dispersion-free along x and z, so
    # a wave along an axis moves by exactly one cell per step, whatever its shape
    rng = np.random.default_rng(11)
    n = 48
    d = (0.5, 1.0, 0.5)
    dt = d[0]
    f = np.convolve(rng.normal(size=n), np.ones(5) / 5, mode="same")
    zero = np.zeros((n, n))
    if axis == "x":
        # wave along +x: Ez = f(x - c t), By = -Ez / c; Ez at (i, k+1/2),
        # By at (i+1/2, k+1/2) and t = -dt/2: By[i] = -f(x_{i+1/2} + c dt/2) = -f(x_{i+1})
        Ez = np.tile(f[None, :], (n, 1))
        By = -np.tile(np.roll(f, -1)[None, :], (n, 1))
        E, B = [zero, zero, Ez], [zero, By, zero]
    else:
        # wave along +z: Ex = f(z - c t), By = Ex / c; Ex at (i+1/2, k),
        # By at (i+1/2, k+1/2): By[k] = f(z_{k+1})
        Ex = np.tile(f[:, None], (1, n))
        By = np.tile(np.roll(f, -1)[:, None], (1, n))
        E, B = [Ex, zero, zero], [zero, By, zero]
    for step in range(1, 31):
        E, B = C.fdtd_step(E, B, d=d, dt=dt, scheme="ckc")
    if axis == "x":
        assert np.max(np.abs(E[2] - np.tile(np.roll(f, 30)[None, :], (n, 1)))) < 1e-13
    else:
        assert np.max(np.abs(E[0] - np.tile(np.roll(f, 30)[:, None], (1, n)))) < 1e-13


def _div_plus(B, d):
    """Divergence of the Yee-grid B at the cell centres (forward differences)."""
    out = (np.roll(B[0], -1, axis=2) - B[0]) / d[0]
    out += (np.roll(B[1], -1, axis=1) - B[1]) / d[1]
    out += (np.roll(B[2], -1, axis=0) - B[2]) / d[2]
    return out


def _div_minus(E, d):
    out = (E[0] - np.roll(E[0], 1, axis=2)) / d[0]
    out += (E[1] - np.roll(E[1], 1, axis=1)) / d[1]
    out += (E[2] - np.roll(E[2], 1, axis=0)) / d[2]
    return out


def test_yee_keeps_div_b_and_gauss_under_continuity():
    rng = np.random.default_rng(5)
    shape = (10, 8, 12)
    d = (1.0, 0.8, 1.2)
    dt = 0.8 * C.courant_limit("yee", d, 3)
    E = [rng.normal(size=shape) for _ in range(3)]
    B = [rng.normal(size=shape) for _ in range(3)]
    rho = _div_minus(E, d) + 0.0  # Gauss residual starts at 0 with eps0 = 1
    divb0 = _div_plus(B, d)
    for _ in range(12):
        J = [rng.normal(size=shape) for _ in range(3)]
        rho = rho - dt * _div_minus(J, d)  # discrete continuity
        E, B = C.fdtd_step(E, B, J, d=d, dt=dt)
    assert np.max(np.abs(_div_plus(B, d) - divb0)) < 1e-12
    assert np.max(np.abs(_div_minus(E, d) - rho)) < 1e-12


def test_yee_s_pol_matches_the_separate_s_pol_stepper():
    rng = np.random.default_rng(9)
    shape = (12, 20)
    d = (0.5, 1.0, 0.4)
    dt = 0.7 * C.courant_limit("yee", d, 2)
    E = [rng.normal(size=shape) for _ in range(3)]
    B = [rng.normal(size=shape) for _ in range(3)]
    Ey, Bx, Bz = E[1], B[0], B[2]
    for _ in range(5):
        E, B = C.fdtd_step(E, B, d=d, dt=dt)
        Ey, Bx, Bz = D.yee_step_s_pol(Ey, Bx, Bz, d[0], d[2], dt)
    assert np.max(np.abs(E[1] - Ey)) < 1e-12
    assert np.max(np.abs(B[0] - Bx)) < 1e-12
    assert np.max(np.abs(B[2] - Bz)) < 1e-12


@pytest.mark.parametrize("stepper", ["yee", "ckc", "pstd"])
def test_uniform_current_drives_only_e(stepper):
    # the k = 0 mode: E -= dt J / eps0, B unchanged
    shape = (8, 12)
    d, dt, eps0 = (1.0, 1.0, 1.0), 0.3, 2.0
    E = [np.full(shape, v) for v in (1.0, -2.0, 0.5)]
    B = [np.full(shape, v) for v in (0.25, 3.0, -1.0)]
    J = [np.full(shape, v) for v in (0.7, 0.1, -0.4)]
    if stepper == "pstd":
        En, Bn = C.pstd_step(E, B, J, d=d, dt=dt, eps0=eps0)
    else:
        En, Bn = C.fdtd_step(E, B, J, d=d, dt=dt, eps0=eps0, scheme=stepper)
    for i in range(3):
        assert np.allclose(En[i], E[i] - dt * J[i] / eps0, atol=1e-14)
        assert np.allclose(Bn[i], B[i], atol=1e-14)


def test_pstd_converges_to_psatd_at_second_order():
    # PSTD tends to PSATD as dt -> 0 (Sec. IV.C); leapfrog is second order
    # (smooth fields; B = 0 so that div B = 0, and the J form of PSATD, which
    # keeps a longitudinal E static as PSTD does)
    rng = np.random.default_rng(21)
    shape = (16, 16)
    d = (1.0, 1.0, 1.0)
    m = np.fft.fftfreq(16, 1 / 16)
    low = (np.abs(m)[:, None] <= 3) & (np.abs(m)[None, :] <= 3)
    E0 = [np.real(np.fft.ifft2(np.fft.fft2(rng.normal(size=shape)) * low)) for _ in range(3)]
    B0 = [np.zeros(shape) for _ in range(3)]
    T = 1.2
    ref_E, _ = oracle.psatd_run(E0, B0, 1, d=d, dt=T, form="J")
    errs = []
    for nsteps in (8, 16, 32):
        dt = T / nsteps
        # B at -dt/2 from the exact (PSATD) evolution
        _, Bh = oracle.psatd_step(E0, B0, d=d, dt=-0.5 * dt, form="J")
        E, B = E0, Bh
        for _ in range(nsteps):
            E, B = C.pstd_step(E, B, d=d, dt=dt)
        errs.append(np.sqrt(sum(np.sum((a - b) ** 2) for a, b in zip(E, ref_E))))
    assert errs[0] / errs[1] == pytest.approx(4.0, rel=0.05)
    assert errs[1] / errs[2] == pytest.approx(4.0, rel=0.05)
