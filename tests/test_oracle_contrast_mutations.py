"""Planted mistakes in the contrast steppers must be caught by their pins (CPU).

Each case patches one plausible error into ``oracle.contrast`` (a difference
taken the wrong way, a transverse average along the wrong axis or with the
wrong weights, a sign, a non-leapfrog update) and checks that the pins of
tests/test_oracle_contrast.py (Table 1 eigenvalues, CKC exactness along the
axes, div B) see it.
"""

import numpy as np
import pytest

import oracle
from oracle import contrast as C
from oracle import dispersion as D


def fdtd_eig_error(scheme, order=2):
    d = (1.0, 1.0, 1.0)
    shape = (16, 24)
    dt = 0.6 * C.courant_limit(scheme, d, 2, order=order)
    beta = D.BETA_CKC if scheme == "ckc" else 0.0
    worst = 0.0
    for m in [(3, 0, 2), (7, 0, -5), (11, 0, 1)]:
        M = C.amplification_matrix(
            lambda E, B: C.fdtd_step(E, B, d=d, dt=dt, scheme=scheme, order=order),
            shape, m, d, True)
        ev = np.linalg.eigvals(M)
        ph = np.sort(np.abs(np.angle(ev)))
        kx, kz = 2 * np.pi * m[0] / 24, 2 * np.pi * m[2] / 16
        if order == 2:
            w = D.omega_fdtd(kx, kz, d[0], d[2], dt, beta=beta)
        else:
            kp = np.hypot(D.modified_k(kx, 1.0, order), D.modified_k(kz, 1.0, order))
            w = 2 / dt * np.arcsin(0.5 * dt * kp)
        worst = max(worst, np.max(np.abs(ph[2:] - w * dt)), np.max(np.abs(np.abs(ev) - 1)))
    return worst


def pstd_eig_error():
    d = (1.0, 1.0, 1.0)
    shape = (16, 24)
    dt = 0.6 * C.courant_limit("pstd", d, 2)
    worst = 0.0
    for m in [(3, 0, 2), (7, 0, -5)]:
        M = C.amplification_matrix(lambda E, B: C.pstd_step(E, B, d=d, dt=dt), shape, m, d, False)
        ev = np.linalg.eigvals(M)
        ph = np.sort(np.abs(np.angle(ev)))
        K = np.hypot(oracle.ktable(24, 1.0)[m[0] % 24], oracle.ktable(16, 1.0)[m[2] % 16])
        w = K / D.index_pstd(K, dt)
        worst = max(worst, np.max(np.abs(ph[2:] - w * dt)), np.max(np.abs(np.abs(ev) - 1)))
    return worst


def ckc_axis_error():
    n = 32
    rng = np.random.default_rng(1)
    f = rng.normal(size=n)
    zero = np.zeros((n, n))
    Ez = np.tile(f[None, :], (n, 1))
    By = -np.tile(np.roll(f, -1)[None, :], (n, 1))
    E, B = [zero, zero, Ez], [zero, By, zero]
    for _ in range(10):
        E, B = C.fdtd_step(E, B, d=(1.0, 1.0, 1.0), dt=1.0, scheme="ckc")
    return np.max(np.abs(E[2] - np.tile(np.roll(f, 10)[None, :], (n, 1))))


def all_pins_pass():
    return (fdtd_eig_error("yee") < 1e-12 and fdtd_eig_error("ckc") < 1e-12
            and fdtd_eig_error("yee", 4) < 1e-12 and pstd_eig_error() < 1e-12
            and ckc_axis_error() < 1e-12)


def test_unmutated_contrast_oracle_passes_all_pins():
    assert all_pins_pass()


def _dplus_off_by_one(f, a, d, weights):
    ax = C._axis(f.shape, a)
    if ax is None:
        return np.zeros_like(f)
    out = np.zeros_like(f)
    for l, cl in enumerate(weights, start=1):
        out = out + cl * (np.roll(f, -l, axis=ax) - np.roll(f, l, axis=ax))
    return out / d[a]


def _smooth_same_axis(g, a, beta):
    other = 2 if a == 0 else 0
    return _ORIG["_smooth"](g, other, beta)


def _smooth_full_beta(g, a, beta):
    ax = C._axis(g.shape, a)
    return (1.0 - beta) * g + beta * (np.roll(g, -1, axis=ax) + np.roll(g, 1, axis=ax))


def _fdtd_faraday_sign(E, B, J=None, **kw):
    En, Bn = _ORIG["fdtd_step"](E, B, J, **kw)
    # flip the sign of the update of By only
    Bn[1] = 2 * B[1] - Bn[1]
    return En, Bn


def _pstd_no_leapfrog(E, B, J=None, *, d, dt, c=1.0, eps0=1.0, order=0, stencil="staggered",
                      workers=None):
    # Ampere with B^{n-1/2} instead of B^{n+1/2} (complex inputs only: the pins)
    import scipy.fft as sfft
    kx, ky, kz = oracle.psatd._kvectors(E[0].shape, d, "c2c", order, stencil)
    Ek = [sfft.fftn(f) for f in E]
    Bk = [sfft.fftn(f) for f in B]
    kxE = (ky * Ek[2] - kz * Ek[1], kz * Ek[0] - kx * Ek[2], kx * Ek[1] - ky * Ek[0])
    kxB = (ky * Bk[2] - kz * Bk[1], kz * Bk[0] - kx * Bk[2], kx * Bk[1] - ky * Bk[0])
    Bn = [Bk[i] - 1j * dt * kxE[i] for i in range(3)]
    En = [Ek[i] + 1j * c * c * dt * kxB[i] for i in range(3)]
    return [sfft.ifftn(f) for f in En], [sfft.ifftn(f) for f in Bn]


_ORIG = {"_dplus": C._dplus, "_dminus": C._dminus, "_smooth": C._smooth,
         "fdtd_step": C.fdtd_step, "pstd_step": C.pstd_step}

MUTANTS = {
    "curl of B with forward differences": ("_dminus", lambda f, a, d, w: _ORIG["_dplus"](f, a, d, w)),
    "D+ reads i-l instead of i-l+1": ("_dplus", _dplus_off_by_one),
    "CKC average along the difference axis": ("_smooth", _smooth_same_axis),
    "CKC neighbour weights beta instead of beta/2": ("_smooth", _smooth_full_beta),
    "Faraday sign of By": ("fdtd_step", _fdtd_faraday_sign),
    "PSTD Ampere with the old B": ("pstd_step", _pstd_no_leapfrog),
}


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_planted_mistake_is_caught(name, monkeypatch):
    attr, fn = MUTANTS[name]
    monkeypatch.setattr(C, attr, fn)
    assert not all_pins_pass(), f"pins missed: {name}"
