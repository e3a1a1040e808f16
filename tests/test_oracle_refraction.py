"""Pins of the refraction model (Sec. IV, eq. 1; oracle/refraction.py).

- The Newton-Raphson solution satisfies eq. 1 to 1e-12 for every solver.
- The signs Sec. IV.B and Fig. 4 describe: with n_r > 1 (Yee, CKC) the
  harmonics bend toward the normal, more so at higher frequency; with n_r < 1
  (PSTD) away from it, more so at higher frequency; PSATD (n = 1) does not
  bend at all.
- The printed total-reflection example (Sec. IV.B.2): PSTD at its Courant
  limit, k dx = pi/2, n_r = 0.978 and theta_l = arcsin(0.978) = 77.96 deg; the
  model has a refracted wave just below theta_l and none just above.
- The cut-off of Fig. 5 / Sec. IV.B.2 at 80 degrees: PSTD loses its refracted
  harmonics in the mid-teens (the paper: around order 17), PSATD never does.
- The root solve agrees with the closed-form index formulas of Table 1 and
  with a brute-force scan for the sign change of eq. 1.
"""

import json
import os

import numpy as np
import pytest

from oracle import dispersion as D
from oracle import refraction as R

GOLDEN = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_values.json")))
DX = 1.0 / 70.0  # lambda0 / 70, the resolution of Fig. 4
W0 = 2.0 * np.pi  # omega0 in normalized units (lambda0 = c = 1)
TH_I = np.deg2rad(55.0)  # incidence of Fig. 4
SOLVERS = {"yee": 0.999 / np.sqrt(2.0), "ckc": 0.999, "pstd": np.sqrt(2.0) / np.pi, "psatd": 1.0}


def _theta(solver, n, th_i=TH_I, **kw):
    return R.refraction_angle(solver, n * W0, th_i, DX, DX, SOLVERS[solver] * DX, **kw)


@pytest.mark.parametrize("solver", sorted(SOLVERS))
def test_solution_satisfies_snell_descartes(solver):
    for n in (10, 15, 20, 25, 30):
        th = _theta(solver, n)
        nr = R.index_at(solver, n * W0, th, DX, DX, SOLVERS[solver] * DX)
        assert abs(nr * np.sin(th) - np.sin(TH_I)) <= 1e-12


def test_refraction_signs_follow_the_index():
    ns = (10, 15, 20, 25, 30)
    for solver in ("yee", "ckc"):  # n_r > 1, rising with frequency: toward the normal
        th = [_theta(solver, n) for n in ns]
        assert all(t < TH_I for t in th)
        assert all(a > b for a, b in zip(th, th[1:]))
    th = [_theta("pstd", n) for n in ns]  # n_r < 1, falling: away from the normal
    assert all(t > TH_I for t in th)
    assert all(a < b for a, b in zip(th, th[1:]))
    for n in ns:  # dispersion-free
        assert abs(_theta("psatd", n) - TH_I) <= 1e-12


def test_psatd_order_p_bends_slightly_toward_the_normal():
    # k_p < k for a finite staggered stencil, so n = |k|/|k_p| >= 1 (Table 1):
    # a small bend toward the normal that grows with frequency and shrinks with p
    d16 = [TH_I - _theta("psatd", n, order=16) for n in (10, 20, 30)]
    d128 = [TH_I - _theta("psatd", n, order=128) for n in (10, 20, 30)]
    assert all(x >= 0.0 for x in d16 + d128)
    assert d16[0] < d16[1] < d16[2]
    assert all(b <= a for a, b in zip(d16, d128))
    assert d128[1] < 1e-6


def test_printed_total_reflection_limit():
    dt = np.sqrt(2.0) / np.pi * DX
    w = float(R.omega_num("pstd", np.pi / 2 / DX, 0.0, DX, DX, dt))
    nr = R.index_at("pstd", w, 0.4, DX, DX, dt)  # isotropic: any direction
    assert round(nr, GOLDEN["pstd_index_at_kdx_pi_over_2"]["decimals"]) == \
        GOLDEN["pstd_index_at_kdx_pi_over_2"]["value"]
    assert round(float(D.limit_angle_deg(GOLDEN["pstd_index_at_kdx_pi_over_2"]["value"])), 2) == \
        GOLDEN["pstd_limit_angle_deg"]["value"]
    th_l = np.arcsin(nr)
    below = R.refraction_angle("pstd", w, th_l - np.deg2rad(0.02), DX, DX, dt)
    above = R.refraction_angle("pstd", w, th_l + np.deg2rad(0.02), DX, DX, dt)
    assert np.isfinite(below) and below > np.deg2rad(85.0)
    assert np.isnan(above)


def test_cutoff_at_grazing_incidence():
    th80 = np.deg2rad(80.0)
    cut = next(n for n in range(5, 40) if np.isnan(_theta("pstd", n, th80)))
    assert 13 <= cut <= 19  # the paper: a cut-off around order 17
    # PSATD keeps every harmonic up to the grid's limit (order 35 at lambda/70)
    assert all(np.isfinite(_theta("psatd", n, th80)) for n in range(5, 36))
    # at 0.9 of the PSTD Courant limit the cut-off falls on order 17 exactly
    dt = 0.9 * np.sqrt(2.0) / np.pi * DX
    cut09 = next(n for n in range(5, 40)
                 if np.isnan(R.refraction_angle("pstd", n * W0, th80, DX, DX, dt)))
    assert cut09 == 17


@pytest.mark.parametrize("solver,formula", [("yee", D.index_yee), ("ckc", D.index_ckc)])
def test_index_root_matches_table1_formula(solver, formula):
    dt = SOLVERS[solver] * DX
    for n in (12, 20):  # below the Yee cut-off along the axes at this resolution
        for th in np.deg2rad([0.0, 20.0, 45.0, 70.0]):
            nr = R.index_at(solver, n * W0, th, DX, DX, dt)
            k = nr * n * W0  # c = 1
            assert abs(float(formula(k * np.cos(th), k * np.sin(th), DX, DX, dt)) - nr) < 1e-12


def test_newton_matches_a_brute_force_scan():
    for solver in ("yee", "ckc", "pstd"):
        dt = SOLVERS[solver] * DX
        w = 22 * W0
        grid = np.linspace(np.deg2rad(30.0), np.deg2rad(80.0), 5001)
        g = np.array([R.index_at(solver, w, t, DX, DX, dt) * np.sin(t) for t in grid]) - np.sin(TH_I)
        i = int(np.nonzero(np.diff(np.sign(g)))[0][0])
        t0 = grid[i] - g[i] * (grid[i + 1] - grid[i]) / (g[i + 1] - g[i])
        assert abs(R.refraction_angle(solver, w, TH_I, DX, DX, dt) - t0) < 1e-7


def test_index_map_of_figure_2():
    kdx = np.linspace(0.05, np.pi / 2, 40)
    th = np.deg2rad(np.linspace(0.0, 90.0, 19))
    yee = R.index_map("yee", 1 / np.sqrt(2), kdx, th)
    ckc = R.index_map("ckc", 1.0, kdx, th)
    pstd = R.index_map("pstd", np.sqrt(2) / np.pi, kdx, th)
    psatd = R.index_map("psatd", 1.0, kdx, th)
    assert np.all(yee >= 1.0 - 1e-15) and np.all(ckc >= 1.0 - 1e-15)
    assert np.all(pstd <= 1.0 + 1e-15)
    assert np.max(np.abs(psatd - 1.0)) < 1e-15
    # Yee at its Courant limit is dispersion-free along the diagonal (Appendix A)
    assert np.max(np.abs(yee[9] - 1.0)) < 1e-12
    # CKC at c dt = dx is dispersion-free along the axes (Sec. III.A)
    assert np.max(np.abs(ckc[[0, -1]] - 1.0)) < 1e-12
    # the map agrees with the closed-form rows of Table 1
    K = kdx[None, :] * np.ones((len(th), 1))
    assert np.allclose(yee, D.index_yee(K * np.cos(th)[:, None], K * np.sin(th)[:, None], 1.0, 1.0,
                                        1 / np.sqrt(2)), rtol=0, atol=1e-13)
    assert np.allclose(pstd, D.index_pstd(K, np.sqrt(2) / np.pi), rtol=0, atol=1e-13)


def test_planted_mistake_inverted_index_is_caught(monkeypatch):
    # eq. 1 written with 1/n_r: the FDTD harmonics would bend away from the normal
    orig = R.index_at
    monkeypatch.setattr(R, "index_at", lambda *a, **k: 1.0 / orig(*a, **k))
    th = _theta("yee", 20)
    assert not th < TH_I
