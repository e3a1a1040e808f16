"""Plain FP64 CPU oracle for the PSATD field step -- TEST INFRASTRUCTURE.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.  The product path (the HIP library in
``paper_1608_05739_amd`` and its Python binding) never imports, links or
calls anything here, and this package imports nothing from it: the two share
no code.  Inputs come from the seeded generators in ``fixtures``.

Contents
  psatd       k tables, PSATD coefficients, the per-mode update (rho-form and
              J-form) and the full step (r2c or c2c transforms), written from
              Sec. III.B item 2 and Table 1 (PSATD row).
  dispersion  refractive-index formulas of Table 1, the order-p stencils,
              Appendix A and a CPU Yee FDTD stepper, used only as the
              contrast the paper draws against PSATD.
  refraction  the Snell-Descartes refraction model of Sec. IV (eq. 1): each
              solver's index n_r(omega, theta), the Newton-Raphson solve for
              theta_r(omega), and the index maps of Fig. 2.
  contrast    the contrast solvers as full field steps (Sec. III.A, Table 1):
              Yee and order-p FDTD on the staggered grid, CKC, and PSTD.
  decomposition  the guard-cell domain decomposition (Sec. II.A).

Pins (see tests/test_oracle_*.py): brute-force O(N^2) DFT sums, the matrix
exponential of the per-mode Maxwell system, exact lattice plane-wave phase,
energy and constraint invariants, rho-form == J-form, r2c == c2c, semigroup
(k steps of dt == one step of k*dt), and the numbers the paper prints in
Sec. IV.B and Appendix A.
"""

from .psatd import (  # noqa: F401
    ktable,
    rktable,
    psatd_coefficients,
    g_series,
    update_modes,
    psatd_step,
    psatd_run,
    field_energy,
    forward,
    inverse,
)
