"""The large 3D workload's inputs built directly in device memory.

The 1024 x 1024 x 512 workload's fields are lattice plane waves and its
currents are separable (Q_c(z, y) G(x)), so both can be formed on the GPU
from their parameters -- the same seeded draws as :func:`fixtures.workload`
-- by outer products of one-dimensional factors, without building the
arrays on the host.  Only synthesis happens here: sums of cosines and
products of factors (no transform, no part of the field step).
"""

from __future__ import annotations

import numpy as np

from .fields import LAMBDA0, current_factors, plane_wave_list, source_time_factors
from .workloads import CONFIG_NAMES, Patch


def _axis_phase(torch, m, n, device):
    """exp(2 pi i m j / n), j = 0..n-1, with the phase reduced exactly (m j mod n)."""
    j = torch.arange(n, device=device, dtype=torch.int64)
    ph = ((m * j) % n).to(torch.float64) * (2.0 * np.pi / n)
    return torch.polar(torch.ones_like(ph), ph)


def workload4_device(torch, shape=None, device="cuda:0", dtype=None):
    """Workload 4 (3D, plane-wave packets n = 1..100 at angles within 40
    degrees, current sheet with continuity-consistent rho) at ``shape``
    (default 512 x 1024 x 1024, [z][y][x]), built on ``device``.

    Returns (patch, E, B, J, rho_old, rho_new): flat tensors of ``dtype``
    (default float32) holding the fields at t = 0 and the sources of step 0
    (J^(1/2), rho^0 = 0, rho^1 = -dt div J^(1/2)).
    """
    dtype = dtype or torch.float32
    nz, ny, nx = shape or (512, 1024, 1024)
    rng = np.random.default_rng(1004)
    dx = LAMBDA0 / 256
    p = Patch(3, nx, ny, nz, dx, dx, dx, dx)
    waves = plane_wave_list((nz, ny, nx), p.d, nharm=100, max_angle_deg=40.0, rng=rng)
    Qs, G, Gx, Qy, Qz = current_factors((nz, ny, nx), p.d, width=2.0 * LAMBDA0 / 8, nmodes=16,
                                        min_wavelength=LAMBDA0 / 4, rng=rng)
    phases = rng.uniform(0.0, 2.0 * np.pi, size=(3, 40))
    E = [torch.zeros((nz, ny, nx), dtype=torch.float64, device=device) for _ in range(3)]
    B = [torch.zeros((nz, ny, nx), dtype=torch.float64, device=device) for _ in range(3)]
    for m, e, b, phase in waves:
        fz = _axis_phase(torch, m[2], nz, device)
        fy = _axis_phase(torch, m[1], ny, device)
        fx = _axis_phase(torch, m[0], nx, device) * complex(np.exp(1j * phase))
        w = torch.real(fz[:, None, None] * fy[None, :, None] * fx[None, None, :])
        for i in range(3):
            if e[i] != 0.0:
                E[i].add_(w, alpha=float(e[i]))
            if b[i] != 0.0:
                B[i].add_(w, alpha=float(b[i]))
        del w
    f = source_time_factors(0.5 * p.dt, phases)
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(device)  # noqa: E731
    g, gx = t(G), t(Gx)
    J = [(t(Qs[c])[:, :, None] * g[None, None, :]) * float(f[c]) for c in range(3)]
    divJ = (t(Qs[0])[:, :, None] * gx[None, None, :]) * float(f[0])
    divJ += (t(Qy)[:, :, None] * g[None, None, :]) * float(f[1])
    divJ += (t(Qz)[:, :, None] * g[None, None, :]) * float(f[2])
    rho_old = torch.zeros((nz * ny * nx,), dtype=dtype, device=device)
    rho_new = (divJ * (-p.dt)).to(dtype).reshape(-1)
    del divJ

    def flat(a):
        return a.to(dtype).reshape(-1)

    return (p, [flat(a) for a in E], [flat(a) for a in B], [flat(a) for a in J], rho_old, rho_new)


NAME = CONFIG_NAMES[4]


class DeviceSourceSchedule:
    """The per-step sources of a :class:`fixtures.SourceSchedule`, generated on
    the GPU.

    The profiles P_c and their divergence factors D_c (FP64) are copied to the
    device once; each step then forms
        J_c = f_c(t^{n+1/2}) P_c,   rho^{n+1} = -dt sum_c F_c(n+1) D_c
    with the host schedule's scalar coefficients, in the same FP64 operation
    order as the host schedule, then rounds to the storage type.  rho^n of
    step n is rho^{n+1} of step n - 1, kept from the previous call.
    """

    def __init__(self, schedule, torch, device="cuda:0", dtype=None):
        self.torch = torch
        self.s = schedule
        self.dtype = dtype or torch.float32
        dev = lambda a: torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64).ravel()).to(device)  # noqa: E731
        self.P = [dev(a) for a in schedule.P]
        self.D = [dev(a) for a in schedule.D]
        self.cells = self.P[0].numel()
        self._tmp = torch.empty(self.cells, dtype=torch.float64, device=device)
        self._acc = torch.empty(self.cells, dtype=torch.float64, device=device)

    def _rho_into(self, F, out):
        acc = self._acc
        torch = self.torch
        torch.mul(self.D[0], float(F[0]), out=acc)
        for c in (1, 2):
            torch.mul(self.D[c], float(F[c]), out=self._tmp)
            acc.add_(self._tmp)
        acc.mul_(-self.s.dt)
        out[: self.cells].copy_(acc)

    def sources_into(self, n, J, rho_old=None, rho_new=None):
        """Write step n's J^{n+1/2} (3 flat tensors) and, if given, rho^n and
        rho^{n+1} into the first ``cells`` elements of the given tensors."""
        f, F0, F1 = self.s.coefficients(n)
        for c in range(3):
            self.torch.mul(self.P[c], float(f[c]), out=self._tmp)
            J[c][: self.cells].copy_(self._tmp)
        if rho_old is not None:
            self._rho_into(F0, rho_old)
        if rho_new is not None:
            self._rho_into(F1, rho_new)

    def advance_into(self, n, J, rho_old, rho_new):
        """Step n's sources when the caller keeps rho_new of step n - 1 in
        rho_old (the buffers swap roles each step): only J and rho^{n+1} are
        formed.  Step 0 forms rho^0 too."""
        f, F0, F1 = self.s.coefficients(n)
        for c in range(3):
            self.torch.mul(self.P[c], float(f[c]), out=self._tmp)
            J[c][: self.cells].copy_(self._tmp)
        if n == 0:
            self._rho_into(F0, rho_old)
        self._rho_into(F1, rho_new)
