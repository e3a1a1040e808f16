"""The five benchmark workloads, at full or reduced size, plus lattice test modes.

Each workload is a list of periodic patches (one for a single grid) with its
initial E, B and, when sources are on, a :class:`SourceSchedule`.  The seed of
workload i is 1000 + i (PCG64); draws happen in a fixed order so that a
reduced-size variant of a workload keeps its spacing, time step and seed.

Inputs stand in for the plasma-mirror runs of the paper (Sec. II.B, Fig. 1):
a p-polarized laser at oblique incidence carrying a comb of harmonics with
amplitude n^(-4/3), and a smooth current sheet oscillating at harmonics of
omega0.  No data from those runs is available; these are synthetic.
"""

from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from .fields import (
    LAMBDA0,
    C_LIGHT,
    SourceSchedule,
    current_profile,
    laser_2d,
    laser_3d,
    plane_wave_packets_3d,
)

CONFIG_NAMES = {
    0: "2d-128x128-vacuum-100steps",
    1: "2d-4096x4096-sources-1000steps",
    2: "3d-512x512x512-sources-200steps",
    3: "2d-256patches-64to512-vacuum-500steps",
    4: "3d-1024x1024x512-sources-100steps",
}

PATCH_SIDES = (64, 96, 128, 192, 256, 384, 512)


@dataclass
class Patch:
    """One periodic grid: real shape [z][x] (ny = 1) or [z][y][x]."""

    ndim: int
    nx: int
    ny: int
    nz: int
    dx: float
    dy: float
    dz: float
    dt: float

    @property
    def shape(self):
        return (self.nz, self.nx) if self.ndim == 2 else (self.nz, self.ny, self.nx)

    @property
    def cells(self):
        return self.nx * self.ny * self.nz

    @property
    def d(self):
        return (self.dx, self.dy, self.dz)


@dataclass
class Workload:
    name: str
    index: int
    patches: list
    steps: int
    sources: bool
    E0: list = field(default_factory=list)   # per patch: [Ex, Ey, Ez]
    B0: list = field(default_factory=list)   # per patch: [Bx, By, Bz]
    schedule: list = field(default_factory=list)  # per patch SourceSchedule or None

    @property
    def cells(self):
        return sum(p.cells for p in self.patches)


def _laser_2d_fields(p: Patch, rng, nharm=20, angle=30.0, waist=4.0, tau=3.0):
    return laser_2d(p.nx, p.nz, p.dx, p.dz, angle_deg=angle, waist=waist * LAMBDA0,
                    tau=tau, nharm=nharm, rng=rng)


def workload(index: int, *, shape=None, steps=None, npatches=None, build_fields=True) -> Workload:
    """Build workload ``index`` (0..4).

    ``shape`` overrides the grid (same dx, dt and seed) for reduced-size
    parity runs; ``npatches`` keeps the first patches of workload 3.
    """
    rng = np.random.default_rng(1000 + index)
    if index == 0:
        nz, nx = shape or (128, 128)
        dx = LAMBDA0 / 32
        p = Patch(2, nx, 1, nz, dx, dx, dx, dx / C_LIGHT)
        w = Workload(CONFIG_NAMES[0], 0, [p], steps or 100, False)
        if build_fields:
            E, B = _laser_2d_fields(p, rng)
            w.E0, w.B0, w.schedule = [E], [B], [None]
        return w
    if index == 1:
        nz, nx = shape or (4096, 4096)
        dx = LAMBDA0 / 32
        p = Patch(2, nx, 1, nz, dx, dx, dx, dx / C_LIGHT)
        w = Workload(CONFIG_NAMES[1], 1, [p], steps or 1000, True)
        if build_fields:
            E, B = _laser_2d_fields(p, rng)
            P, D = current_profile(p.shape, p.d, width=2.0 * LAMBDA0, nmodes=16,
                                   min_wavelength=2.0 * LAMBDA0, rng=rng)
            phases = rng.uniform(0.0, 2.0 * np.pi, size=(3, 30))
            w.E0, w.B0 = [E], [B]
            w.schedule = [SourceSchedule(P, D, phases, p.dt)]
        return w
    if index == 2:
        nz, ny, nx = shape or (512, 512, 512)
        dx = LAMBDA0 / 24
        p = Patch(3, nx, ny, nz, dx, dx, dx, dx / C_LIGHT)
        w = Workload(CONFIG_NAMES[2], 2, [p], steps or 200, True)
        if build_fields:
            E, B = laser_3d(nx, ny, nz, p.d, angle_deg=45.0, waist=3.0 * LAMBDA0,
                            tau=3.0, nharm=40, rng=rng)
            P, D = current_profile(p.shape, p.d, width=2.0 * LAMBDA0, nmodes=16,
                                   min_wavelength=2.0 * LAMBDA0, rng=rng)
            phases = rng.uniform(0.0, 2.0 * np.pi, size=(3, 40))
            w.E0, w.B0 = [E], [B]
            w.schedule = [SourceSchedule(P, D, phases, p.dt)]
        return w
    if index == 3:
        total = 256
        sides = rng.choice(PATCH_SIDES, size=(total, 2))
        dts = rng.uniform(0.5, 2.0, size=total)
        seeds = rng.integers(0, 2 ** 31, size=total)
        count = npatches or total
        dx = LAMBDA0 / 32
        patches = [Patch(2, int(sides[i, 0]), 1, int(sides[i, 1]), dx, dx, dx,
                         float(dts[i]) * dx / C_LIGHT) for i in range(count)]
        w = Workload(CONFIG_NAMES[3], 3, patches, steps or 500, False)
        if build_fields:
            for i, p in enumerate(patches):
                E, B = _laser_2d_fields(p, np.random.default_rng(int(seeds[i])))
                w.E0.append(E)
                w.B0.append(B)
                w.schedule.append(None)
        return w
    if index == 4:
        nz, ny, nx = shape or (512, 1024, 1024)
        dx = LAMBDA0 / 256
        p = Patch(3, nx, ny, nz, dx, dx, dx, dx / C_LIGHT)
        w = Workload(CONFIG_NAMES[4], 4, [p], steps or 100, True)
        if build_fields:
            E, B, _waves = plane_wave_packets_3d(p.shape, p.d, nharm=100, max_angle_deg=40.0,
                                                 rng=rng)
            P, D = current_profile(p.shape, p.d, width=2.0 * LAMBDA0 / 8, nmodes=16,
                                   min_wavelength=LAMBDA0 / 4, rng=rng)
            phases = rng.uniform(0.0, 2.0 * np.pi, size=(3, 40))
            w.E0, w.B0 = [E], [B]
            w.schedule = [SourceSchedule(P, D, phases, p.dt)]
        return w
    raise ValueError(f"no workload {index}")


def lattice_plane_wave(shape, d, m, e, phase=0.0, t=0.0):
    """Exact lattice plane wave E = e cos(k.x - c|k|t + phase), B = k_hat x E / c.

    ``m`` = (m_x, m_y, m_z) integer mode numbers (m_y ignored in 2D), k_i =
    2 pi m_i / (N_i d_i).  ``e`` must be orthogonal to k.  Returns (E, B, k).
    """
    if len(shape) == 2:
        nz, nx = shape
        ny = 1
    else:
        nz, ny, nx = shape
    k = np.array([2 * np.pi * m[0] / (nx * d[0]),
                  2 * np.pi * m[1] / (ny * d[1]) if len(shape) == 3 else 0.0,
                  2 * np.pi * m[2] / (nz * d[2])])
    kn = np.linalg.norm(k)
    x = np.arange(nx) * d[0]
    y = np.arange(ny) * d[1]
    z = np.arange(nz) * d[2]
    if len(shape) == 2:
        arg = k[0] * x[None, :] + k[2] * z[:, None]
    else:
        arg = k[0] * x[None, None, :] + k[1] * y[None, :, None] + k[2] * z[:, None, None]
    cs = np.cos(arg - C_LIGHT * kn * t + phase)
    e = np.asarray(e, dtype=float)
    b = np.cross(k / kn, e) / C_LIGHT
    return [e[i] * cs for i in range(3)], [b[i] * cs for i in range(3)], k
