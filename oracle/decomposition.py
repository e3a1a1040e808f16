"""Guard-cell domain decomposition of the PSATD step, FP64 -- TEST INFRASTRUCTURE.

What the paper describes (Sec. II.A, the pseudo-spectral solvers of PXR): the
domain is split into subdomains as for FDTD solvers.  Each subdomain is
extended by guard regions that hold copies of the adjacent subdomains, and
Maxwell's equations are solved on it with local FFTs instead of global ones.
The result carries a small truncation error (fields near a subdomain edge feel
the periodic wrap of the local grid instead of the true neighbours).  That
error depends on the stencil order p, the guard width and the resolution, and
is smallest for high p with a moderate number of guards.

One step here, for each subdomain s (a box of n_a / parts_a cells per axis):
  1. local grid = the box extended by `guard` cells on both sides of every
     split axis, filled from the global fields at the periodic global
     positions (this is the guard exchange: the copies come from the
     neighbours' current interiors);
  2. one PSATD step (``psatd_step``, order p) on the local grid as a periodic
     patch;
  3. the box's interior cells of the result are the new global fields there.
Sources (J, rho) are scattered the same way.  Axes with parts_a = 1 are not
split and get no guards (2D: axis y is never split).
"""

from __future__ import annotations

import numpy as np

from .psatd import psatd_step


def _axes(shape):
    # array axes of (x, y, z) for [z][x] or [z][y][x] arrays
    return {0: 1, 2: 0} if len(shape) == 2 else {0: 2, 1: 1, 2: 0}


def local_index(shape, parts, guard, s):
    """Global index arrays (per array axis) of the local grid of subdomain ``s``
    (a tuple of subdomain coordinates along x, y, z)."""
    ax = _axes(shape)
    idx = [None] * len(shape)
    for a, arr_axis in ax.items():
        n = shape[arr_axis]
        p = parts[a]
        g = guard[a] if p > 1 else 0
        ns = n // p
        idx[arr_axis] = (s[a] * ns - g + np.arange(ns + 2 * g)) % n
    return idx


def decomposed_step(E, B, J=None, rho_old=None, rho_new=None, *, parts, guard, d, dt,
                    c=1.0, eps0=1.0, order=0, stencil="staggered", form="rho"):
    """One step of the guard-cell decomposition; returns global (E', B')."""
    shape = E[0].shape
    ax = _axes(shape)
    for a, arr_axis in ax.items():
        if shape[arr_axis] % parts[a] != 0:
            raise ValueError("every axis must split evenly")
    En = [np.empty(shape) for _ in range(3)]
    Bn = [np.empty(shape) for _ in range(3)]
    ranges = [range(parts[0]), range(parts[1] if len(shape) == 3 else 1), range(parts[2])]
    for sx in ranges[0]:
        for sy in ranges[1]:
            for sz in ranges[2]:
                s = (sx, sy, sz)
                idx = local_index(shape, parts, guard, s)
                grid = np.ix_(*idx)

                def loc(f):
                    return None if f is None else np.asarray(f, np.float64)[grid]

                El, Bl = psatd_step([loc(f) for f in E], [loc(f) for f in B],
                                    None if J is None else [loc(f) for f in J],
                                    loc(rho_old), loc(rho_new), d=d, dt=dt, c=c, eps0=eps0,
                                    order=order, stencil=stencil, form=form)
                # interior of the local grid -> its global box
                inner_local, inner_global = [], []
                for a, arr_axis in sorted(ax.items(), key=lambda t: t[1]):
                    n = shape[arr_axis]
                    p = parts[a]
                    g = guard[a] if p > 1 else 0
                    ns = n // p
                    inner_local.append(slice(g, g + ns))
                    inner_global.append(slice(s[a] * ns, s[a] * ns + ns))
                for dst, src in zip(En + Bn, El + Bl):
                    dst[tuple(inner_global)] = src[tuple(inner_local)]
    return En, Bn
