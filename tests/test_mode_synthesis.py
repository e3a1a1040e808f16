"""CPU check of the lattice-mode bookkeeping used by the full-size 3D GPU
tests: synthesizing the modes on a whole small grid and running the oracle's
full step (FFTs included) gives the same fields as the per-mode exact update
synthesized point by point.  Even axes, so the Nyquist modes are covered."""

import numpy as np
import pytest

import oracle
import test_gpu_fullsize_modes as fm


@pytest.mark.parametrize("sources", [False, True])
def test_mode_synthesis_matches_full_oracle_step(sources):
    shape = (16, 12, 18)
    d, dt, K = (0.1, 0.13, 0.07), 0.05, 3
    modes = fm._setup(shape, d, dt, sources, np.random.default_rng(1))
    nz, ny, nx = shape
    iz, iy, ix = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")

    def full(amp):
        acc = np.zeros(shape)
        for md in modes:
            m = md["m"]
            th = 2 * np.pi * (((m[0] * ix) % nx) / nx + ((m[1] * iy) % ny) / ny
                              + ((m[2] * iz) % nz) / nz)
            acc += 2 * np.real(amp(md) * np.exp(1j * th))
        return acc

    E = [full(lambda md, i=i: md["E"][i]) for i in range(3)]
    B = [full(lambda md, i=i: md["B"][i]) for i in range(3)]
    J = [full(lambda md, i=i: md["J"][i]) for i in range(3)]
    dr = full(lambda md: md["drho"])
    for n in range(K):
        if sources:
            E, B = oracle.psatd_step(E, B, J, n * dr, (n + 1) * dr, d=d, dt=dt)
        else:
            E, B = oracle.psatd_step(E, B, d=d, dt=dt)
    ex = fm._exact(modes, K, dt, sources)
    idx = np.arange(int(np.prod(shape)))
    ref = ([fm._synth(modes, [e for e, _ in ex], c, idx, shape) for c in range(3)]
           + [fm._synth(modes, [b for _, b in ex], c, idx, shape) for c in range(3)])
    got = [a.ravel() for a in E + B]
    num = sum(np.sum((g - r) ** 2) for g, r in zip(got, ref))
    den = sum(np.sum(r * r) for r in ref)
    assert np.sqrt(num / den) < 1e-13
