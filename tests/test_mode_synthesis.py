"""CPU check of the lattice-mode bookkeeping used by the full-size 3D GPU
tests (tests/test_gpu_fullsize_modes.py).

- The input synthesis (modes scattered into a half spectrum, one inverse
  FFT) equals the mode sum evaluated point by point.
- Running the oracle's full step (FFTs included) on the synthesized grid for
  K steps gives the fields that the per-mode exact update, synthesized plane
  by plane, predicts.  Even axes, so the Nyquist modes are covered; every kx
  column carries a mode.
"""

import numpy as np
import pytest

import oracle
import test_gpu_fullsize_modes as fm


def _pointwise(m, amp, shape):
    nz, ny, nx = shape
    iz, iy, ix = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    acc = np.zeros(shape)
    for (a, b, c), v in zip(m, amp):
        th = 2 * np.pi * (((a * ix) % nx) / nx + ((b * iy) % ny) / ny + ((c * iz) % nz) / nz)
        acc += 2 * np.real(v * np.exp(1j * th))
    return acc


def test_half_spectrum_synthesis_matches_pointwise_sum():
    import torch
    shape = (8, 6, 10)
    md = fm._setup(shape, (0.1, 0.2, 0.3), 0.05, True, np.random.default_rng(0), extra=20)
    for amp in (md["E"][:, 1], md["J"][:, 0], md["drho"]):
        got = fm._device_field(torch, shape, md["m"], amp, device="cpu").double().numpy()
        ref = _pointwise(md["m"], amp, shape).ravel()
        # the synthesis returns FP32
        assert np.max(np.abs(got - ref)) <= 2e-7 * np.max(np.abs(ref))


@pytest.mark.parametrize("sources", [False, True])
def test_mode_synthesis_matches_full_oracle_step(sources):
    shape = (16, 12, 18)
    d, dt, K = (0.1, 0.13, 0.07), 0.05, 3
    md = fm._setup(shape, d, dt, sources, np.random.default_rng(1), extra=30)
    assert set(md["m"][:, 0] % shape[2]) >= set(range(shape[2] // 2 + 1))
    E = [_pointwise(md["m"], md["E"][:, i], shape) for i in range(3)]
    B = [_pointwise(md["m"], md["B"][:, i], shape) for i in range(3)]
    J = [_pointwise(md["m"], md["J"][:, i], shape) for i in range(3)]
    dr = _pointwise(md["m"], md["drho"], shape)
    for n in range(K):
        if sources:
            E, B = oracle.psatd_step(E, B, J, n * dr, (n + 1) * dr, d=d, dt=dt)
        else:
            E, B = oracle.psatd_step(E, B, d=d, dt=dt)
    amps = fm._exact(md, K, dt, sources)
    for axis, n_ax in ((0, shape[0]), (1, shape[1]), (2, shape[2])):
        for pos in range(n_ax):
            for c, f in enumerate(E + B):
                got = f[pos] if axis == 0 else (f[:, pos] if axis == 1 else f[:, :, pos])
                ref = fm._plane(md["m"], amps[:, c], shape, axis, pos)
                assert np.max(np.abs(got - ref)) < 1e-13 * max(1.0, np.max(np.abs(ref)))
