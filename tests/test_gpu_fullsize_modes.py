"""GPU parity at the full sizes of the 3D and batched workloads.

The 3D grids (512^3 and 1024 x 1024 x 512) are too large for the FP64
oracle to transform whole in a test, so their inputs are a seeded
superposition of a few lattice Fourier modes: each mode evolves on its own,
the oracle's update (``oracle.update_modes``) gives its exact spectrum after
K steps, and the result is synthesized at 2^20 sampled grid points and
compared with the GPU output there.  The modes include a generic and
near-Nyquist wavevectors, an x-Nyquist mode (the r2c packing of the Nyquist
column), a pure z-Nyquist mode and the DC mode (both k = 0), with transverse
E and B, currents with a longitudinal part, and rho from exact discrete
continuity.  The batched workload (256 patches) runs whole against the
oracle, patch by patch.
"""

import numpy as np
import pytest

import fixtures
import oracle
import paper_1608_05739_amd as pk
from gpu_support import rel_l2, say

pytestmark = pytest.mark.gpu

NSAMPLE = 1 << 20


def _modes(shape, rng):
    nz, ny, nx = shape
    return [(5, 3, -7), (nx // 2 - 1, 1, 2), (1, -(ny // 2 - 3), nz // 2 - 2),
            (nx // 2, 4, 3), (0, 0, nz // 2), (0, 0, 0), (17, -11, 29)]


def _keff(m, n, d):
    """Wavenumber of lattice index m on an axis of n points (Nyquist -> 0)."""
    mm = m % n
    if n % 2 == 0 and mm == n // 2:
        return 0.0
    if mm > n // 2:
        mm -= n
    return 2.0 * np.pi * mm / (n * d)


def _setup(shape, d, dt, sources, rng):
    nz, ny, nx = shape
    modes = []
    for m in _modes(shape, rng):
        k = np.array([_keff(m[0], nx, d[0]), _keff(m[1], ny, d[1]), _keff(m[2], nz, d[2])])
        kn = np.linalg.norm(k)

        def transverse():
            v = rng.normal(size=3) + 1j * rng.normal(size=3)
            if kn > 0:
                kh = k / kn
                v = v - kh * (kh @ v)
            return 0.5 * v

        E = transverse()
        B = transverse()
        J = (0.3 * (rng.normal(size=3) + 1j * rng.normal(size=3))) if sources else np.zeros(3, complex)
        modes.append({"m": m, "k": k, "E": E, "B": B, "J": J,
                      # d rho / dt = -i k.J  (exact discrete continuity), rho^0 = 0
                      "drho": -dt * 1j * (k @ J)})
    return modes


def _exact(modes, K, dt, sources):
    """Spectral amplitudes after K steps (J constant, rho^n = n drho)."""
    out = []
    for md in modes:
        E = [np.array([md["E"][i]]) for i in range(3)]
        B = [np.array([md["B"][i]]) for i in range(3)]
        k = tuple(np.array([md["k"][i]]) for i in range(3))
        for n in range(K):
            if sources:
                J = [np.array([md["J"][i]]) for i in range(3)]
                E, B = oracle.update_modes(E, B, k, dt, Jk=J, rho_old_k=np.array([n * md["drho"]]),
                                           rho_new_k=np.array([(n + 1) * md["drho"]]))
            else:
                E, B = oracle.update_modes(E, B, k, dt)
        out.append((np.array([e[0] for e in E]), np.array([b[0] for b in B])))
    return out


def _phase_factors(torch, m, shape):
    """exp(2 pi i m_a i_a / n_a) per axis, exact integer phases, complex128 on the GPU."""
    nz, ny, nx = shape
    f = []
    for mi, n in ((m[2], nz), (m[1], ny), (m[0], nx)):
        i = torch.arange(n, device="cuda:0", dtype=torch.int64)
        ph = ((mi * i) % n).to(torch.float64) * (2.0 * np.pi / n)
        f.append(torch.polar(torch.ones_like(ph), ph))
    return f[0][:, None, None], f[1][None, :, None], f[2][None, None, :]


def _field(torch, shape, modes, amp):
    """sum_m 2 Re(amp(m) exp(i theta_m(x))) as a flat FP32 device tensor."""
    acc = torch.zeros(shape, dtype=torch.float64, device="cuda:0")
    for md in modes:
        a = complex(amp(md))
        if a == 0:
            continue
        fz, fy, fx = _phase_factors(torch, md["m"], shape)
        acc += 2.0 * torch.real(a * (fz * fy * fx))
    return acc.to(torch.float32).reshape(-1)


def _synth(modes, amps, comp, idx, shape):
    nz, ny, nx = shape
    iz, rem = np.divmod(idx, ny * nx)
    iy, ix = np.divmod(rem, nx)
    val = np.zeros(idx.size)
    for md, a in zip(modes, amps):
        m = md["m"]
        th = 2 * np.pi * (((m[0] * ix) % nx) / nx + ((m[1] * iy) % ny) / ny + ((m[2] * iz) % nz) / nz)
        val += 2.0 * np.real(a[comp] * np.exp(1j * th))
    return val


@pytest.mark.parametrize("index,sources", [(2, False), (2, True), (4, False), (4, True)])
def test_fullsize_3d_lattice_modes(index, sources):
    import torch
    w = fixtures.workload(index, build_fields=False)
    p = w.patches[0]
    shape = p.shape
    K = 3
    rng = np.random.default_rng(5000 + 10 * index + int(sources))
    say(f"workload {index} full size {shape}, {'rho form' if sources else 'vacuum'}, {K} steps")
    modes = _setup(shape, p.d, p.dt, sources, rng)
    E = [_field(torch, shape, modes, lambda md, i=i: md["E"][i]) for i in range(3)]
    B = [_field(torch, shape, modes, lambda md, i=i: md["B"][i]) for i in range(3)]
    mode = "rho" if sources else "vacuum"
    plan = pk.Plan([p], precision="fp32", source_mode=mode, path="fused")
    if sources:
        J = [_field(torch, shape, modes, lambda md, i=i: md["J"][i]) for i in range(3)]
        drho = _field(torch, shape, modes, lambda md: md["drho"]).to(torch.float64)
        ro = torch.empty(drho.shape, dtype=torch.float32, device="cuda:0")
        rn = torch.empty_like(ro)
        for n in range(K):
            ro.copy_(drho * n)
            rn.copy_(drho * (n + 1))
            plan.push(E, B, J, ro, rn, steps=1)
    else:
        plan.push(E, B, steps=K)
    torch.cuda.synchronize()
    plan.close()
    exact = _exact(modes, K, p.dt, sources)
    idx = np.sort(rng.choice(p.cells, size=NSAMPLE, replace=False))
    tidx = torch.from_numpy(idx).to("cuda:0")
    got, ref = [], []
    for c in range(3):
        got.append(E[c][tidx].double().cpu().numpy())
        ref.append(_synth(modes, [e for e, _ in exact], c, idx, shape))
    for c in range(3):
        got.append(B[c][tidx].double().cpu().numpy())
        ref.append(_synth(modes, [b for _, b in exact], c, idx, shape))
    err = rel_l2(got, ref)
    say(f"  rel L2 over {NSAMPLE} sampled points = {err:.3e}")
    assert err < 1e-5


def test_fullsize_batched_256_patches_vs_oracle():
    """All 256 patches of the batched workload, one plan, 2 steps, each patch
    against the oracle (FP32 storage; oracle on the FP32-rounded inputs)."""
    import torch
    w = fixtures.workload(3)
    say(f"workload 3: {len(w.patches)} patches, {w.cells} cells, 2 steps")
    plan = pk.Plan(w.patches, precision="fp32", source_mode="vacuum", path="fused")

    def pack(arrs):
        flat = np.zeros(plan.total_elements, np.float32)
        for off, a in zip(plan.offsets, arrs):
            flat[off:off + a.size] = np.asarray(a, np.float32).ravel()
        return torch.from_numpy(flat).to("cuda:0")

    E = [pack([w.E0[i][c] for i in range(len(w.patches))]) for c in range(3)]
    B = [pack([w.B0[i][c] for i in range(len(w.patches))]) for c in range(3)]
    plan.push(E, B, steps=2)
    torch.cuda.synchronize()
    host = [t.cpu().numpy().astype(np.float64) for t in E + B]
    offs = list(plan.offsets)
    plan.close()
    num = den = 0.0
    worst = 0.0
    for i, p in enumerate(w.patches):
        E0 = [np.asarray(a, np.float32).astype(np.float64) for a in w.E0[i]]
        B0 = [np.asarray(a, np.float32).astype(np.float64) for a in w.B0[i]]
        Er, Br = oracle.psatd_run(E0, B0, 2, d=p.d, dt=p.dt)
        got = [h[offs[i]:offs[i] + p.cells].reshape(p.shape) for h in host]
        ref = Er + Br
        n_i = sum(float(np.sum((g - r) ** 2)) for g, r in zip(got, ref))
        d_i = sum(float(np.sum(r * r)) for r in ref)
        num += n_i
        den += d_i
        worst = max(worst, np.sqrt(n_i / d_i))
    err = np.sqrt(num / den)
    say(f"  rel L2 over all patches = {err:.3e}, worst patch = {worst:.3e}")
    assert err < 1e-5
    assert worst < 1e-5
