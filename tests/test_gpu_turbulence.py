"""The library's standalone 3D FFT (mh_fft3) against numpy, and the
phase-parametrised turbulent initial condition (turbulence.py): its forward
map against a numpy construction of the same field, its written-out reverse
pass against finite differences, and the turbulence reconstruction lowering
its projected-density misfit."""
import math

import numpy as np
import pytest

import paper_2512_13403_amd as mh
from paper_2512_13403_amd import turbulence as tb

pytestmark = pytest.mark.gpu


@pytest.fixture(autouse=True)
def _name(request):
    print(f"\n[gpu case] {request.node.nodeid}", flush=True)
    yield


def dev(a, dtype="f64"):
    import torch

    return torch.tensor(np.asarray(a), dtype=torch.float64 if dtype == "f64" else torch.float32,
                        device="cuda:0")


# n = 2 .. 128: one to three line blocks per workgroup regime, radix-2/4
# remainders, one and two radix-8 passes, XCD-ordered grids of 8 to 1024 blocks
@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("n", [2, 8, 16, 32, 64, 128])
def test_fft3_matches_numpy(dtype, n):
    rng = np.random.default_rng(n)
    z = rng.standard_normal((n, n, n)) + 1j * rng.standard_normal((n, n, n))
    x = dev(np.stack([z.real, z.imag], axis=-1), dtype).contiguous()
    tol = 1e-12 if dtype == "f64" else 2e-5
    fwd = mh.fft3(x.clone(), inverse=False).cpu().numpy()
    ref = np.fft.fftn(z)
    assert np.abs(fwd[..., 0] + 1j * fwd[..., 1] - ref).max() < tol * np.abs(ref).max()
    inv = mh.fft3(x.clone(), inverse=True).cpu().numpy()
    ref = np.fft.ifftn(z) * n ** 3
    assert np.abs(inv[..., 0] + 1j * inv[..., 1] - ref).max() < tol * np.abs(ref).max()


def test_fft3_512_sampled_outputs_and_round_trip():
    """512^3 fp32 (three radix-8 passes, z lines striding 2 MB planes): the
    inverse of the forward transform returns n^3 x, and sampled outputs match
    the DFT sum written out in fp64."""
    import torch

    n = 512
    g = torch.Generator(device="cuda:0").manual_seed(7)
    x = torch.randn((n, n, n, 2), dtype=torch.float32, device="cuda:0", generator=g)
    X = mh.fft3(x.clone())
    y = mh.fft3(X.clone(), inverse=True)
    assert float((y / n ** 3 - x).abs().max()) < 1e-5 * float(x.abs().max())
    del y
    Xs = {}
    samples = [(0, 0, 1), (3, 500, 1), (256, 17, 257), (511, 256, 257)]  # (kz, ky, kx)
    for kz, ky, kx in samples:
        Xs[(kz, ky, kx)] = complex(X[kz, ky, kx, 0].item(), X[kz, ky, kx, 1].item())
    del X
    xc = x.double().cpu().numpy()
    z = xc[..., 0] + 1j * xc[..., 1]
    del xc, x
    l2 = float(np.sqrt((np.abs(z) ** 2).sum()))
    j = np.arange(n)
    for kx in sorted({s[2] for s in samples}):
        S = z @ np.exp(-2j * np.pi * kx * j / n)  # [z][y]: the sum over x
        for kz, ky, kx2 in samples:
            if kx2 != kx:
                continue
            ref = np.exp(-2j * np.pi * kz * j / n) @ S @ np.exp(-2j * np.pi * ky * j / n)
            assert abs(Xs[(kz, ky, kx)] - ref) < 2e-5 * l2, (kz, ky, kx)


def numpy_field(phases, n, kmin, kmax, power, zeta, mach, rho0, p0, gamma):
    k1 = np.fft.fftfreq(n, d=1.0 / n)
    kz, ky, kx = np.meshgrid(k1, k1, k1, indexing="ij")
    ks = (kx, ky, kz)
    k2 = kx * kx + ky * ky + kz * kz
    k = np.sqrt(k2)
    A = np.where((k >= kmin) & (k <= kmax), np.where(k > 0, k, 1.0) ** (power / 2), 0.0)
    k2s = np.where(k2 > 0, k2, 1.0)
    u = []
    for i in range(3):
        X = np.zeros((n, n, n), complex)
        for j in range(3):
            C = ks[i] * ks[j] / k2s
            M = zeta * ((1.0 if i == j else 0.0) - C) + (1 - zeta) * C
            X += A * M * np.exp(1j * phases[j])
        u.append(np.real(np.fft.ifftn(X)) * n ** 3)
    u = np.array(u)
    v = u * mach * math.sqrt(gamma * p0 / rho0) / math.sqrt((u * u).sum(axis=0).mean())
    E = p0 / (gamma - 1) + 0.5 * rho0 * (v * v).sum(axis=0)
    return np.concatenate([np.full((1, n, n, n), rho0), rho0 * v, E[None]])


KW = dict(kmin=2.0, kmax=4.0, power=-5.0 / 3.0, zeta=0.7)


def test_phase_initial_condition_matches_numpy():
    import torch

    n = 16
    phases = np.random.default_rng(3).uniform(0, 2 * np.pi, (3, n, n, n))
    basis = tb.spectral_basis(n, dtype=torch.float64, device="cuda:0", **KW)
    U = tb.initial_state(dev(phases), basis, mach=1.3).cpu().numpy()
    ref = numpy_field(phases, n, mach=1.3, rho0=1.0, p0=1.0, gamma=5 / 3, **KW)
    assert np.abs(U - ref).max() < 1e-12 * np.abs(ref).max()


def test_phase_gradient_matches_finite_differences():
    import torch

    n = 8
    rng = np.random.default_rng(4)
    phases = rng.uniform(0, 2 * np.pi, (3, n, n, n))
    w = dev(rng.standard_normal((5, n, n, n)))
    basis = tb.spectral_basis(n, dtype=torch.float64, device="cuda:0", **KW)
    p = dev(phases).requires_grad_(True)
    (tb.initial_state(p, basis) * w).sum().backward()
    g = p.grad.cpu().numpy()
    A = basis[0].cpu().numpy()
    idx = np.argwhere(A > 0)
    picks = idx[rng.choice(len(idx), 6, replace=False)]
    eps = 1e-6
    for q in picks:
        for j in range(3):
            e = np.zeros_like(phases)
            e[(j,) + tuple(q)] = eps
            lp = float((tb.initial_state(dev(phases + e), basis) * w).sum())
            lm = float((tb.initial_state(dev(phases - e), basis) * w).sum())
            fd = (lp - lm) / (2 * eps)
            assert g[(j,) + tuple(q)] == pytest.approx(fd, rel=1e-6, abs=1e-8), (j, q)


def test_turbulent_phase_inversion_reduces_misfit():
    import torch

    n, nsteps = 32, 20
    g = mh.grid_desc((n, n, n), (1.0 / n,) * 3, dtype="f64")
    s = mh.Solver(g, mh.physics_desc())
    basis = tb.spectral_basis(n, dtype=torch.float64, device="cuda:0", **KW)
    rng = np.random.default_rng(11)
    true = dev(rng.uniform(0, 2 * np.pi, (3, n, n, n)))
    s.set_state(tb.initial_state(true, basis))
    dts = s.step(nsteps, 0.0, record=True)
    target = s.get_state_device()[0].sum(dim=0).clone()
    start = dev(np.random.default_rng(12).uniform(0, 2 * np.pi, (3, n, n, n)))
    _, losses = tb.invert_turbulent_phases(s, start, target, dts, basis, iters=25, lr=0.1, K=5)
    print("phase misfit", losses[0], "->", losses[-1], flush=True)
    assert all(np.isfinite(losses))
    assert losses[-1] < 0.5 * losses[0]
