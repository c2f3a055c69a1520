"""Pins of the oracle's multigrid Poisson solver and gravity (paper Sec. 6,
6.2, App. C) against independent facts:

* the seven-point Laplacian's eigenvalues on a single Fourier mode;
* the converged MG solution against numpy's FFT solve of the same discrete
  operator (eigenvalues (2cos(2 pi nx/N)+2cos(2 pi ny/N)+2cos(2 pi nz/N)-6)/h^2);
* the V(2,2) convergence factor;
* the self-adjointness of the converged solve, (A^-1)^T = A^-1 (Sec. 6.2.4);
* the gravity acceleration of a single density mode in closed form.
"""
import math

import numpy as np
import pytest

import oracle
import workloads as wl


def mgcfg(n, **kw):
    g = wl.cube(n)
    return oracle.make_config(g.shape, g.h, **kw)


def fft_solve(F, h):
    n = F.shape[0]
    k = 2 * np.pi * np.fft.fftfreq(n, 1.0 / n) / n
    kz, ky, kx = np.meshgrid(k, k, k, indexing="ij")
    lam = (2 * np.cos(kx) + 2 * np.cos(ky) + 2 * np.cos(kz) - 6.0) / (h * h)
    Fh = np.fft.fftn(F)
    lam[0, 0, 0] = 1.0
    ph = Fh / lam
    ph[0, 0, 0] = 0.0
    return np.real(np.fft.ifftn(ph))


def test_laplacian_eigenvalue():
    n, h = 16, 1.0 / 16
    z, y, x = np.meshgrid(*(wl.centres(n),) * 3, indexing="ij")
    m = (2, 1, 3)
    phi = np.cos(2 * np.pi * (m[0] * x + m[1] * y + m[2] * z) + 0.3)
    lam = (2 * np.cos(2 * np.pi * m[0] / n) + 2 * np.cos(2 * np.pi * m[1] / n) +
           2 * np.cos(2 * np.pi * m[2] / n) - 6.0) / h ** 2
    out = oracle.laplacian(n, h, phi)
    assert np.abs(out - lam * phi).max() < 1e-10 * abs(lam)


@pytest.mark.parametrize("n", [16, 32])
def test_mg_matches_fft_solve(n):
    rng = np.random.default_rng(n)
    h = 1.0 / n
    F = rng.standard_normal((n, n, n))
    F -= F.mean()
    c = mgcfg(n, mg_tol=1e-13, mg_max_cycles=60)
    phi, cyc = oracle.mg_solve(c, n, h, np.zeros_like(F), F)
    ref = fft_solve(F, h)
    assert np.abs(phi - ref).max() < 1e-10 * np.abs(ref).max()
    assert cyc < 60


@pytest.mark.parametrize("n", [32, 64])
def test_vcycle_convergence_factor(n):
    rng = np.random.default_rng(1)
    h = 1.0 / n
    F = rng.standard_normal((n, n, n))
    F -= F.mean()
    c = mgcfg(n)
    phi = np.zeros_like(F)
    res = []
    for _ in range(6):
        r = F - oracle.laplacian(n, h, phi)
        res.append(math.sqrt((r * r).sum()))
        phi = oracle.mg_vcycle(c, n, h, phi, F)
        phi -= phi.mean()
    factors = [res[i + 1] / res[i] for i in range(len(res) - 1)]
    assert max(factors[1:]) < 0.5, factors


def test_converged_solve_is_self_adjoint():
    n = 16
    h = 1.0 / n
    rng = np.random.default_rng(5)
    x = rng.standard_normal((n, n, n)); x -= x.mean()
    y = rng.standard_normal((n, n, n)); y -= y.mean()
    c = mgcfg(n, mg_tol=1e-13, mg_max_cycles=60)
    Ax, _ = oracle.mg_solve(c, n, h, np.zeros_like(x), x)
    Ay, _ = oracle.mg_solve(c, n, h, np.zeros_like(y), y)
    a, b = (Ax * y).sum(), (x * Ay).sum()
    assert a == pytest.approx(b, rel=1e-11)


def test_gravity_of_single_mode():
    n = 32
    h = 1.0 / n
    G = 2.5
    eps = 0.01
    m = (1, 2, 3)
    z, y, x = np.meshgrid(*(wl.centres(n),) * 3, indexing="ij")
    th = 2 * np.pi * (m[0] * x + m[1] * y + m[2] * z)
    rho = 1.0 + eps * np.cos(th)
    o = np.zeros_like(rho)
    U = wl.conserved(rho, o, o, o, np.ones_like(rho), 5 / 3)
    c = mgcfg(n, flags=oracle.SRC_GRAVITY, grav_G=G, mg_tol=1e-13, mg_max_cycles=60)
    acc, phi, cyc = oracle.gravity_accel(c, U, np.zeros_like(rho))
    lam = sum(2 * np.cos(2 * np.pi * mi / n) - 2 for mi in m) / h ** 2
    amp = 4 * np.pi * G * eps / lam
    assert np.abs(phi - amp * np.cos(th)).max() < 1e-10 * abs(amp)
    # central difference of cos(th) along axis a: -sin(th) sin(2 pi m_a / n) / h
    for a in range(3):
        g = amp * np.sin(th) * np.sin(2 * np.pi * m[a] / n) / h
        assert np.abs(acc[a] - g).max() < 1e-9 * np.abs(g).max(), a


def test_warm_start_and_cycle_cap():
    n = 16
    h = 1.0 / n
    rng = np.random.default_rng(2)
    F = rng.standard_normal((n, n, n)); F -= F.mean()
    c = mgcfg(n, mg_tol=1e-10, mg_max_cycles=40)
    phi, cyc = oracle.mg_solve(c, n, h, np.zeros_like(F), F)
    assert 1 <= cyc < 40
    phi2, cyc2 = oracle.mg_solve(c, n, h, phi, F)
    assert cyc2 == 0
    c0 = mgcfg(n, mg_tol=0.0, mg_max_cycles=3)
    _, cyc3 = oracle.mg_solve(c0, n, h, np.zeros_like(F), F)
    assert cyc3 == 3
