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


# ---------------------------------------------------------------- W-cycle, RBGS

@pytest.mark.parametrize("cycle,smoother", [(oracle.MG_W, oracle.SMOOTH_JACOBI),
                                            (oracle.MG_V, oracle.SMOOTH_RBGS),
                                            (oracle.MG_W, oracle.SMOOTH_RBGS)])
def test_cycle_and_smoother_variants_match_fft_solve(cycle, smoother):
    n = 32
    rng = np.random.default_rng(7)
    h = 1.0 / n
    F = rng.standard_normal((n, n, n))
    F -= F.mean()
    c = mgcfg(n, mg_tol=1e-13, mg_max_cycles=60, mg_cycle=cycle, mg_smoother=smoother)
    phi, cyc = oracle.mg_solve(c, n, h, np.zeros_like(F), F)
    ref = fft_solve(F, h)
    assert np.abs(phi - ref).max() < 1e-10 * np.abs(ref).max()
    assert cyc < 60


def _factors(n, **kw):
    rng = np.random.default_rng(1)
    h = 1.0 / n
    F = rng.standard_normal((n, n, n))
    F -= F.mean()
    c = mgcfg(n, **kw)
    phi = np.zeros_like(F)
    res = []
    for _ in range(6):
        r = F - oracle.laplacian(n, h, phi)
        res.append(math.sqrt((r * r).sum()))
        phi = oracle.mg_vcycle(c, n, h, phi, F)
        phi -= phi.mean()
    return [res[i + 1] / res[i] for i in range(len(res) - 1)]


@pytest.mark.parametrize("smoother", [oracle.SMOOTH_JACOBI, oracle.SMOOTH_RBGS])
def test_wcycle_converges_faster_than_vcycle(smoother):
    """App. C: the W-cycle's stronger coarse-grid correction reduces the
    residual more per cycle than the V-cycle, cycle by cycle (with 8-cell
    averaging, trilinear prolongation and weighted Jacobi the smoother limits
    both to about 0.3 per cycle; red-black Gauss-Seidel gets the W-cycle to
    below 0.1, the order of magnitude App. C reports)."""
    fv = _factors(64, mg_smoother=smoother)
    fw = _factors(64, mg_cycle=oracle.MG_W, mg_smoother=smoother)
    assert all(w < v for w, v in zip(fw, fv)), (fw, fv)
    if smoother == oracle.SMOOTH_RBGS:
        assert max(fw[1:]) < 0.1, fw


def test_rbgs_sweep_zeroes_the_residual_on_black_cells():
    """A red-black Gauss-Seidel sweep updates the black cells last, each to
    the value that satisfies its own equation given its (red) neighbours, so
    afterwards the residual vanishes on every black cell and not on the red
    ones (a swapped colour order, a Jacobi-style update or a wrong stencil
    breaks this)."""
    n = 16
    h = 1.0 / n
    rng = np.random.default_rng(3)
    F = rng.standard_normal((n, n, n)); F -= F.mean()
    phi0 = rng.standard_normal((n, n, n))
    c = mgcfg(n, mg_smoother=oracle.SMOOTH_RBGS)
    phi = oracle.mg_smooth(c, n, h, phi0, F)
    Aphi = oracle.laplacian(n, h, phi)
    r = F - Aphi
    k, j, i = np.meshgrid(*(np.arange(n),) * 3, indexing="ij")
    black = (i + j + k) % 2 == 1
    tiny = 1e-12 * np.abs(Aphi).max()
    assert np.abs(r[black]).max() < tiny
    assert np.abs(r[~black]).max() > 1e6 * tiny


# ---------------------------------------------------------------- spectral gravity

def test_dft3_matches_numpy_fft():
    rng = np.random.default_rng(4)
    for n in (5, 8):
        x = rng.standard_normal((n, n, n)) + 1j * rng.standard_normal((n, n, n))
        assert np.abs(oracle.dft3(x) - np.fft.fftn(x)).max() < 1e-12 * n ** 3
        assert np.abs(oracle.dft3(x, inverse=True) - np.fft.ifftn(x)).max() < 1e-13 * n ** 3


@pytest.mark.parametrize("n", [8, 12])
def test_spectral_gravity_of_single_mode(n):
    """Sec. 6.1 on rho = 1 + A cos(kappa . x + p): Phi = -4 pi G A cos(.) /
    |kappa|^2 and a = -grad Phi = -4 pi G A kappa sin(.) / |kappa|^2 exactly."""
    L = 2.0
    h = L / n
    G, A, p = 1.7, 0.05, 0.4
    m = (1, -2, 3)
    c = oracle.make_config((n, n, n), (h,) * 3, grav_G=G, grav_solver=oracle.GRAV_FFT)
    z, y, x = np.meshgrid(*((np.arange(n) + 0.5) * h,) * 3, indexing="ij")
    kap = [2 * np.pi * mi / L for mi in m]
    th = kap[0] * x + kap[1] * y + kap[2] * z + p
    phi, acc = oracle.fft_gravity(c, 1.0 + A * np.cos(th))
    k2 = sum(k * k for k in kap)
    assert np.abs(phi + 4 * np.pi * G * A * np.cos(th) / k2).max() < 1e-13
    for a in range(3):
        want = -4 * np.pi * G * A * kap[a] * np.sin(th) / k2
        assert np.abs(acc[a] - want).max() < 1e-13, a


def test_spectral_gravity_nyquist_mode_has_no_gradient():
    """Reading: the derivative of the Nyquist mode is dropped (its i kappa
    factor has no real counterpart), while it still enters the potential."""
    n = 8
    h = 1.0 / n
    G, A = 1.0, 0.1
    c = oracle.make_config((n, n, n), (h,) * 3, grav_G=G, grav_solver=oracle.GRAV_FFT)
    i = np.arange(n).reshape(1, 1, n) * np.ones((n, n, 1))
    phi, acc = oracle.fft_gravity(c, 1.0 + A * (-1.0) ** i)
    kN = np.pi * n
    assert np.abs(phi + 4 * np.pi * G * A * (-1.0) ** i / kN ** 2).max() < 1e-14
    assert np.abs(acc).max() < 1e-14


def test_spectral_gravity_adjoint_identity():
    """rho -> acc is linear: <g, J v> = <J^T g, v> to round-off."""
    n = 8
    h = 1.0 / n
    c = oracle.make_config((n, n, n), (h,) * 3, grav_G=2.0, grav_solver=oracle.GRAV_FFT)
    rng = np.random.default_rng(9)
    v = rng.standard_normal((n, n, n))
    g = rng.standard_normal((3, n, n, n))
    _, Jv = oracle.fft_gravity(c, v)
    lhs = (g * Jv).sum()
    rhs = (oracle.fft_gravity_vjp(c, g) * v).sum()
    assert lhs == pytest.approx(rhs, rel=1e-12)


def test_solve_stops_at_the_round_off_floor():
    """With a tolerance below what the arithmetic can reach, the solve stops
    once a cycle no longer cuts the residual by 10 % (the round-off floor),
    well before the cycle cap, with the residual at the floor; with a
    tolerance of 0 it runs exactly the cap."""
    n = 32
    c = mgcfg(n, mg_tol=1e-30, mg_max_cycles=200)
    rng = np.random.default_rng(3)
    F = rng.standard_normal((n, n, n))
    F -= F.mean()
    phi, cycles = oracle.mg_solve(c, n, 1.0 / n, np.zeros((n, n, n)), F)
    assert 10 < cycles < 60, cycles
    r = F - oracle.laplacian(n, 1.0 / n, phi)
    assert np.linalg.norm(r) < 1e-12 * np.linalg.norm(F)
    c0 = mgcfg(n, mg_tol=0.0, mg_max_cycles=7)
    assert oracle.mg_solve(c0, n, 1.0 / n, np.zeros((n, n, n)), F)[1] == 7
