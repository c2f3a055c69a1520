"""Pins of the oracle's source terms (paper Sec. 3.1.1 OU forcing, Sec. 4
cooling, Sec. 2.1 force-listing kick) against independent facts:

* cooling: the closed form against a high-accuracy adaptive ODE integration
  (scipy DOP853) of dT/dt = -(gamma-1) rho Lambda(T); monotonicity; floor;
* OU: the solenoidal/compressive projection (k . a = 0 / k x a = 0), the
  Parseval normalisation against the grid rms, the DFT of the real-space field
  (only the forced modes, divergence free), Gaussian statistics of the noise,
  the stationary variance and e^{-s/tau} autocorrelation of the OU process;
* kick: exact momentum / energy bookkeeping.
"""
import math

import numpy as np
import pytest
from scipy.integrate import solve_ivp

import oracle
import workloads as wl

CC = wl.COOLING_CURVE


def lam(T):
    if T >= CC["tc"]:
        return CC["lambda0"] * math.sqrt(T / CC["tc"])
    return CC["lambda0"] * math.exp((T - CC["tc"]) / CC["ts"])


@pytest.mark.parametrize("rho", [0.1, 1.0, 7.0])
def test_cooling_closed_form_matches_ode_integration(rho):
    gam = 5.0 / 3.0
    for T0 in (10.0, 1.0, 0.05, 0.0101, 0.01, 0.0099, 5e-3, 1e-3, 2e-4):
        for dt in (1e-4, 1e-2, 0.3, 2.0):
            Tn = oracle.cool_temperature(rho, T0, dt, gam, CC["lambda0"], CC["tc"], CC["ts"], 0.0)
            sol = solve_ivp(lambda t, y: [-(gam - 1.0) * rho * lam(y[0])], (0.0, dt), [T0],
                            method="DOP853", rtol=1e-13, atol=1e-16)
            Tref = sol.y[0, -1]
            # the closed form may legitimately go below 0 only far past the floor
            assert Tn == pytest.approx(Tref, rel=2e-9, abs=1e-13), (T0, dt, Tn, Tref)


def test_cooling_monotone_and_floor():
    gam = 5.0 / 3.0
    T0 = 3.0
    prev = T0
    for dt in np.linspace(0.0, 200.0, 800):
        Tn = oracle.cool_temperature(2.0, T0, dt, gam, CC["lambda0"], CC["tc"], CC["ts"], CC["tfloor"])
        assert Tn <= prev + 1e-15
        assert Tn >= CC["tfloor"]
        prev = Tn
    assert prev == CC["tfloor"]
    assert oracle.cool_temperature(2.0, T0, 0.0, gam, CC["lambda0"], CC["tc"], CC["ts"],
                                   CC["tfloor"]) == pytest.approx(T0, rel=1e-15)


def test_cooling_changes_only_thermal_energy():
    grid = wl.cube(6)
    U = wl.random_state(grid.shape, seed=4)
    c = oracle.make_config(grid.shape, grid.h, flags=oracle.SRC_COOLING)
    out = oracle.cool(c, U, 0.05)
    assert np.array_equal(out[:4], U[:4])
    gam = 5.0 / 3.0
    ek = 0.5 * (U[1] ** 2 + U[2] ** 2 + U[3] ** 2) / U[0]
    T0 = (gam - 1) * (U[4] - ek) / U[0]
    T1 = (gam - 1) * (out[4] - ek) / U[0]
    assert np.all(T1 < T0)
    for q in [(0, 0, 0), (3, 2, 1), (5, 5, 5)]:
        Tq = oracle.cool_temperature(U[0][q], T0[q], 0.05, gam, CC["lambda0"], CC["tc"], CC["ts"],
                                     CC["tfloor"])
        assert T1[q] == pytest.approx(Tq, rel=1e-13)


# ------------------------------------------------------------------ OU forcing

def test_ou_mode_set():
    nv = oracle.ou_modes(1.0, 2.0)
    assert len(nv) == 16  # 32 integer vectors with 1 <= |n| <= 2, one per +- pair
    k = np.sqrt((nv ** 2).sum(1))
    assert np.all((k >= 1) & (k <= 2))
    full = {tuple(v) for v in nv} | {tuple(-v) for v in nv}
    assert len(full) == 32


def test_ou_noise_statistics():
    vals = np.array([oracle.ou_gauss(123, g, m, c) for g in range(200) for m in range(16)
                     for c in range(3)])
    assert abs(vals.real.mean()) < 0.02 and abs(vals.imag.mean()) < 0.02
    assert vals.real.var() == pytest.approx(0.5, rel=0.04)
    assert vals.imag.var() == pytest.approx(0.5, rel=0.04)
    assert abs(np.corrcoef(vals.real, vals.imag)[0, 1]) < 0.03
    # the stream depends on the seed
    assert oracle.ou_gauss(1, 0, 0, 0) != oracle.ou_gauss(2, 0, 0, 0)


@pytest.mark.parametrize("zeta", [1.0, 0.0, 0.4])
def test_ou_projection(zeta):
    grid = wl.cube(8)
    c = oracle.make_config(grid.shape, grid.h, flags=oracle.SRC_FORCING, ou_zeta=zeta)
    nv = oracle.ou_modes(1.0, 2.0)
    a = oracle.ou_advance(c, nv, oracle.ou_init(c, nv), 0, 0.1)
    ah = (a[0::2] + 1j * a[1::2]).reshape(-1, 3)
    div = np.abs((ah * nv).sum(1))
    curl = np.abs(np.cross(ah, nv)).sum(1)
    if zeta == 1.0:
        assert div.max() < 1e-14
    elif zeta == 0.0:
        assert curl.max() < 1e-14
    else:
        assert div.max() > 1e-3 and curl.max() > 1e-3


def test_ou_realspace_field_parseval_and_spectrum():
    shape = (6, 7, 8)
    grid = wl.Grid(shape, (1 / 8, 1 / 7, 1 / 6))
    c = oracle.make_config(shape, grid.h, flags=oracle.SRC_FORCING, ou_arms=1.7)
    nv = oracle.ou_modes(1.0, 2.0)
    a = oracle.ou_init(c, nv)
    acc = oracle.ou_accel(c, nv, a)
    rms = math.sqrt(np.mean((acc ** 2).sum(0)))
    assert rms == pytest.approx(1.7, rel=1e-13)
    # the DFT holds exactly the forced modes and is divergence free
    F = [np.fft.fftn(acc[i]) for i in range(3)]
    nz, ny, nx = shape
    kz, ky, kx = np.meshgrid(np.fft.fftfreq(nz, 1 / nz), np.fft.fftfreq(ny, 1 / ny),
                             np.fft.fftfreq(nx, 1 / nx), indexing="ij")
    power = sum(np.abs(f) ** 2 for f in F)
    forced = np.zeros(shape, bool)
    for v in nv:
        for s in (1, -1):
            forced[(s * v[2]) % nz, (s * v[1]) % ny, (s * v[0]) % nx] = True
    assert power[~forced].max() < 1e-20 * power.max()
    div = np.abs(kx * F[0] + ky * F[1] + kz * F[2])
    assert div.max() < 1e-11 * math.sqrt(power.max())
    # every component of every mode: coefficient = scale * ahat * (half-cell phase)
    scale = oracle.ou_scale(c, a)
    for m, v in enumerate(nv):
        shift = np.exp(1j * np.pi * (v[0] / nx + v[1] / ny + v[2] / nz))
        for comp in range(3):
            ah = complex(a[6 * m + 2 * comp], a[6 * m + 2 * comp + 1])
            coeff = F[comp][v[2] % nz, v[1] % ny, v[0] % nx] / (nx * ny * nz)
            assert coeff == pytest.approx(scale * ah * shift, rel=1e-11, abs=1e-14)


def test_ou_stationary_variance_and_autocorrelation():
    grid = wl.cube(8)
    c = oracle.make_config(grid.shape, grid.h, flags=oracle.SRC_FORCING, ou_seed=9)
    nv = oracle.ou_modes(1.0, 2.0)
    a = oracle.ou_init(c, nv)
    dt, nstep = 0.05, 6000
    hist = np.empty((nstep, a.size))
    for s in range(nstep):
        a = oracle.ou_advance(c, nv, a, s, dt)
        hist[s] = a
    # stationary: E|P eta|^2 = trace(P) = 2 per mode (Re and Im each 1/2 per comp)
    per_mode = (hist ** 2).reshape(nstep, 16, 6).sum(2).mean(0)
    assert per_mode.mean() == pytest.approx(2.0, rel=0.05)
    # autocorrelation at lag s*dt follows exp(-s dt / tau)
    for lag in (2, 10):
        x, y = hist[:-lag].ravel(), hist[lag:].ravel()
        r = (x * y).mean() / (x * x).mean()
        assert r == pytest.approx(math.exp(-lag * dt / 0.5), abs=0.04)


def test_kick_bookkeeping():
    grid = wl.cube(5)
    U = wl.random_state(grid.shape, seed=8)
    rng = np.random.default_rng(0)
    acc = rng.standard_normal((3,) + grid.shape)
    c = oracle.make_config(grid.shape, grid.h)
    dt = 0.03
    out = oracle.kick(c, U, acc, dt)
    assert np.array_equal(out[0], U[0])
    for i in range(3):
        assert np.allclose(out[1 + i] - U[1 + i], U[0] * acc[i] * dt, rtol=0, atol=1e-15)
    dE = (U[1] * acc[0] + U[2] * acc[1] + U[3] * acc[2]) * dt
    assert np.allclose(out[4] - U[4], dE, rtol=0, atol=1e-14)


def test_step_source_order_forcing_then_cooling():
    """A full step with forcing and cooling equals RK2, then the kick with the
    advanced OU modes, then cooling, each on the previous result."""
    grid = wl.cube(6)
    U = wl.smooth_random_state(grid.shape, seed=1)
    c = oracle.make_config(grid.shape, grid.h, flags=oracle.SRC_FORCING | oracle.SRC_COOLING)
    sim = oracle.Simulation(c, U)
    a0 = sim.ahat.copy()
    dt = 0.01
    sim.advance(1, dt)
    V = oracle.rk2(c, U, dt)
    a1 = oracle.ou_advance(c, sim.nvec, a0, 0, dt)
    V = oracle.kick(c, V, oracle.ou_accel(c, sim.nvec, a1), dt)
    V = oracle.cool(c, V, dt)
    assert np.array_equal(sim.U, V)
    assert np.array_equal(sim.ahat, a1)


# ---------------------------------------------------------------- tabulated model (Sec. 4)

def table_cfg(**kw):
    base = dict(cool_model=oracle.COOL_TABLE, cool_table=wl.synthetic_cie_table(),
                **wl.COOLING_TABLE_MODEL)
    base.update(kw)
    return oracle.make_config((2, 2, 2), (0.5,) * 3, flags=oracle.SRC_COOLING, **base)


def test_table_interpolation_is_exact_for_a_power_law():
    """log-log linear interpolation reproduces a pure power law between any
    nodes, and is flat beyond the table's ends."""
    A, b = 0.7, -0.6
    logT = np.array([-2.0, -1.3, -0.2, 0.4, 1.5])
    c = table_cfg(cool_table=(logT, np.log10(A) + b * logT))
    for T in (0.01, 0.02, 0.31, 1.0, 2.5, 30.0):
        assert oracle.cool_lambda(c, T) == pytest.approx(A * T ** b, rel=1e-13)
    assert oracle.cool_lambda(c, 1e3) == pytest.approx(A * 10 ** (1.5 * b), rel=1e-13)


def test_table_search_stops_for_a_non_finite_temperature():
    """A NaN temperature (a non-finite cell) does not walk the interval search
    past the table: the table model returns NaN for it, and every integrator
    returns without reading beyond the nodes (the same bound as the device's
    search).  Finite temperatures are unaffected (the interpolation pin
    above)."""
    nan = float("nan")
    for integ in (oracle.COOLINT_TRAPEZOID, oracle.COOLINT_SUBCYCLE, oracle.COOLINT_AUTO):
        c = table_cfg(cool_integrator=integ, cool_nsub_max=50, cool_frac=0.1)
        assert math.isnan(oracle.cool_lambda(c, nan))
        assert math.isnan(oracle.cool_edot(c, 1.0, nan))
        oracle.cool_eth_step(c, 1.0, nan, 0.1)
        oracle.cool_eth_step(c, nan, 1.0, 0.1)
        oracle.cool_eth_step_d(c, 1.0, nan, 0.1)


def _run(c, rho, E0, t, nsteps):
    E = E0
    for _ in range(nsteps):
        E = oracle.cool_eth_step(c, rho, E, t / nsteps)
    return E


def test_trapezoid_is_second_order_and_subcycling_first_order():
    """Against the closed form for a linear curve Lambda = A T (no heating,
    above tc), T(t) = T0 exp(-(gamma-1) rho A t): halving dt quarters the
    trapezoid's error; doubling the substeps halves the subcycled update's
    error (the fractional change per substep is constant, below the limiter's
    bound)."""
    A, rho, g = 0.5, 1.3, 5.0 / 3.0
    logT = np.array([-2.0, 2.0])
    kw = dict(cool_table=(logT, np.log10(A) + logT), cool_heat=0.0)
    T0, t = 1.0, 0.4
    k = (g - 1) * rho * A
    E0 = rho * T0 / (g - 1)
    Tex = T0 * math.exp(-k * t)
    ct = table_cfg(cool_integrator=oracle.COOLINT_TRAPEZOID, **kw)
    et = [abs(_run(ct, rho, E0, t, m) * (g - 1) / rho - Tex) for m in (8, 16, 32)]
    assert 3.6 < et[0] / et[1] < 4.4 and 3.6 < et[1] / et[2] < 4.4, et
    es = []
    for nsub in (64, 128, 256):
        # N = ceil(k t / f) = nsub
        cs = table_cfg(cool_integrator=oracle.COOLINT_SUBCYCLE, cool_frac=k * t / (nsub - 0.5),
                       cool_nsub_max=100000, **kw)
        E = oracle.cool_eth_step(cs, rho, E0, t)
        assert E == pytest.approx(E0 * (1 - k * t / nsub) ** nsub, rel=1e-12)
        es.append(abs(E * (g - 1) / rho - Tex))
    assert 1.8 < es[0] / es[1] < 2.2 and 1.8 < es[1] / es[2] < 2.2, es


def test_heating_equilibrium_is_a_fixed_point():
    """Below tc, where Gamma_0 = rho Lambda(T_eq), both integrators keep T_eq."""
    from scipy.optimize import brentq

    rho, g = 1.0, 5.0 / 3.0
    c = table_cfg()
    f = lambda T: oracle.cool_edot(c, rho, rho * T / (g - 1))
    Teq = brentq(f, 1e-3, 9e-3, xtol=1e-15)
    for integ in (oracle.COOLINT_TRAPEZOID, oracle.COOLINT_SUBCYCLE, oracle.COOLINT_AUTO):
        ci = table_cfg(cool_integrator=integ)
        E = rho * Teq / (g - 1)
        assert oracle.cool_eth_step(ci, rho, E, 10.0) == pytest.approx(E, rel=1e-9)
    # and it attracts: a perturbed cell relaxes towards it (relaxation rate
    # about 12 here, so dt = 0.025 keeps the explicit update stable)
    E1 = _run(table_cfg(), rho, 1.5 * rho * Teq / (g - 1), 50.0, 2000)
    assert abs(E1 * (g - 1) / rho - Teq) < 1e-3 * Teq


def test_floor_and_fractional_limiter():
    rho, g = 50.0, 5.0 / 3.0
    c = table_cfg(cool_integrator=oracle.COOLINT_SUBCYCLE, cool_nsub_max=4, cool_frac=0.1)
    E0 = rho * 0.1 / (g - 1)
    E1 = oracle.cool_eth_step(c, rho, E0, 1.0)
    # four substeps, each at most a 10 % change
    assert E1 >= E0 * 0.9 ** 4 * (1 - 1e-14)
    cf = table_cfg(cool_integrator=oracle.COOLINT_TRAPEZOID, cool=(0.3, 1e-2, 1e-3, 0.05))
    assert oracle.cool_eth_step(cf, rho, E0, 10.0) == pytest.approx(rho * 0.05 / (g - 1), rel=1e-14)


def test_auto_integrator_picks_by_the_first_step_change():
    rho, g = 1.0, 5.0 / 3.0
    ca, ct, cs = (table_cfg(cool_integrator=m) for m in (oracle.COOLINT_AUTO,
                                                          oracle.COOLINT_TRAPEZOID,
                                                          oracle.COOLINT_SUBCYCLE))
    E = rho * 0.15 / (g - 1)
    small, large = 1e-4, 1.0  # |Edot| dt / E is about 0.002 and 20
    assert oracle.cool_eth_step(ca, rho, E, small) == oracle.cool_eth_step(ct, rho, E, small)
    assert oracle.cool_eth_step(ca, rho, E, large) == oracle.cool_eth_step(cs, rho, E, large)


def test_cooling_time_step_limit():
    """Sec. 4.3: dt <= c_cool min t_cool with t_cool = E_th / |rho Gamma -
    rho^2 Lambda|; for a uniform state the closed form."""
    n, rho, p, g = 4, 2.0, 0.3, 5.0 / 3.0
    U = wl.rest_state((n, n, n), rho=rho, p=p, gamma=g)
    c = oracle.make_config((n, n, n), (1 / n,) * 3, flags=oracle.SRC_COOLING, cool_ccool=0.2,
                           cool_model=oracle.COOL_TABLE, cool_table=wl.synthetic_cie_table(),
                           **wl.COOLING_TABLE_MODEL)
    Eth = p / (g - 1)
    tcool = Eth / abs(oracle.cool_edot(c, rho, Eth))
    cs = math.sqrt(g * p / rho)
    assert oracle.cfl_dt(c, U) == pytest.approx(min(0.4 / (n * cs), 0.2 * tcool), rel=1e-14)
    assert 0.2 * tcool < 0.4 / (n * cs)


@pytest.mark.parametrize("integ", [oracle.COOLINT_TRAPEZOID, oracle.COOLINT_SUBCYCLE,
                                   oracle.COOLINT_AUTO])
def test_tabulated_step_derivatives_match_finite_differences(integ):
    """dE'/dE_th and dE'/drho of the tabulated model's step (forward-mode
    derivatives through the branches taken) against central differences,
    across the heating branch, tc and the table."""
    g = 5.0 / 3.0
    c = table_cfg(cool_integrator=integ, cool_frac=0.05, cool_nsub_max=50)
    for rho, T, dt in ((0.7, 0.002, 0.3), (1.6, 0.008, 0.01), (1.2, 0.05, 0.003),
                       (0.9, 0.4, 0.02), (2.0, 3.0, 0.05)):
        E = rho * T / (g - 1)
        v, dE, dr = oracle.cool_eth_step_d(c, rho, E, dt)
        assert v == oracle.cool_eth_step(c, rho, E, dt)
        h = 1e-7
        fE = (oracle.cool_eth_step(c, rho, E * (1 + h), dt) -
              oracle.cool_eth_step(c, rho, E * (1 - h), dt)) / (2 * h * E)
        fr = (oracle.cool_eth_step(c, rho * (1 + h), E, dt) -
              oracle.cool_eth_step(c, rho * (1 - h), E, dt)) / (2 * h * rho)
        assert dE == pytest.approx(fE, rel=1e-5, abs=1e-9), (rho, T)
        assert dr == pytest.approx(fr, rel=1e-5, abs=1e-9 * abs(v / rho)), (rho, T)
