"""Pins of the oracle's hydrodynamic step against facts fixed by the paper and
by the mathematics, not by the oracle itself (paper App. A.1-A.4):

* exact Riemann solution of the Sod tube (independent solver, Toro ch. 4,
  itself pinned to Toro's printed star values in tests/golden/);
* closed forms: the CFL step of a uniform state; HLLC reducing to exact upwind
  transport for a contact discontinuity;
* invariants: uniform-state fixed point, stationary contact, discrete
  conservation, transverse invariance, axis permutation and mirror symmetry;
* convergence orders in space and time.
"""
import json
import math
import os

import numpy as np
import pytest

import exact_riemann as er
import oracle
import workloads as wl

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def cfg_for(grid, **kw):
    return oracle.make_config(grid.shape, grid.h, grid.bc, **kw)


def rel_field_err(a, b):
    """max over fields of ||a_f - b_f||_inf / D_f, D_rho = ||rho||_inf,
    D_E = ||E||_inf, D_m = sqrt(||rho|| ||E||)."""
    Dr = np.abs(b[0]).max()
    DE = np.abs(b[4]).max()
    D = [Dr, math.sqrt(Dr * DE), math.sqrt(Dr * DE), math.sqrt(Dr * DE), DE]
    return max(np.abs(a[f] - b[f]).max() / D[f] for f in range(5))


# --------------------------------------------------------------------- exact solver pin

def test_exact_riemann_matches_toro_table():
    g = json.load(open(os.path.join(GOLDEN, "sod_star_toro.json")))
    ps, us, res = er.star_state(g["left"], g["right"], g["gamma"])
    assert abs(res) < 1e-13
    assert ps == pytest.approx(g["p_star"], rel=5e-5)
    assert us == pytest.approx(g["u_star"], rel=5e-5)
    # star densities: just left of the contact and just right of it
    rl = er.sample(g["left"], g["right"], g["gamma"], us - 1e-9)[0]
    rr = er.sample(g["left"], g["right"], g["gamma"], us + 1e-9)[0]
    assert rl == pytest.approx(g["rho_star_left"], rel=5e-5)
    assert rr == pytest.approx(g["rho_star_right"], rel=5e-5)


def test_exact_riemann_trivial_cases():
    ps, us, _ = er.star_state((1.0, 0.3, 2.0), (1.0, 0.3, 2.0), 1.4)
    assert ps == pytest.approx(2.0, rel=1e-14) and us == pytest.approx(0.3, rel=1e-14)
    # symmetric rarefactions: u* = 0 by symmetry
    ps, us, _ = er.star_state((1.0, -1.0, 1.0), (1.0, 1.0, 1.0), 1.4)
    assert abs(us) < 1e-14 and ps < 1.0


# --------------------------------------------------------------------- closed forms

def test_cfl_dt_closed_form():
    grid = wl.Grid((4, 5, 6), (0.1, 0.2, 0.05))
    gam = 1.4
    U = wl.rest_state(grid.shape, rho=1.3, p=0.7, gamma=gam, v=(0.3, -0.2, 0.1))
    c = cfg_for(grid, gamma=gam, cfl=0.4)
    cs = math.sqrt(gam * 0.7 / 1.3)
    smax = max((0.3 + cs) / 0.1, (0.2 + cs) / 0.2, (0.1 + cs) / 0.05)
    assert oracle.cfl_dt(c, U) == pytest.approx(0.4 / smax, rel=1e-15)


@pytest.mark.parametrize("u", [0.5, -0.5, 2.0, -2.0])
@pytest.mark.parametrize("axis", [0, 1, 2])
def test_hllc_contact_is_exact_upwind(u, axis):
    """First order (no slopes): a contact at uniform velocity u and pressure p
    is transported by HLLC exactly like the upwind scheme,
    U_i' = U_i - (dt u / h)(U_i - U_{i-1}) for u > 0 (mirror for u < 0)."""
    n = 16
    shape = [1, 1, 1]
    shape[2 - axis] = n
    h = [0.5, 0.5, 0.5]
    h[axis] = 1.0 / n
    grid = wl.Grid(tuple(shape), tuple(h))
    rng = np.random.default_rng(3)
    rho = rng.uniform(0.5, 2.0, shape)
    v = [0.0, 0.0, 0.0]
    v[axis] = u
    U = wl.conserved(rho, np.full(shape, v[0]), np.full(shape, v[1]), np.full(shape, v[2]),
                     np.full(shape, 1.0), 1.4)
    c = cfg_for(grid, gamma=1.4, limiter=oracle.LIM_NONE)
    dt = 0.3 / n / abs(u)
    out = oracle.euler(c, U, dt)
    arr_axis = 3 - axis  # axis of the (5, nz, ny, nx) array
    up = np.roll(U, 1 if u > 0 else -1, axis=arr_axis)
    expect = U - dt * abs(u) * n * (U - up)
    assert rel_field_err(out, expect) < 2e-14


# --------------------------------------------------------------------- invariants

def test_uniform_state_is_bitwise_fixed_point():
    grid = wl.Grid((5, 6, 8), (0.1, 0.13, 0.07))
    U = wl.rest_state(grid.shape, rho=0.8, p=1.7, v=(0.4, -0.9, 0.25))
    c = cfg_for(grid)
    out = oracle.rk2(c, U, 1e-3)
    assert np.array_equal(out, U)


def test_stationary_contact_is_preserved():
    n = 32
    grid = wl.Grid((1, 1, n), (1.0 / n, 1.0, 1.0))
    rng = np.random.default_rng(1)
    rho = np.repeat(rng.uniform(0.2, 5.0, 4), n // 4).reshape(1, 1, n)
    z = np.zeros((1, 1, n))
    U = wl.conserved(rho, z, z, z, np.full((1, 1, n), 1.0), 5.0 / 3.0)
    c = cfg_for(grid)
    sim = oracle.Simulation(c, U).advance(100)
    assert rel_field_err(sim.U, U) < 1e-14


def test_conservation_periodic_random():
    grid = wl.Grid((8, 10, 12), (1 / 12, 1 / 10, 1 / 8))
    U = wl.random_state(grid.shape, seed=7)
    c = cfg_for(grid)
    sim = oracle.Simulation(c, U).advance(5)
    for f in range(5):
        s0 = math.fsum(U[f].ravel())
        s1 = math.fsum(sim.U[f].ravel())
        scale = math.fsum(np.abs(U[f]).ravel())
        assert abs(s1 - s0) / scale < 1e-13, f


def test_permutation_symmetry():
    """Cyclic relabelling x->y->z->x of a random cube state commutes with the step."""
    n = 8
    grid = wl.cube(n)
    U = wl.random_state(grid.shape, seed=11)
    c = cfg_for(grid)
    dt = 0.5 * oracle.cfl_dt(c, U)

    def perm(V):
        # new x <- old z, new y <- old x, new z <- old y; arrays are (f, z, y, x)
        A = np.transpose(V, (0, 2, 1, 3))          # (f, y, z, x)
        A = np.transpose(A, (0, 1, 3, 2))          # (f, y, x, z): axes z'=y, y'=x, x'=z
        return np.ascontiguousarray(A[[0, 3, 1, 2, 4]])

    a = perm(oracle.rk2(c, U, dt))
    b = oracle.rk2(c, perm(U), dt)
    assert rel_field_err(a, b) < 1e-14


@pytest.mark.parametrize("axis", [0, 1, 2])
def test_mirror_symmetry(axis):
    grid = wl.Grid((6, 7, 8), (1 / 8, 1 / 7, 1 / 6))
    U = wl.random_state(grid.shape, seed=5 + axis)
    c = cfg_for(grid)
    dt = 0.5 * oracle.cfl_dt(c, U)
    arr_axis = 3 - axis

    def mirror(V):
        A = np.flip(V, axis=arr_axis).copy()
        A[1 + axis] *= -1.0
        return A

    a = mirror(oracle.rk2(c, U, dt))
    b = oracle.rk2(c, mirror(U), dt)
    assert rel_field_err(a, b) < 1e-14


def test_rk2_is_average_of_two_euler_stages():
    grid = wl.Grid((6, 6, 6), (1 / 6,) * 3)
    U = wl.random_state(grid.shape, seed=2)
    c = cfg_for(grid)
    dt = 0.4 * oracle.cfl_dt(c, U)
    ee = oracle.euler(c, oracle.euler(c, U, dt), dt)
    assert np.array_equal(oracle.rk2(c, U, dt), 0.5 * U + 0.5 * ee)


# --------------------------------------------------------------------- Sod

def _sod_run(nx, ny=1, nz=1, limiter=oracle.LIM_MINMOD, riemann=oracle.RS_HLLC):
    grid = wl.sod_grid(nx, ny, nz)
    U = wl.sod_state(grid)
    c = cfg_for(grid, gamma=1.4, cfl=0.4, limiter=limiter, riemann=riemann)
    sim = oracle.Simulation(c, U)
    nsteps = sim.run_to(0.2)
    return sim, nsteps


def _sod_l1(sim, nx):
    ra, _, _ = er.cell_average_profile((1.0, 0.0, 1.0), (0.125, 0.0, 0.1), 1.4, nx, 0.5, 0.2)
    return np.mean(np.abs(sim.U[0, 0, 0] - ra))


@pytest.fixture(scope="module")
def sod128():
    return _sod_run(128, 16, 16)


def test_sod_reaches_t_exactly_and_counts_steps(sod128):
    sim, nsteps = sod128
    assert sim.t == pytest.approx(0.2, abs=1e-15)
    # the CFL step shrinks once the shock forms: 76 steps at the initial
    # signal speed, noticeably more in practice
    assert 100 < nsteps < 200


def test_sod_transverse_invariance_is_bitwise(sod128):
    sim, _ = sod128
    U = sim.U
    ref = U[:, :1, :1, :]
    assert np.array_equal(U, np.broadcast_to(ref, U.shape))
    assert np.all(U[2] == 0.0) and np.all(U[3] == 0.0)


def test_sod_mass_energy_conserved_and_momentum_bookkeeping(sod128):
    sim, _ = sod128
    grid = wl.sod_grid(128, 16, 16)
    U0 = wl.sod_state(grid)
    for f in (0, 4):
        s0, s1 = math.fsum(U0[f].ravel()), math.fsum(sim.U[f].ravel())
        assert abs(s1 - s0) / s0 < 1e-13
    # outflow ends keep v = 0 and uniform p, so per pencil sum_i m_i grows by
    # dt (p_left - p_right) / h every step
    growth = math.fsum(sim.dts) * (1.0 - 0.1) * 128 * 16 * 16
    assert math.fsum(sim.U[1].ravel()) == pytest.approx(growth, rel=1e-12)


def test_sod_against_exact_solution(sod128):
    sim, _ = sod128
    nx = 128
    x = (np.arange(nx) + 0.5) / nx
    rho = sim.U[0, 0, 0]
    u = sim.U[1, 0, 0] / rho
    p = (1.4 - 1) * (sim.U[4, 0, 0] - 0.5 * rho * u * u)
    ps, us, _ = er.star_state((1.0, 0.0, 1.0), (0.125, 0.0, 0.1), 1.4)
    # star plateau between the rarefaction tail and the shock, away from fronts
    tail = 0.5 + 0.2 * (us - math.sqrt(1.4 * ps / 0.42632) * 1.0)
    plateau = (x > tail + 0.03) & (x < 0.5 + 0.2 * us - 0.03)
    assert np.all(np.abs(p[plateau] / ps - 1) < 0.01)
    assert np.all(np.abs(u[plateau] / us - 1) < 0.01)
    # positions: contact at 0.5 + 0.2 u*, shock at 0.5 + 0.2 S_shock
    ex_r, _, _ = er.cell_average_profile((1.0, 0.0, 1.0), (0.125, 0.0, 0.1), 1.4, 4096, 0.5, 0.2)
    xf = (np.arange(4096) + 0.5) / 4096

    def front(xs, r, lo, hi, level):
        m = (xs > lo) & (xs < hi)
        idx = np.where(m & (r < level))[0]
        return xs[idx[0]]

    shock_ex = front(xf, ex_r, 0.75, 0.95, 0.5 * (0.26557 + 0.125))
    shock = front(x, rho, 0.75, 0.95, 0.5 * (0.26557 + 0.125))
    contact_ex = front(xf, ex_r, 0.6, 0.75, 0.5 * (0.42632 + 0.26557))
    contact = front(x, rho, 0.6, 0.75, 0.5 * (0.42632 + 0.26557))
    assert abs(shock - shock_ex) < 2.0 / nx
    assert abs(contact - contact_ex) < 2.0 / nx


@pytest.mark.parametrize("limiter,riemann", [
    (oracle.LIM_MINMOD, oracle.RS_HLLC),
    (oracle.LIM_VANLEER, oracle.RS_HLLC),
    (oracle.LIM_MC, oracle.RS_HLLC),
    (oracle.LIM_SUPERBEE, oracle.RS_HLLC),
    (oracle.LIM_NONE, oracle.RS_HLLC),
    (oracle.LIM_MINMOD, oracle.RS_HLL),
    (oracle.LIM_MINMOD, oracle.RS_RUSANOV),
])
def test_sod_l1_converges(limiter, riemann):
    errs = []
    for nx in (64, 128, 256, 512):
        sim, _ = _sod_run(nx, limiter=limiter, riemann=riemann)
        errs.append(_sod_l1(sim, nx))
    errs = np.array(errs)
    assert np.all(np.diff(errs) < 0)
    order = math.log2(errs[-2] / errs[-1])
    assert order > (0.45 if limiter == oracle.LIM_NONE else 0.6)
    if limiter == oracle.LIM_MINMOD and riemann == oracle.RS_HLLC:
        assert errs[1] < 0.01


# --------------------------------------------------------------------- orders

def _advect_l1(n, limiter=oracle.LIM_MINMOD):
    grid = wl.Grid((1, 1, n), (1.0 / n, 1.0, 1.0))
    x = wl.centres(n).reshape(1, 1, n)
    rho = 1.0 + 0.2 * np.sin(2 * np.pi * x)
    o = np.ones((1, 1, n))
    U = wl.conserved(rho, o, 0 * o, 0 * o, o, 1.4)
    c = cfg_for(grid, gamma=1.4, cfl=0.4, limiter=limiter)
    sim = oracle.Simulation(c, U)
    sim.run_to(1.0)
    return np.mean(np.abs(sim.U[0] - rho))


def test_smooth_advection_order():
    """A density wave at uniform velocity and pressure is linear advection:
    PLM converges at order between 1.5 and 2 in L1 (minmod clips extrema)."""
    e = [_advect_l1(n) for n in (32, 64, 128, 256)]
    orders = [math.log2(e[i] / e[i + 1]) for i in range(3)]
    assert orders[-1] > 1.5, orders
    assert orders[-1] < 2.3, orders
    e2 = [_advect_l1(n, oracle.LIM_VANLEER) for n in (64, 128, 256)]
    assert math.log2(e2[-2] / e2[-1]) > 1.7


def test_temporal_order_of_rk2():
    """On a fixed grid the step is a two-stage RK method for the semi-discrete
    system: halving dt reduces the time error about fourfold."""
    n = 32
    grid = wl.Grid((1, 1, n), (1.0 / n, 1.0, 1.0))
    x = wl.centres(n).reshape(1, 1, n)
    o = np.ones((1, 1, n))
    U = wl.conserved(1.0 + 0.01 * np.sin(2 * np.pi * x), 0.01 * np.sin(2 * np.pi * x), 0 * o,
                     0 * o, 1.0 + 0.014 * np.sin(2 * np.pi * x), 1.4)
    c = cfg_for(grid, gamma=1.4, limiter=oracle.LIM_NONE)
    T = 0.25
    outs = []
    for m in (8, 16, 32, 64):
        outs.append(oracle.Simulation(c, U).advance(m, T / m).U)
    d = [np.abs(outs[i] - outs[i + 1]).max() for i in range(3)]
    ratio = d[1] / d[2]
    assert 3.3 < ratio < 4.7, d


def test_temporal_order_of_ssprk3():
    """The SSPRK3 option is a third-order method for the semi-discrete system:
    halving dt reduces the time error about eightfold."""
    n = 32
    grid = wl.Grid((1, 1, n), (1.0 / n, 1.0, 1.0))
    x = wl.centres(n).reshape(1, 1, n)
    o = np.ones((1, 1, n))
    U = wl.conserved(1.0 + 0.01 * np.sin(2 * np.pi * x), 0.01 * np.sin(2 * np.pi * x), 0 * o,
                     0 * o, 1.0 + 0.014 * np.sin(2 * np.pi * x), 1.4)
    c = cfg_for(grid, gamma=1.4, limiter=oracle.LIM_NONE, integrator=oracle.RK_SSP3)
    T = 0.25
    outs = []
    for m in (8, 16, 32, 64):
        outs.append(oracle.Simulation(c, U).advance(m, T / m).U)
    d = [np.abs(outs[i] - outs[i + 1]).max() for i in range(3)]
    ratio = d[1] / d[2]
    assert 6.5 < ratio < 9.5, d


STABILITY_POLYNOMIAL = {
    oracle.RK_EULER: lambda z: 1 + z,
    oracle.RK_SSP2: lambda z: 1 + z + z * z / 2,
    oracle.RK_SSP3: lambda z: 1 + z + z * z / 2 + z ** 3 / 6,
}


@pytest.mark.parametrize("integrator", sorted(STABILITY_POLYNOMIAL))
@pytest.mark.parametrize("k", [1, 3, 6])
def test_integrator_amplifies_a_density_wave_by_its_stability_polynomial(integrator, k):
    """A density wave at uniform velocity u > 0 and pressure, with piecewise
    constant faces, is exactly linear upwind advection (HLLC returns the
    upwind flux at a contact), d rho_i/dt = -(u/h)(rho_i - rho_{i-1}), whose
    Fourier mode exp(i theta j) has the eigenvalue lambda = -(u/h)(1 - exp(-i
    theta)).  One step multiplies the mode by the integrator's stability
    polynomial R(dt lambda): 1 + z (Euler), 1 + z + z^2/2 (two-stage SSP),
    1 + z + z^2/2 + z^3/6 (SSPRK3), a closed form independent of the stage
    coefficients; the velocity and pressure stay uniform."""
    n = 16
    grid = wl.Grid((1, 1, n), (1.0 / n, 1.0, 1.0))
    j = np.arange(n)
    theta = 2.0 * np.pi * k / n
    amp = 0.1 * np.exp(0.4j)
    rho = 1.0 + np.real(amp * np.exp(1j * theta * j))
    u, p, gamma = 0.7, 1.0, 1.4
    o = np.ones((1, 1, n))
    U = wl.conserved(rho.reshape(1, 1, n), u * o, 0 * o, 0 * o, p * o, gamma)
    c = cfg_for(grid, gamma=gamma, limiter=oracle.LIM_NONE, integrator=integrator)
    dt = 0.02
    out = oracle.integrate(c, U, dt)
    lam = -(u * n) * (1.0 - np.exp(-1j * theta))
    want = 1.0 + np.real(STABILITY_POLYNOMIAL[integrator](dt * lam) * amp * np.exp(1j * theta * j))
    assert np.abs(out[0, 0, 0] - want).max() < 1e-14
    assert np.abs(out[1, 0, 0] / out[0, 0, 0] - u).max() < 1e-14
    W = oracle.primitives(c, out)
    assert np.abs(W[4] - p).max() < 1e-13
