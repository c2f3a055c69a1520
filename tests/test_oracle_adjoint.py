"""Pins of the oracle's hand-written adjoint (reverse-mode derivative at fixed
dt, paper Sec. 2.3 and Sec. 6.2.4) against fp64 central finite differences of
the oracle's own forward maps: the dot-product identity
w . (J v) = (J^T w) . v with J v from central differences, and single entries
of J^T w against difference quotients along unit vectors.  Inputs are
cell-wise random states, whose minmod decisions have margins of order 1e-4
(a smooth field puts many cells at the |a| = |b| kink, and a state at rest at
the ab = 0 kink, where the one-sided derivatives differ and a difference
quotient straddles them), or perturbations that keep the kinked fields fixed."""
import math

import numpy as np
import pytest

import oracle
import workloads as wl


def fd_jvp(f, U, v, eps):
    """Central difference (f(U + eps v) - f(U - eps v)) / (2 eps)."""
    return (f(U + eps * v) - f(U - eps * v)) / (2.0 * eps)


def check_dot(f, vjp, U, seed, eps=1e-6, rtol=2e-7, trials=3, fields=None):
    """fields: indices of the state fields to perturb (default all)."""
    rng = np.random.default_rng(seed)
    for _ in range(trials):
        v = rng.standard_normal(U.shape) * np.abs(U).mean(axis=tuple(range(1, U.ndim)), keepdims=True)
        if fields is not None:
            mask = np.zeros(U.shape[0])
            mask[list(fields)] = 1.0
            v = v * mask.reshape((-1,) + (1,) * (U.ndim - 1))
        w = rng.standard_normal(U.shape)
        jv = fd_jvp(f, U, v, eps)
        lhs = float((w * jv).sum())
        rhs = float((vjp(w) * v).sum())
        assert lhs == pytest.approx(rhs, rel=rtol), (lhs, rhs)


def check_entries(f, vjp, U, seed, count=12, eps=1e-6, rtol=2e-6):
    rng = np.random.default_rng(seed)
    w = rng.standard_normal(U.shape)
    g = vjp(w)
    flat = rng.choice(U.size, count, replace=False)
    for q in flat:
        e = np.zeros(U.size)
        e[q] = 1.0
        e = e.reshape(U.shape)
        d = float((w * fd_jvp(f, U, e, eps * max(abs(U.flat[q]), 1.0))).sum())
        assert g.flat[q] == pytest.approx(d, rel=rtol, abs=1e-7 * (abs(d) + 1.0)), q


GRIDS = [
    ("periodic", wl.Grid((6, 7, 8), (1 / 8, 1 / 7, 1 / 6))),
    ("outflow", wl.Grid((5, 6, 9), (1 / 9, 1 / 6, 1 / 5), (1, 1, 1))),
    ("mixed", wl.Grid((4, 1, 10), (1 / 10, 1.0, 1 / 4), (1, 0, 0))),
]


@pytest.mark.parametrize("name,grid", GRIDS)
@pytest.mark.parametrize("limiter", [oracle.LIM_MINMOD, oracle.LIM_NONE])
def test_rhs_vjp_dot_product(name, grid, limiter):
    U = wl.random_state(grid.shape, seed=3, vmax=0.7)
    c = oracle.make_config(grid.shape, grid.h, grid.bc, limiter=limiter)
    check_dot(lambda X: oracle.rhs(c, X), lambda w: oracle.rhs_vjp(c, U, w), U, seed=1)


def test_rhs_vjp_entries_rough_state():
    """Cell-wise random state: shocks, every HLLC region and minmod branch."""
    grid = wl.Grid((4, 5, 6), (1 / 6, 1 / 5, 1 / 4))
    U = wl.random_state(grid.shape, seed=21, vmax=1.5)
    c = oracle.make_config(grid.shape, grid.h)
    check_entries(lambda X: oracle.rhs(c, X), lambda w: oracle.rhs_vjp(c, U, w), U, seed=2,
                  count=40, eps=1e-7)


def test_rhs_vjp_supersonic_regions():
    """Uniform supersonic flow plus a small smooth perturbation: every face is
    in the one-sided regions (S_L >= 0), which the dot test then covers."""
    grid = wl.Grid((4, 4, 8), (1 / 8, 1 / 4, 1 / 4))
    U = wl.random_state(grid.shape, seed=4, vmax=0.2)
    U[4] += 0.5 * ((U[1] + 3.0 * U[0]) ** 2 - U[1] ** 2) / U[0]
    U[1] += 3.0 * U[0]  # +3 in vx: Mach > 2
    c = oracle.make_config(grid.shape, grid.h)
    check_dot(lambda X: oracle.rhs(c, X), lambda w: oracle.rhs_vjp(c, U, w), U, seed=5)


SCHEMES = [(oracle.LIM_VANLEER, oracle.RS_HLLC), (oracle.LIM_MC, oracle.RS_HLLC),
           (oracle.LIM_SUPERBEE, oracle.RS_HLLC), (oracle.LIM_MINMOD, oracle.RS_HLL),
           (oracle.LIM_MINMOD, oracle.RS_RUSANOV), (oracle.LIM_VANLEER, oracle.RS_HLL),
           (oracle.LIM_NONE, oracle.RS_RUSANOV)]


@pytest.mark.parametrize("name,grid", GRIDS)
@pytest.mark.parametrize("limiter,riemann", SCHEMES)
def test_rhs_vjp_scheme_variants_dot_product(name, grid, limiter, riemann):
    """Reverse of the other limiters and Riemann solvers of App. A.1/A.2."""
    U = wl.random_state(grid.shape, seed=3, vmax=0.7)
    c = oracle.make_config(grid.shape, grid.h, grid.bc, limiter=limiter, riemann=riemann)
    check_dot(lambda X: oracle.rhs(c, X), lambda w: oracle.rhs_vjp(c, U, w), U, seed=1)


@pytest.mark.parametrize("limiter,riemann", SCHEMES)
def test_rhs_vjp_scheme_variants_entries_rough_state(limiter, riemann):
    grid = wl.Grid((4, 5, 6), (1 / 6, 1 / 5, 1 / 4))
    U = wl.random_state(grid.shape, seed=22, vmax=1.5)
    c = oracle.make_config(grid.shape, grid.h, limiter=limiter, riemann=riemann)
    check_entries(lambda X: oracle.rhs(c, X), lambda w: oracle.rhs_vjp(c, U, w), U, seed=2,
                  count=40, eps=1e-7)


@pytest.mark.parametrize("riemann", [oracle.RS_HLL, oracle.RS_RUSANOV])
def test_rhs_vjp_supersonic_other_solvers(riemann):
    """Every face one-sided for HLL (S_L >= 0); Rusanov's speed from the
    positive |v| branch."""
    grid = wl.Grid((4, 4, 8), (1 / 8, 1 / 4, 1 / 4))
    U = wl.random_state(grid.shape, seed=4, vmax=0.2)
    U[4] += 0.5 * ((U[1] + 3.0 * U[0]) ** 2 - U[1] ** 2) / U[0]
    U[1] += 3.0 * U[0]
    c = oracle.make_config(grid.shape, grid.h, limiter=oracle.LIM_VANLEER, riemann=riemann)
    # van Leer's curvature near a + b = 0 needs the smaller difference step
    check_dot(lambda X: oracle.rhs(c, X), lambda w: oracle.rhs_vjp(c, U, w), U, seed=5, eps=1e-7)


def test_limiter_partials_cover_every_branch():
    """The rough test states visit each branch of MC and superbee (so the
    entry checks above exercise each partial), judged from the forward
    differences of the oracle's own primitives."""
    U = wl.random_state((4, 5, 6), seed=22, vmax=1.5)
    W = oracle.primitives(oracle.make_config((4, 5, 6), (1 / 6, 1 / 5, 1 / 4)), U)
    a = (np.roll(W, -1, axis=3) - W).ravel()
    b = (W - np.roll(W, 1, axis=3)).ravel()
    same = a * b > 0
    aa, ab = np.abs(a[same]), np.abs(b[same])
    cen = 0.5 * (aa + ab)
    mc = [np.sum(cen <= np.minimum(2 * aa, 2 * ab)), np.sum((cen > np.minimum(2 * aa, 2 * ab)) & (aa <= ab)),
          np.sum((cen > np.minimum(2 * aa, 2 * ab)) & (aa > ab))]
    s1, s2 = np.minimum(2 * aa, ab), np.minimum(aa, 2 * ab)
    sb = [np.sum((s1 >= s2) & (2 * aa <= ab)), np.sum((s1 >= s2) & (2 * aa > ab)),
          np.sum((s1 < s2) & (aa <= 2 * ab)), np.sum((s1 < s2) & (aa > 2 * ab))]
    assert min(mc) > 5 and min(sb) > 5, (mc, sb)


def test_rk2_vjp():
    grid = wl.Grid((5, 6, 7), (1 / 7, 1 / 6, 1 / 5))
    U = wl.random_state(grid.shape, seed=6, vmax=0.6)
    c = oracle.make_config(grid.shape, grid.h)
    dt = 0.5 * oracle.cfl_dt(c, U)
    check_dot(lambda X: oracle.rk2(c, X, dt), lambda w: oracle.rk2_vjp(c, U, dt, w), U, seed=7)
    check_entries(lambda X: oracle.rk2(c, X, dt), lambda w: oracle.rk2_vjp(c, U, dt, w), U, seed=8)


@pytest.mark.parametrize("T0", [3.0, 0.02, 0.005])
def test_cool_vjp(T0):
    """Three regimes: stays above Tc, crosses Tc within dt, starts below Tc."""
    grid = wl.cube(4)
    rng = np.random.default_rng(9)
    shape = grid.shape
    rho = rng.uniform(0.5, 1.5, shape)
    v = rng.uniform(-0.5, 0.5, (3,) + shape)
    T = T0 * rng.uniform(0.9, 1.1, shape)
    U = wl.conserved(rho, v[0], v[1], v[2], rho * T, 5 / 3)
    c = oracle.make_config(shape, grid.h, flags=oracle.SRC_COOLING)
    dt = {3.0: 0.2, 0.02: 0.05, 0.005: 0.01}[T0]
    Tn = [oracle.cool_temperature(rho.flat[i], T.flat[i], dt, 5 / 3, 0.3, 1e-2, 1e-3, 1e-4)
          for i in range(rho.size)]
    assert min(Tn) > 2e-4  # away from the floor
    check_dot(lambda X: oracle.cool(c, X, dt), lambda w: oracle.cool_vjp(c, U, dt, w), U, seed=10)
    check_entries(lambda X: oracle.cool(c, X, dt), lambda w: oracle.cool_vjp(c, U, dt, w), U,
                  seed=11)


def test_kick_vjp():
    grid = wl.cube(4)
    U = wl.random_state(grid.shape, seed=12)
    acc = np.random.default_rng(13).standard_normal((3,) + grid.shape)
    c = oracle.make_config(grid.shape, grid.h)
    check_dot(lambda X: oracle.kick(c, X, acc, 0.1), lambda w: oracle.kick_vjp(c, U, acc, 0.1, w)[0],
              U, seed=14)
    # derivative with respect to the acceleration
    w = np.random.default_rng(15).standard_normal(U.shape)
    _, accb = oracle.kick_vjp(c, U, acc, 0.1, w)
    da = np.random.default_rng(16).standard_normal(acc.shape)
    jv = fd_jvp(lambda A: oracle.kick(c, U, A, 0.1), acc, da, 1e-6)
    assert float((w * jv).sum()) == pytest.approx(float((accb * da).sum()), rel=1e-8)


@pytest.mark.parametrize("solver,cycle", [(oracle.GRAV_MG, oracle.MG_V),
                                          (oracle.GRAV_MG, oracle.MG_W),
                                          (oracle.GRAV_FFT, oracle.MG_V)])
def test_gravity_vjp(solver, cycle):
    n = 16
    U = wl.grf_density_state(n, seed=2)
    c = oracle.make_config((n, n, n), (1 / n,) * 3, flags=oracle.SRC_GRAVITY, grav_G=wl.JEANS_G,
                           mg_tol=1e-13, mg_max_cycles=80, grav_solver=solver, mg_cycle=cycle)
    dt = 1e-3
    phi0 = np.zeros((n, n, n))

    def fwd(X):
        acc, _, _ = oracle.gravity_accel(c, X, phi0)
        return oracle.kick(c, X, acc, dt)

    check_dot(fwd, lambda w: oracle.gravity_vjp(c, U, dt, phi0, w), U, seed=17, rtol=1e-6)


@pytest.mark.parametrize("integrator", [oracle.RK_SSP3, oracle.RK_EULER])
def test_other_integrators_vjp(integrator):
    """Reverse of the SSPRK3 and forward-Euler updates (App. A.3)."""
    grid = wl.Grid((5, 6, 7), (1 / 7, 1 / 6, 1 / 5))
    U = wl.random_state(grid.shape, seed=6, vmax=0.6)
    c = oracle.make_config(grid.shape, grid.h, integrator=integrator)
    dt = 0.5 * oracle.cfl_dt(c, U)
    f = lambda X: oracle.integrate(c, X, dt)
    g = lambda w: oracle.integrate_vjp(c, U, dt, w)
    check_dot(f, g, U, seed=27)
    check_entries(f, g, U, seed=28)


@pytest.mark.parametrize("flags,integrator", [(0, oracle.RK_SSP2),
                                              (oracle.SRC_FORCING | oracle.SRC_COOLING, oracle.RK_SSP2),
                                              (oracle.SRC_FORCING | oracle.SRC_COOLING, oracle.RK_SSP3)])
def test_step_vjp_against_full_steps(flags, integrator):
    grid = wl.cube(8)
    U = wl.random_state(grid.shape, seed=18, vmax=0.5)
    c = oracle.make_config(grid.shape, grid.h, flags=flags, integrator=integrator)
    dt = 0.6 * oracle.cfl_dt(c, U)
    nvec = oracle.ou_modes(1.0, 2.0) if flags & oracle.SRC_FORCING else np.zeros((0, 3), np.int32)
    ahat = oracle.ou_init(c, nvec) if flags & oracle.SRC_FORCING else np.zeros(6)
    phi = np.zeros(grid.shape)

    def fwd(X):
        sim = oracle.Simulation(c, X, nvec=nvec, ahat=ahat.copy(), phi=phi.copy())
        sim.step_index = 4
        return sim.advance(1, dt).U

    check_dot(fwd, lambda w: oracle.step_vjp(c, U, dt, 4, nvec, ahat, phi, w), U, seed=19)


def test_step_vjp_fiducial_scheme():
    """The paper's fiducial scheme (van Leer + HLLC, RK2) with forcing and
    cooling, through full steps."""
    grid = wl.cube(8)
    U = wl.random_state(grid.shape, seed=23, vmax=0.5)
    flags = oracle.SRC_FORCING | oracle.SRC_COOLING
    c = oracle.make_config(grid.shape, grid.h, flags=flags, limiter=oracle.LIM_VANLEER)
    dt = 0.6 * oracle.cfl_dt(c, U)
    nvec = oracle.ou_modes(1.0, 2.0)
    ahat = oracle.ou_init(c, nvec)
    phi = np.zeros(grid.shape)

    def fwd(X):
        sim = oracle.Simulation(c, X, nvec=nvec, ahat=ahat.copy(), phi=phi.copy())
        sim.step_index = 2
        return sim.advance(1, dt).U

    check_dot(fwd, lambda w: oracle.step_vjp(c, U, dt, 2, nvec, ahat, phi, w), U, seed=24,
              eps=1e-7)


@pytest.mark.parametrize("solver", [oracle.GRAV_MG, oracle.GRAV_FFT])
def test_step_vjp_gravity(solver):
    n = 8
    U = wl.grf_density_state(n, seed=3)
    c = oracle.make_config((n, n, n), (1 / n,) * 3,
                           flags=oracle.SRC_GRAVITY | oracle.SRC_COOLING, grav_G=wl.JEANS_G,
                           mg_tol=1e-13, mg_max_cycles=80, grav_solver=solver)
    dt = 0.5 * oracle.cfl_dt(c, U)
    phi = np.zeros((n, n, n))

    def fwd(X):
        return oracle.Simulation(c, X, phi=phi.copy()).advance(1, dt).U

    nv = np.zeros((0, 3), np.int32)
    # perturb the density only: the state is at rest with uniform pressure, so
    # velocity and pressure slopes sit exactly on the minmod kink at 0; density
    # perturbations leave them there in both difference runs
    check_dot(fwd, lambda w: oracle.step_vjp(c, U, dt, 0, nv, np.zeros(6), phi, w), U, seed=20,
              rtol=1e-6, fields=[0])


# ---------------------------------------------------------------- flux correction (Sec. 8)

@pytest.mark.parametrize("name,grid", GRIDS)
def test_flux_correction_enters_as_a_face_flux(name, grid):
    """L(U) with a correction field B equals L(U) plus the difference of B
    over each cell's faces: -sum_a (B_i - B_{i-e_a}) / h_a with the face
    below the first cell taking B of its mapped cell (periodic wrap, or the
    cell itself with outflow); a uniform B changes nothing with periodic
    boundaries."""
    rng = np.random.default_rng(40)
    U = wl.random_state(grid.shape, seed=41, vmax=0.5)
    B = rng.standard_normal((5,) + grid.shape)
    c0 = oracle.make_config(grid.shape, grid.h, grid.bc)
    c1 = oracle.make_config(grid.shape, grid.h, grid.bc, flux_corr=B)
    d = oracle.rhs(c1, U) - oracle.rhs(c0, U)
    want = np.zeros_like(B)
    for a, axis in enumerate((3, 2, 1)):  # x, y, z axes of the [5][z][y][x] arrays
        lower = np.roll(B, 1, axis=axis)
        if grid.bc[a] == 1:  # outflow: the face below cell 0 carries B of cell 0
            sl = [slice(None)] * 4
            sl[axis] = 0
            lower[tuple(sl)] = B[tuple(sl)]
        want -= (B - lower) / grid.h[a]
    assert np.abs(d - want).max() < 1e-12 * np.abs(want).max()
    if all(b == 0 for b in grid.bc):
        cu = oracle.make_config(grid.shape, grid.h, grid.bc,
                                flux_corr=np.ones((5,) + grid.shape) * rng.standard_normal((5, 1, 1, 1)))
        assert np.abs(oracle.rhs(cu, U) - oracle.rhs(c0, U)).max() < 1e-12


@pytest.mark.parametrize("integrator", [oracle.RK_SSP2, oracle.RK_SSP3, oracle.RK_EULER])
def test_flux_correction_adjoint(integrator):
    """The adjoint of the flux-correction field through a full step (with
    forcing and cooling) against central differences of the step in B."""
    grid = wl.Grid((5, 6, 7), (1 / 7, 1 / 6, 1 / 5), (1, 0, 0))
    U = wl.random_state(grid.shape, seed=42, vmax=0.5)
    rng = np.random.default_rng(43)
    B = 0.05 * rng.standard_normal((5,) + grid.shape)
    flags = oracle.SRC_FORCING | oracle.SRC_COOLING
    c = oracle.make_config(grid.shape, grid.h, grid.bc, flags=flags, integrator=integrator,
                           flux_corr=B)
    dt = 0.4 * oracle.cfl_dt(c, U)
    nvec = oracle.ou_modes(1.0, 2.0)
    ahat = oracle.ou_init(c, nvec)
    phi = np.zeros(grid.shape)
    w = rng.standard_normal(U.shape)
    _, g = oracle.step_vjp_flux(c, U, dt, 1, nvec, ahat, phi, w)

    def fwd(Bx):
        cx = oracle.make_config(grid.shape, grid.h, grid.bc, flags=flags, integrator=integrator,
                                flux_corr=Bx)
        sim = oracle.Simulation(cx, U, nvec=nvec, ahat=ahat.copy(), phi=phi.copy())
        sim.step_index = 1
        return sim.advance(1, dt).U

    for trial in range(3):
        v = rng.standard_normal(B.shape) * 0.05
        eps = 1e-6
        jv = (fwd(B + eps * v) - fwd(B - eps * v)) / (2 * eps)
        assert float((w * jv).sum()) == pytest.approx(float((g * v).sum()), rel=2e-7)


@pytest.mark.parametrize("integ", [oracle.COOLINT_TRAPEZOID, oracle.COOLINT_SUBCYCLE])
def test_tabulated_cooling_step_vjp(integ):
    """Full steps with forcing and the tabulated cooling model (Sec. 4)."""
    grid = wl.cube(8)
    U = wl.random_state(grid.shape, seed=44, vmax=0.4, rho=(0.5, 2.0), p=(0.002, 1.0))
    c = oracle.make_config(grid.shape, grid.h, flags=oracle.SRC_FORCING | oracle.SRC_COOLING,
                           cool_model=oracle.COOL_TABLE, cool_table=wl.synthetic_cie_table(),
                           cool_integrator=integ, cool_frac=0.05, cool_nsub_max=50,
                           **wl.COOLING_TABLE_MODEL)
    dt = 0.5 * oracle.cfl_dt(c, U)
    nvec = oracle.ou_modes(1.0, 2.0)
    ahat = oracle.ou_init(c, nvec)
    phi = np.zeros(grid.shape)

    def fwd(X):
        sim = oracle.Simulation(c, X, nvec=nvec, ahat=ahat.copy(), phi=phi.copy())
        sim.step_index = 3
        return sim.advance(1, dt).U

    check_dot(fwd, lambda w: oracle.step_vjp(c, U, dt, 3, nvec, ahat, phi, w), U, seed=45,
              eps=1e-7, rtol=1e-6)
