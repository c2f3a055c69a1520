"""GPU parity: the HIP library (through its C ABI) against the FP64 oracle on
the same seeded inputs.  Tolerances (relative field norm of parity.rel_err):
1e-12 for fp64, 1e-5 for fp32.  Sizes span several 64 x 8 tiles with ragged
edges; the full workload sizes are checked on sampled cells."""
import math

import numpy as np
import pytest

import oracle
import paper_2512_13403_amd as mh
import workloads as wl
from parity import TOL, as_input, oracle_step_sampled, pair, rel_err

pytestmark = pytest.mark.gpu


@pytest.fixture(autouse=True)
def _name(request):
    print(f"\n[gpu case] {request.node.nodeid}", flush=True)
    yield


def run_both(shape, h, U0, dtype, nsteps, dt=None, bc=(0, 0, 0), **kw):
    s, oc = pair(shape, h, bc, dtype, **kw)
    Uin = as_input(U0, dtype)
    if dt is None:
        dt = 0.8 * oracle.cfl_dt(oc, Uin)
    s.set_state(Uin)
    s.step(nsteps, dt)
    sim = oracle.Simulation(oc, Uin).advance(nsteps, dt)
    return s, sim


# ---------------------------------------------------------------- hydro

@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("nsteps", [1, 10])
def test_random_state_ragged_periodic(dtype, nsteps):
    shape = (19, 21, 77)  # (nz, ny, nx): x spans 2 tiles, y 3, both ragged
    h = (1 / 77, 1 / 21, 1 / 19)
    U0 = wl.random_state(shape, seed=1, vmax=0.6)
    s, sim = run_both(shape, h, U0, dtype, nsteps)
    assert rel_err(s.get_state(), sim.U) < TOL[dtype]


SCHEMES = [(oracle.LIM_VANLEER, oracle.RS_HLLC), (oracle.LIM_MC, oracle.RS_HLLC),
           (oracle.LIM_SUPERBEE, oracle.RS_HLLC), (oracle.LIM_MINMOD, oracle.RS_HLL),
           (oracle.LIM_MINMOD, oracle.RS_RUSANOV), (oracle.LIM_VANLEER, oracle.RS_HLL),
           (oracle.LIM_NONE, oracle.RS_RUSANOV)]


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("limiter,riemann", SCHEMES)
def test_scheme_variants_ragged(dtype, limiter, riemann):
    """The other limiters and Riemann solvers of App. A.1/A.2 (run-time scheme
    kernel) against the oracle, 3 steps on a ragged grid with outflow in x."""
    shape = (9, 11, 70)
    h = (1 / 70, 1 / 11, 1 / 9)
    U0 = wl.random_state(shape, seed=8, vmax=0.6)
    s, sim = run_both(shape, h, U0, dtype, 3, bc=(1, 0, 0), limiter=limiter, riemann=riemann)
    assert rel_err(s.get_state(), sim.U) < TOL[dtype]


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_scheme_variant_with_sources(dtype):
    shape = (12, 14, 66)
    h = (1 / 66, 1 / 14, 1 / 12)
    U0 = wl.random_state(shape, seed=9, vmax=0.5)
    s, sim = run_both(shape, h, U0, dtype, 2, limiter=oracle.LIM_VANLEER, riemann=oracle.RS_HLL,
                      flags=oracle.SRC_FORCING | oracle.SRC_COOLING, ou_seed=3)
    assert rel_err(s.get_state(), sim.U) < TOL[dtype]


@pytest.mark.parametrize("limiter,riemann", [(oracle.LIM_VANLEER, oracle.RS_HLLC),
                                             (oracle.LIM_MC, oracle.RS_HLL)])
def test_sod_full_run_scheme_variants_fp64(limiter, riemann):
    grid = wl.sod_grid(128, 16, 16)
    U0 = wl.sod_state(grid)
    s, oc = pair(grid.shape, grid.h, grid.bc, "f64", gamma=1.4, limiter=limiter, riemann=riemann)
    s.set_state(U0)
    dts = s.run_to(0.2)
    sim = oracle.Simulation(oc, U0)
    assert len(dts) == sim.run_to(0.2)
    U = s.get_state()
    assert rel_err(U, sim.U) < 1e-12
    assert np.array_equal(U, np.broadcast_to(U[:, :1, :1, :], U.shape))


INTEGRATORS = [oracle.RK_SSP3, oracle.RK_EULER]


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("integrator", INTEGRATORS)
def test_other_integrators_ragged(dtype, integrator):
    """SSPRK3 (stage kernel with an inner stage) and forward Euler (a lone
    final stage) of App. A.3 against the oracle, 5 steps on a ragged grid."""
    shape = (19, 21, 77)
    h = (1 / 77, 1 / 21, 1 / 19)
    U0 = wl.random_state(shape, seed=2, vmax=0.6)
    s, sim = run_both(shape, h, U0, dtype, 5, integrator=integrator)
    assert rel_err(s.get_state(), sim.U) < TOL[dtype]


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("integrator", INTEGRATORS)
def test_other_integrators_with_sources_and_variant(dtype, integrator):
    """The run-time-scheme kernel (van Leer + HLL) with forcing and cooling."""
    shape = (12, 14, 66)
    h = (1 / 66, 1 / 14, 1 / 12)
    U0 = wl.random_state(shape, seed=10, vmax=0.5)
    s, sim = run_both(shape, h, U0, dtype, 3, limiter=oracle.LIM_VANLEER, riemann=oracle.RS_HLL,
                      flags=oracle.SRC_FORCING | oracle.SRC_COOLING, ou_seed=5,
                      integrator=integrator)
    assert rel_err(s.get_state(), sim.U) < TOL[dtype]


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_ssprk3_gravity_cooling(dtype):
    n = 32
    U0 = wl.grf_density_state(n, seed=1)
    s, sim = run_both((n, n, n), (1 / n,) * 3, U0, dtype, 3,
                      flags=oracle.SRC_GRAVITY | oracle.SRC_COOLING, grav_G=wl.JEANS_G,
                      mg_tol=0.0, mg_max_cycles=3, integrator=oracle.RK_SSP3)
    assert rel_err(s.get_state(), sim.U) < TOL[dtype]


def test_sod_full_run_ssprk3_fp64():
    grid = wl.sod_grid(128, 16, 16)
    U0 = wl.sod_state(grid)
    s, oc = pair(grid.shape, grid.h, grid.bc, "f64", gamma=1.4, integrator=oracle.RK_SSP3)
    s.set_state(U0)
    dts = s.run_to(0.2)
    sim = oracle.Simulation(oc, U0)
    assert len(dts) == sim.run_to(0.2)
    U = s.get_state()
    assert rel_err(U, sim.U) < 1e-12
    assert np.array_equal(U, np.broadcast_to(U[:, :1, :1, :], U.shape))


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("bc", [(1, 1, 1), (1, 0, 0), (0, 1, 0), (0, 0, 1)])
def test_outflow_boundaries(dtype, bc):
    shape = (12, 10, 70)
    h = (1 / 70, 1 / 10, 1 / 12)
    U0 = wl.random_state(shape, seed=2, vmax=0.8)
    s, sim = run_both(shape, h, U0, dtype, 3, bc=bc)
    assert rel_err(s.get_state(), sim.U) < TOL[dtype]


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_first_order_reconstruction(dtype):
    shape = (9, 17, 33)
    U0 = wl.random_state(shape, seed=3)
    s, sim = run_both(shape, (1 / 33, 1 / 17, 1 / 9), U0, dtype, 4, limiter=oracle.LIM_NONE)
    assert rel_err(s.get_state(), sim.U) < TOL[dtype]


def test_cfl_steps_fp64_match_dt_sequence():
    shape = (16, 24, 40)
    h = (1 / 40, 1 / 24, 1 / 16)
    U0 = wl.smooth_random_state(shape, seed=4)
    s, oc = pair(shape, h, dtype="f64")
    s.set_state(U0)
    dts = s.step(10, 0.0, record=True)
    sim = oracle.Simulation(oc, U0).advance(10, 0.0)
    assert np.allclose(dts, sim.dts, rtol=1e-13, atol=0)
    assert rel_err(s.get_state(), sim.U) < 1e-12
    t, step = s.clock()
    assert step == 10 and t == pytest.approx(sum(sim.dts), rel=1e-14)


def test_cfl_dt_fp32_close_to_oracle():
    shape = (16, 16, 64)
    U0 = as_input(wl.smooth_random_state(shape, seed=5), "f32")
    s, oc = pair(shape, (1 / 64, 1 / 16, 1 / 16), dtype="f32")
    s.set_state(U0)
    dts = s.step(1, 0.0, record=True)
    assert dts[0] == pytest.approx(oracle.cfl_dt(oc, U0), rel=1e-6)


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_uniform_state_is_bitwise_fixed_point(dtype):
    shape = (8, 9, 70)
    U0 = as_input(wl.rest_state(shape, rho=1.3, p=0.9, v=(0.3, -0.2, 0.5)), dtype)
    s, _ = pair(shape, (0.1, 0.1, 0.1), dtype=dtype)
    s.set_state(U0)
    s.step(5, 0.01)
    assert np.array_equal(s.get_state().astype(np.float64), U0)


@pytest.mark.parametrize("dtype,tol", [("f64", 1e-13), ("f32", 1e-6)])
def test_conservation_periodic(dtype, tol):
    shape = (24, 20, 66)
    U0 = as_input(wl.random_state(shape, seed=6, vmax=0.5), dtype)
    s, oc = pair(shape, (1 / 66, 1 / 20, 1 / 24), dtype=dtype)
    s.set_state(U0)
    s.step(10, 0.0)
    U = s.get_state().astype(np.float64)
    for f in range(5):
        s0, s1 = math.fsum(U0[f].ravel()), math.fsum(U[f].ravel())
        assert abs(s1 - s0) / math.fsum(np.abs(U0[f]).ravel()) < tol, f


def test_sod_full_run_fp64():
    grid = wl.sod_grid(128, 16, 16)
    U0 = wl.sod_state(grid)
    s, oc = pair(grid.shape, grid.h, grid.bc, "f64", gamma=1.4)
    s.set_state(U0)
    dts = s.run_to(0.2)
    sim = oracle.Simulation(oc, U0)
    n = sim.run_to(0.2)
    assert len(dts) == n
    assert np.allclose(dts, sim.dts, rtol=1e-12, atol=1e-16)
    U = s.get_state()
    assert rel_err(U, sim.U) < 1e-12
    # transverse invariance on the GPU: all pencils bitwise identical, m_y = m_z = 0
    assert np.array_equal(U, np.broadcast_to(U[:, :1, :1, :], U.shape))
    assert np.all(U[2] == 0.0) and np.all(U[3] == 0.0)
    t, _ = s.clock()
    assert t == pytest.approx(0.2, abs=1e-15)


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("nsteps", [1, 10])
def test_kelvin_helmholtz_64(dtype, nsteps):
    n = 64
    U0 = as_input(wl.kh_state(n, seed=0), dtype)
    s, oc = pair((n, n, n), (1 / n,) * 3, dtype=dtype)
    # fp64 runs the device CFL step on both sides; an fp32 CFL step differs
    # from the oracle's in its last bits, so fp32 replays the oracle's dt
    dt = 0.0 if dtype == "f64" else oracle.cfl_dt(oc, U0)
    s.set_state(U0)
    s.step(nsteps, dt)
    sim = oracle.Simulation(oc, U0).advance(nsteps, dt)
    assert rel_err(s.get_state(), sim.U) < TOL[dtype]


def test_deterministic_repeat():
    shape = (20, 20, 70)
    U0 = wl.random_state(shape, seed=8)
    outs = []
    for _ in range(2):
        s, _ = pair(shape, (1 / 70, 1 / 20, 1 / 20), dtype="f32")
        s.set_state(U0)
        s.step(5, 0.0)
        outs.append(s.get_state())
    assert np.array_equal(outs[0], outs[1])


@pytest.mark.parametrize("shape", [(1, 1, 64), (1, 64, 1), (64, 1, 1), (1, 1, 1), (3, 2, 5)])
def test_degenerate_shapes(shape):
    h = tuple(1.0 / max(n, 1) for n in shape[::-1])
    U0 = wl.random_state(shape, seed=9, vmax=0.5)
    s, sim = run_both(shape, h, U0, "f64", 3)
    assert rel_err(s.get_state(), sim.U) < 1e-12


def test_zero_steps_and_t_stop_cap():
    shape = (8, 8, 64)
    U0 = wl.smooth_random_state(shape, seed=10)
    s, oc = pair(shape, (1 / 64, 1 / 8, 1 / 8), dtype="f64")
    s.set_state(U0)
    s.step(0, 0.0)
    assert np.array_equal(s.get_state(), U0)
    dts = s.step(3, 1.0, t_stop=0.004, record=True)
    assert dts[0] == pytest.approx(0.004) and dts[1] == 0.0 and dts[2] == 0.0
    sim = oracle.Simulation(oc, U0).advance(1, 0.004)
    assert rel_err(s.get_state(), sim.U) < 1e-12


def test_health_check_flags_negative_pressure():
    shape = (8, 8, 64)
    U0 = wl.smooth_random_state(shape, seed=11)
    U0[4, 3, 2, 10] = 0.1 * U0[4, 3, 2, 10] - 5.0  # E below kinetic energy: P < 0
    s, _ = pair(shape, (1 / 64, 1 / 8, 1 / 8), dtype="f64")
    s.set_state(U0)
    s.step(1, 1e-4)
    bad, first = s.check()
    assert bad >= 1 and 0 <= first < 8 * 8 * 64
    s.set_state(wl.smooth_random_state(shape, seed=11))
    s.step(1, 1e-4)
    assert s.check() == (0, -1)


# ---------------------------------------------------------------- sources

SRC = {
    "cool": oracle.SRC_COOLING,
    "force": oracle.SRC_FORCING,
    "force+cool": oracle.SRC_FORCING | oracle.SRC_COOLING,
}


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("src", list(SRC))
@pytest.mark.parametrize("nsteps", [1, 10])
def test_sources(dtype, src, nsteps):
    shape = (12, 14, 66)
    h = (1 / 66, 1 / 14, 1 / 12)
    U0 = wl.smooth_random_state(shape, seed=12)
    s, sim = run_both(shape, h, U0, dtype, nsteps, flags=SRC[src], ou_seed=7)
    assert rel_err(s.get_state(), sim.U) < TOL[dtype]
    if "force" in src:
        assert np.allclose(s.ou_state(), sim.ahat, rtol=0, atol=1e-13 * np.abs(sim.ahat).max())


def test_ou_update_every_four_steps():
    shape = (8, 8, 64)
    U0 = wl.smooth_random_state(shape, seed=13)
    s, sim = run_both(shape, (1 / 64, 1 / 8, 1 / 8), U0, "f64", 9, flags=oracle.SRC_FORCING,
                      ou_every=4)
    assert rel_err(s.get_state(), sim.U) < 1e-12
    assert np.allclose(s.ou_state(), sim.ahat, rtol=0, atol=1e-13 * np.abs(sim.ahat).max())


def test_ou_resume_from_saved_state():
    shape = (8, 8, 64)
    U0 = wl.smooth_random_state(shape, seed=14)
    s, oc = pair(shape, (1 / 64, 1 / 8, 1 / 8), dtype="f64", flags=oracle.SRC_FORCING)
    s.set_state(U0)
    s.step(3, 1e-3)
    U3, a3, (t3, k3) = s.get_state(), s.ou_state(), s.clock()
    s.step(2, 1e-3)
    ref = s.get_state()
    s2, _ = pair(shape, (1 / 64, 1 / 8, 1 / 8), dtype="f64", flags=oracle.SRC_FORCING)
    s2.set_state(U3)
    s2.set_ou_state(a3)
    s2.set_clock(t3, k3)
    s2.step(2, 1e-3)
    assert np.array_equal(s2.get_state(), ref)


# ---------------------------------------------------------------- gravity

@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("cool", [False, True])
def test_gravity_fixed_cycles(dtype, cool):
    n = 32
    U0 = wl.grf_density_state(n, seed=0)
    flags = oracle.SRC_GRAVITY | (oracle.SRC_COOLING if cool else 0)
    s, sim = run_both((n, n, n), (1 / n,) * 3, U0, dtype, 3, flags=flags, grav_G=wl.JEANS_G,
                      mg_tol=0.0, mg_max_cycles=3)
    assert s.mg_cycles() == 3
    assert rel_err(s.get_state(), sim.U) < TOL[dtype]
    phi = s.potential().astype(np.float64)
    assert np.abs(phi - sim.phi).max() < 10 * TOL[dtype] * np.abs(sim.phi).max()


MG_VARIANTS = [(oracle.MG_W, oracle.SMOOTH_JACOBI), (oracle.MG_V, oracle.SMOOTH_JACOBI),
               (oracle.MG_W, oracle.SMOOTH_RBGS)]


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("cycle,smoother", MG_VARIANTS)
def test_gravity_cycle_and_smoother_variants(dtype, cycle, smoother):
    """W-cycle and red-black Gauss-Seidel (App. C, Sec. 6.2.1) at 32^3: the
    single-workgroup tail runs the W recursion and is launched twice."""
    n = 32
    U0 = wl.grf_density_state(n, seed=2)
    s, sim = run_both((n, n, n), (1 / n,) * 3, U0, dtype, 3,
                      flags=oracle.SRC_GRAVITY | oracle.SRC_COOLING, grav_G=wl.JEANS_G,
                      mg_tol=0.0, mg_max_cycles=3, mg_cycle=cycle, mg_smoother=smoother)
    assert s.mg_cycles() == 3
    assert rel_err(s.get_state(), sim.U) < TOL[dtype]
    phi = s.potential().astype(np.float64)
    assert np.abs(phi - sim.phi).max() < 10 * TOL[dtype] * np.abs(sim.phi).max()


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_gravity_wcycle_host_levels_64(dtype):
    """64^3: two host-launched levels recurse (W) above the tail."""
    n = 64
    U0 = wl.grf_density_state(n, seed=3)
    s, sim = run_both((n, n, n), (1 / n,) * 3, U0, dtype, 2, flags=oracle.SRC_GRAVITY,
                      grav_G=wl.JEANS_G, mg_tol=0.0, mg_max_cycles=2, mg_cycle=oracle.MG_W,
                      mg_smoother=oracle.SMOOTH_RBGS)
    assert rel_err(s.get_state(), sim.U) < TOL[dtype]
    phi = s.potential().astype(np.float64)
    assert np.abs(phi - sim.phi).max() < 10 * TOL[dtype] * np.abs(sim.phi).max()


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_gravity_non_power_of_two_levels(dtype):
    """48^3: host-launched levels 48 and 24 (colour passes with 24 and 12
    cells of a colour per row), the single-workgroup tail from 12^3 down to
    an odd 3^3 coarsest grid (the one-wave sweeps), red-black V-cycles."""
    n = 48
    U0 = wl.grf_density_state(n, seed=4)
    s, sim = run_both((n, n, n), (1 / n,) * 3, U0, dtype, 2,
                      flags=oracle.SRC_GRAVITY | oracle.SRC_COOLING, grav_G=wl.JEANS_G,
                      mg_tol=0.0, mg_max_cycles=3)
    assert s.mg_cycles() == 3
    assert rel_err(s.get_state(), sim.U) < TOL[dtype]
    phi = s.potential().astype(np.float64)
    assert np.abs(phi - sim.phi).max() < 10 * TOL[dtype] * np.abs(sim.phi).max()


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("n", [16, 32])
def test_gravity_spectral_solver(dtype, n):
    """The spectral Poisson solve and gradient of Sec. 6.1 (own FFT kernels)
    against the oracle's DFT-based version, with cooling, 3 steps."""
    U0 = wl.grf_density_state(n, seed=4)
    U0[1:4] += 0.05 * np.random.default_rng(5).standard_normal((3, n, n, n)) * U0[0]
    s, sim = run_both((n, n, n), (1 / n,) * 3, U0, dtype, 3,
                      flags=oracle.SRC_GRAVITY | oracle.SRC_COOLING, grav_G=wl.JEANS_G,
                      grav_solver=oracle.GRAV_FFT)
    assert s.mg_cycles() == 0
    assert rel_err(s.get_state(), sim.U) < TOL[dtype]
    phi = s.potential().astype(np.float64)
    assert np.abs(phi - sim.phi).max() < 10 * TOL[dtype] * np.abs(sim.phi).max()


def test_gravity_spectral_single_mode_closed_form():
    """One density mode: the GPU potential and the resulting momentum kick are
    the closed forms -4 pi G A cos/|k|^2 and rho a dt (fp64)."""
    n, L = 32, 1.0
    h = L / n
    G, A, dt = 1.3, 0.05, 1e-4
    m = (1, 2, 3)
    z, y, x = np.meshgrid(*((np.arange(n) + 0.5) * h,) * 3, indexing="ij")
    kap = [2 * np.pi * mi / L for mi in m]
    th = kap[0] * x + kap[1] * y + kap[2] * z
    rho = 1.0 + A * np.cos(th)
    o = np.zeros_like(rho)
    U0 = wl.conserved(rho, o, o, o, np.ones_like(rho), 5.0 / 3.0)
    s, _ = pair((n, n, n), (h,) * 3, dtype="f64", flags=oracle.SRC_GRAVITY, grav_G=G,
                grav_solver=oracle.GRAV_FFT)
    s.set_state(U0)
    s.step(1, dt)
    k2 = sum(k * k for k in kap)
    phi = s.potential()
    # at rest with uniform pressure the hydro update leaves the density
    # unchanged up to rounding, so the potential is that of the initial mode
    amp = 4 * np.pi * G * A / k2
    assert np.abs(phi + amp * np.cos(th)).max() < 1e-9 * amp
    # the kick: m = rho a dt with a = -grad Phi = -amp kappa sin(th)
    U = s.get_state()
    for a in range(3):
        want = rho * (-amp * kap[a] * np.sin(th)) * dt
        assert np.abs(U[1 + a] - want).max() < 1e-9 * np.abs(want).max(), a


@pytest.mark.parametrize("solver", [oracle.GRAV_MG, oracle.GRAV_FFT])
def test_gravity_cfl_steps_match_oracle(solver):
    """CFL steps with gravity and cooling: the next step's dt comes from the
    state after all sources (the last stage skips its own CFL reduction when
    a sources kernel follows), so the dt sequence is the oracle's."""
    n = 16
    U0 = wl.grf_density_state(n, seed=8)
    U0[1:4] += 0.2 * np.random.default_rng(9).standard_normal((3, n, n, n)) * U0[0]
    s, oc = pair((n, n, n), (1 / n,) * 3, dtype="f64",
                 flags=oracle.SRC_GRAVITY | oracle.SRC_COOLING, grav_G=wl.JEANS_G, mg_tol=1e-12,
                 mg_max_cycles=60, grav_solver=solver)
    s.set_state(U0)
    dts = s.step(4, 0.0, record=True)
    sim = oracle.Simulation(oc, U0).advance(4)
    assert np.allclose(dts, sim.dts, rtol=1e-12, atol=0.0), (dts, sim.dts)
    assert rel_err(s.get_state(), sim.U) < 1e-11


TABLE_MODEL = dict(cool_model=oracle.COOL_TABLE, cool_table=wl.synthetic_cie_table(),
                   **wl.COOLING_TABLE_MODEL)


def _multiphase_state(shape, seed):
    """Random state whose temperatures T = P/rho span 1e-3 .. 1, across the
    heating branch, tc = 1e-2 and the table."""
    U = wl.random_state(shape, seed=seed, vmax=0.4, rho=(0.5, 2.0), p=(0.002, 1.0))
    return U


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("integ", [oracle.COOLINT_TRAPEZOID, oracle.COOLINT_SUBCYCLE,
                                   oracle.COOLINT_AUTO])
def test_tabulated_cooling(dtype, integ):
    """The paper's cooling model (Sec. 4.1-4.3) as the step's last kernel,
    with forcing, against the oracle."""
    shape = (12, 14, 66)
    h = (1 / 66, 1 / 14, 1 / 12)
    U0 = _multiphase_state(shape, 21)
    s, sim = run_both(shape, h, U0, dtype, 3, flags=oracle.SRC_FORCING | oracle.SRC_COOLING,
                      ou_seed=2, cool_integrator=integ, cool_frac=0.05, cool_nsub_max=200,
                      **TABLE_MODEL)
    assert rel_err(s.get_state(), sim.U) < TOL[dtype]


@pytest.mark.parametrize("solver", [oracle.GRAV_MG, oracle.GRAV_FFT])
def test_tabulated_cooling_with_gravity_and_cfl_limit(solver):
    """CFL steps limited by c_cool min t_cool, with gravity: the dt sequence
    and the state follow the oracle (fp64)."""
    n = 16
    U0 = _multiphase_state((n, n, n), 22)
    s, oc = pair((n, n, n), (1 / n,) * 3, dtype="f64",
                 flags=oracle.SRC_GRAVITY | oracle.SRC_COOLING, grav_G=wl.JEANS_G, mg_tol=1e-12,
                 mg_max_cycles=60, grav_solver=solver, cool_ccool=0.3,
                 cool_integrator=oracle.COOLINT_AUTO, **TABLE_MODEL)
    s.set_state(U0)
    dts = s.step(4, 0.0, record=True)
    sim = oracle.Simulation(oc, U0).advance(4)
    assert np.allclose(dts, sim.dts, rtol=1e-12, atol=0.0), (dts, sim.dts)
    # the cooling limit is the binding one here
    assert dts[0] < 0.99 * oracle.cfl_dt(oracle.make_config((n, n, n), (1 / n,) * 3), U0)
    assert rel_err(s.get_state(), sim.U) < 1e-11


def test_gravity_tolerance_cycle_counts():
    n = 32
    U0 = wl.grf_density_state(n, seed=1)
    s, oc = pair((n, n, n), (1 / n,) * 3, dtype="f64", flags=oracle.SRC_GRAVITY,
                 grav_G=wl.JEANS_G, mg_tol=1e-9, mg_max_cycles=30)
    s.set_state(U0)
    sim = oracle.Simulation(oc, U0)
    for _ in range(3):
        s.step(1, 2e-3)
        sim.advance(1, 2e-3)
        assert s.mg_cycles() == sim.mg_cycles[-1]
    assert rel_err(s.get_state(), sim.U) < 1e-12


# ---------------------------------------------------------------- full sizes, sampled

def _sample_cells(shape, count, seed):
    rng = np.random.default_rng(seed)
    nz, ny, nx = shape
    cells = [(0, 0, 0), (nx - 1, ny - 1, nz - 1)]
    cells += [tuple(int(v) for v in (rng.integers(nx), rng.integers(ny), rng.integers(nz)))
              for _ in range(count - 2)]
    return cells


@pytest.mark.parametrize("dtype", ["f32", "f64"])
def test_kelvin_helmholtz_256_sampled(dtype):
    n = 256
    U0 = as_input(wl.kh_state(n, seed=0), dtype)
    s, oc = pair((n, n, n), (1 / n,) * 3, dtype=dtype)
    dt = oracle.cfl_dt(oc, U0)
    s.set_state(U0)
    s.step(1, dt)
    U = s.get_state()
    cells = _sample_cells(U0.shape[1:], 48, 0)
    ref = oracle_step_sampled(oc, U0, cells, dt)
    got = np.array([[U[f, k, j, i] for (i, j, k) in cells] for f in range(5)], dtype=np.float64)
    assert rel_err(got, ref) < TOL[dtype]


def test_driven_turbulence_512_sampled_fp32():
    """The benchmarked configuration: 512^3, fp32, forcing + cooling, on a
    rough random state so every branch occurs; one CFL step."""
    n = 512
    shape = (n, n, n)
    U0 = as_input(wl.random_state(shape, seed=3, vmax=0.7), "f32")
    flags = oracle.SRC_FORCING | oracle.SRC_COOLING
    s, oc = pair(shape, (1 / n,) * 3, dtype="f32", flags=flags)
    dt = oracle.cfl_dt(oc, U0)
    s.set_state(U0)
    s.step(1, dt)
    U = s.get_state()
    nvec = oracle.ou_modes(1.0, 2.0)
    ahat = oracle.ou_advance(oc, nvec, oracle.ou_init(oc, nvec), 0, dt)
    cells = _sample_cells(shape, 48, 1)
    ref = oracle_step_sampled(oc, U0, cells, dt, ahat=ahat, nvec=nvec)
    got = np.array([[U[f, k, j, i] for (i, j, k) in cells] for f in range(5)], dtype=np.float64)
    assert rel_err(got, ref) < TOL["f32"]


def _cfl_speed(U, gamma, h):
    """max over cells of max_a (|v_a| + c_s) / h_a, from the state in float64"""
    rho = U[0].astype(np.float64)
    v = U[1:4].astype(np.float64) / rho
    p = (gamma - 1.0) * (U[4].astype(np.float64) - 0.5 * rho * (v * v).sum(axis=0))
    cs = np.sqrt(gamma * p / rho)
    return max(((np.abs(v[a]) + cs) / h).max() for a in range(3))


@pytest.mark.parametrize("kind", ["fft", "mg", "table"])
def test_clock_reductions_over_many_cells(kind):
    """The sources kernels that end a step reduce the CFL speed and the health
    counts over a capped, grid-stride grid (several cells per thread above 2^20
    cells): at 128^3 the next step's dt is the CFL dt of the returned state,
    and planted non-finite cells are counted exactly, with the smallest flat
    index."""
    n, gamma, cfl = 128, 5.0 / 3.0, 0.4
    if kind == "table":
        U0 = as_input(_multiphase_state((n, n, n), 31), "f32")
        phys = mh.physics_desc(flags=mh.SRC_COOLING, cool_model=mh.COOL_TABLE,
                               cool_integrator=mh.COOLINT_TRAPEZOID,
                               cool_table=wl.synthetic_cie_table(), **wl.COOLING_TABLE_MODEL)
    else:
        U0 = as_input(wl.grf_density_state(n, seed=12), "f32")
        U0[1:4] += 0.2 * np.random.default_rng(13).standard_normal((3, n, n, n)) * U0[0]
        U0 = as_input(U0, "f32")
        phys = mh.physics_desc(flags=mh.SRC_GRAVITY | mh.SRC_COOLING, grav_G=wl.JEANS_G,
                               mg_tol=1e-5,
                               grav_solver=mh.GRAV_FFT if kind == "fft" else mh.GRAV_MG)
    s = mh.Solver(mh.grid_desc((n, n, n), (1.0 / n,) * 3, dtype="f32", gamma=gamma, cfl=cfl),
                  phys)
    s.set_state(U0)
    s.step(1, 0.0)
    U1 = s.get_state()
    dt2 = s.step(1, 0.0, record=True)[0]
    assert dt2 == pytest.approx(cfl / _cfl_speed(U1, gamma, 1.0 / n), rel=1e-5)
    # non-finite cells late in the flat order: the kernel's count and first
    # index against the returned state
    Ub = U0.copy()
    N = n ** 3
    for q in (N - 70000, N - 3 * n * n - 5, N - 9):
        Ub.reshape(5, -1)[0, q] = np.nan
    s.set_state(Ub)
    s.step(1, 0.5 * dt2)
    bad, first = s.check()
    U = s.get_state().astype(np.float64)
    with np.errstate(invalid="ignore", divide="ignore"):
        p = (gamma - 1.0) * (U[4] - 0.5 * (U[1:4] ** 2).sum(axis=0) / U[0])
        ok = (U[0] > 0) & (p > 0) & np.isfinite(U).all(axis=0)
    want = np.flatnonzero(~ok.reshape(-1))
    assert want.size > 0 and bad == want.size and first == want[0], (bad, first, want.size, want[:3])
