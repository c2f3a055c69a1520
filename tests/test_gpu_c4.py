"""The adjoint inverse problem of the self-gravitating cooling box (Sec. 2.3
checkpointed reverse mode, Sec. 6.2.4 multigrid adjoint, Sec. 7 initial-
condition inversion) as configured: initial density 1 + 0.1 g with g a
Gaussian random field of power spectrum k^-3 (seed 0), at rest with p = 1,
multigrid self-gravity (G for a Jeans length of a third of the box) and
cooling, 200 CFL steps, the misfit L = 1/2 sum (rho_final - rho_target)^2
against the final density of the seed-1 run, its gradient with respect to the
initial density from the checkpointed adjoint rollout (K = 20).

* 16^3 copy, fp64: the same physics over the same time steps (the dt list of
  the configured 128^3 run, replayed), the gradient against central finite
  differences of the GPU forward along random directions, with h from 1e-4
  down to 1e-8 ||rho_0|| (the best h counts: a finite h crosses switches of
  the limiter and the Riemann fan, and the crossings shrink with h), after 10
  and 200 steps, for the multigrid (a fixed cycle count, so the forward map
  is smooth) and the spectral solver; the gradient bitwise independent of the
  checkpoint interval K in {1, 20, 200}.
* Gravity and cooling in the rollout against the oracle's chained step
  adjoints (multigrid with a fixed cycle count, and spectral), bitwise
  independent of K.
* 128^3, the configured size: the gradient over the run's own dt list (the
  target run takes its own CFL steps), its cost and memory, and a
  central-difference check along a smooth direction.

Since the velocity is zero and the pressure fixed, the total energy does not
depend on the initial density, so dL/drho_0 is the density component of the
rollout's adjoint."""
import math
import time

import numpy as np
import pytest

import oracle
import paper_2512_13403_amd as mh
import workloads as wl
from paper_2512_13403_amd import rollout as ro
from parity import pair, rel_err

pytestmark = pytest.mark.gpu


@pytest.fixture(autouse=True)
def _name(request):
    print(f"\n[gpu case] {request.node.nodeid}", flush=True)
    yield


def solver(n, grav_solver, mg_tol=0.0, mg_max_cycles=20):
    """fp64 solver of the box; the multigrid runs exactly mg_max_cycles
    V-cycles per solve when mg_tol = 0."""
    g = mh.grid_desc((n, n, n), (1.0 / n,) * 3, dtype="f64")
    p = mh.physics_desc(flags=mh.SRC_GRAVITY | mh.SRC_COOLING, grav_G=wl.JEANS_G, mg_tol=mg_tol,
                        mg_max_cycles=mg_max_cycles, grav_solver=grav_solver)
    return mh.Solver(g, p)


def dev(a):
    import torch

    return torch.tensor(np.asarray(a), dtype=torch.float64, device="cuda:0")


@pytest.fixture(scope="module")
def configured_dts():
    """The dt list of the configured run: 128^3, seed 0, 200 CFL steps,
    multigrid to 1e-10."""
    n = 128
    s = solver(n, mh.GRAV_MG, mg_tol=1e-10, mg_max_cycles=20)
    s.set_state(dev(wl.grf_density_state(n, seed=0)))
    dts = s.step(200, 0.0, record=True)
    assert s.check()[0] == 0
    s.close()
    return dts


def reset(s, n):
    s.set_clock(0.0, 0)
    s.set_potential(np.zeros((n, n, n)))


def target_density(s, n, dts, nsteps=None):
    """Final density of the seed-1 run over the dt list, or over nsteps CFL
    steps of its own when dts is None (at 128^3 the seed-1 box collapses
    faster than the seed-0 one and needs its own, shorter steps)."""
    reset(s, n)
    s.set_state(dev(wl.grf_density_state(n, seed=1)))
    if dts is None:
        s.step(nsteps, 0.0)
    else:
        for dt in dts:
            s.step(1, float(dt))
    assert s.check()[0] == 0
    return s.get_state_device()[0].clone()


def misfit(s, U0, target, dts):
    """L(U0) for the frozen dt list (a fresh clock and potential)."""
    reset(s, U0.shape[-1])
    Uf, _, _ = ro.rollout_forward(s, U0, len(dts), len(dts), dts)
    d = (Uf[0] - target).double()
    return 0.5 * float((d * d).sum())


def gradient(s, U0, target, dts, K):
    reset(s, U0.shape[-1])
    Uf, _, cks = ro.rollout_forward(s, U0, len(dts), K, dts)
    lam = Uf.clone().zero_()
    lam[0] = Uf[0] - target
    return ro.rollout_backward(s, cks, dts, K, lam)


H_REL = (1e-4, 1e-5, 1e-6, 1e-7, 1e-8)


def fd_check(s, U0, target, dts, g, seeds, tol):
    """Central differences of L along unit density directions v, against
    <g, v>, at h = H_REL ||rho_0||; the best h counts.  A direction whose two
    smallest-h quotients disagree by more than 1e-3 of <g, v> still crosses a
    switch of the scheme at those h and is skipped (at most half of them).
    Returns the best-h errors of the kept directions."""
    n = U0.shape[-1]
    norm = float(U0[0].double().norm())
    errs, skipped = [], 0
    for seed in seeds:
        v = np.random.default_rng(seed).standard_normal((n, n, n))
        v /= np.linalg.norm(v)
        exact = float((g[0].cpu().numpy() * v).sum())
        quot = []
        for hr in H_REL:
            h = hr * norm
            Up, Um = U0.clone(), U0.clone()
            Up[0] += h * dev(v)
            Um[0] -= h * dev(v)
            quot.append((misfit(s, Up, target, dts) - misfit(s, Um, target, dts)) / (2 * h))
        spread = abs(quot[-2] - quot[-1]) / abs(exact)
        e = min(abs(q - exact) / abs(exact) for q in quot)
        print(f"  direction {seed}: <g,v> = {exact:.12e}, rel err per h "
              f"{[f'{abs(q - exact) / abs(exact):.1e}' for q in quot]}, best {e:.2e}", flush=True)
        if spread > 1e-3:
            skipped += 1
            continue
        errs.append(e)
    assert skipped <= len(seeds) // 2, "too many switch crossings"
    assert max(errs) < tol, errs
    return errs


@pytest.mark.parametrize("grav_solver", [mh.GRAV_MG, mh.GRAV_FFT])
@pytest.mark.parametrize("nsteps", [10, 200])
def test_fd_validation_16(configured_dts, grav_solver, nsteps):
    n = 16
    dts = configured_dts[:nsteps]
    s = solver(n, grav_solver)
    target = target_density(s, n, dts)
    U0 = dev(wl.grf_density_state(n, seed=0))
    g = gradient(s, U0, target, dts, K=20)
    assert s.check()[0] == 0
    assert np.isfinite(g.cpu().numpy()).all() and float(g[0].abs().max()) > 0
    # E and m do not depend on rho_0 here: only the density component counts
    fd_check(s, U0, target, dts, g, seeds=(11, 12, 13, 14), tol=1e-5)


@pytest.mark.parametrize("grav_solver", [mh.GRAV_MG, mh.GRAV_FFT])
def test_checkpoint_interval_invariance_16(configured_dts, grav_solver):
    n = 16
    s = solver(n, grav_solver)
    target = target_density(s, n, configured_dts)
    U0 = dev(wl.grf_density_state(n, seed=0))
    grads = {K: gradient(s, U0, target, configured_dts, K).cpu().numpy() for K in (1, 20, 200)}
    assert np.isfinite(grads[1]).all()
    assert np.array_equal(grads[1], grads[20]) and np.array_equal(grads[1], grads[200])


def oracle_rollout_vjp(oc, U0, dts, lam):
    """Chain of oracle step adjoints over the run with the given dt list."""
    sim = oracle.Simulation(oc, U0)
    states = []
    for dt in dts:
        states.append((sim.U.copy(), sim.ahat.copy(), sim.phi.copy(), sim.step_index))
        sim.advance(1, dt)
    nvec = np.zeros((0, 3), np.int32)
    for (U, ahat, phi, k), dt in zip(reversed(states), reversed(list(dts))):
        lam = oracle.step_vjp(oc, U, dt, k, nvec, ahat, phi, lam)
    return sim.U, lam


@pytest.mark.parametrize("grav_solver", [mh.GRAV_MG, mh.GRAV_FFT])
def test_rollout_gravity_cooling_against_oracle(grav_solver):
    import torch

    n, nsteps = 16, 6
    U0 = wl.grf_density_state(n, seed=7)
    U0[1:4] += 0.05 * np.random.default_rng(8).standard_normal((3, n, n, n)) * U0[0]
    kw = dict(grav_G=wl.JEANS_G, grav_solver=grav_solver)
    if grav_solver == mh.GRAV_MG:
        kw.update(mg_tol=0.0, mg_max_cycles=12)  # a fixed cycle count on both sides
    grads = {}
    for K in (1, 4, nsteps):
        s, oc = pair((n, n, n), (1.0 / n,) * 3, dtype="f64",
                     flags=oracle.SRC_GRAVITY | oracle.SRC_COOLING, **kw)
        Uf, dts, cks = ro.rollout_forward(s, dev(U0), nsteps, K)
        lam = dev(np.random.default_rng(9).standard_normal(U0.shape))
        grads[K] = ro.rollout_backward(s, cks, dts, K, lam).cpu().numpy()
    assert np.array_equal(grads[1], grads[4]) and np.array_equal(grads[1], grads[nsteps])
    Uref, gref = oracle_rollout_vjp(oc, U0, dts, lam.cpu().numpy())
    assert rel_err(Uf.cpu().numpy(), Uref) < 1e-12
    assert rel_err(grads[1], gref) < 1e-11
    del torch


def test_configured_gradient_128(configured_dts):
    """128^3, 200 steps, K = 20, multigrid gravity (V-cycles to 1e-10) and
    cooling, fp64: the gradient, its time and memory, and a central
    difference along a smooth direction (a single Fourier mode of the density)."""
    import torch

    n, nsteps, K = 128, 200, 20
    dts = configured_dts
    s = solver(n, mh.GRAV_MG, mg_tol=1e-10, mg_max_cycles=20)
    target = target_density(s, n, None, nsteps)
    U0 = dev(wl.grf_density_state(n, seed=0))
    torch.cuda.synchronize()
    torch.cuda.reset_peak_memory_stats()
    base = torch.cuda.memory_allocated()
    t0 = time.perf_counter()
    reset(s, n)
    Uf, _, cks = ro.rollout_forward(s, U0, nsteps, K, dts)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    lam = Uf.clone().zero_()
    lam[0] = Uf[0] - target
    g = ro.rollout_backward(s, cks, dts, K, lam)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    peak = torch.cuda.max_memory_allocated() - base
    L = 0.5 * float(((Uf[0] - target) ** 2).sum())
    print(f"C4 128^3 fp64: t_end = {sum(dts):.4f}, L = {L:.6e}, forward {t1 - t0:.2f} s "
          f"({1e3 * (t1 - t0) / nsteps:.2f} ms/step), backward {t2 - t1:.2f} s "
          f"({1e3 * (t2 - t1) / nsteps:.2f} ms/step), checkpoints {len(cks)}, "
          f"peak extra device memory {peak / 2 ** 20:.0f} MiB", flush=True)
    gn = g.cpu().numpy()
    assert np.isfinite(gn).all() and np.abs(gn[0]).max() > 0
    # one smooth direction: cos(2 pi (x + 2y + 3z)) / norm
    c = (np.arange(n) + 0.5) / n
    z, y, x = np.meshgrid(c, c, c, indexing="ij")
    v = np.cos(2 * math.pi * (x + 2 * y + 3 * z))
    v /= np.linalg.norm(v)
    exact = float((gn[0] * v).sum())
    norm = float(U0[0].norm())
    quot = []
    for hr in (1e-6, 1e-7):
        h = hr * norm
        Up, Um = U0.clone(), U0.clone()
        Up[0] += h * dev(v)
        Um[0] -= h * dev(v)
        quot.append((misfit(s, Up, target, dts) - misfit(s, Um, target, dts)) / (2 * h))
    e = min(abs(q - exact) / abs(exact) for q in quot)
    print(f"  smooth direction: <g,v> = {exact:.10e}, fd = {quot}, best rel err {e:.2e}",
          flush=True)
    assert e < 1e-4
