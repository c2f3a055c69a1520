"""The learned flux-correction hook (Sec. 8, the solver-in-the-loop flux
term): the step with a correction field against the oracle, the adjoint
step's gradient with respect to the field against the oracle's, and a field
fitted through the adjoint rollout lowering its misfit."""
import numpy as np
import pytest

import oracle
import paper_2512_13403_amd as mh
import workloads as wl
from paper_2512_13403_amd import inversion as inv
from parity import TOL, as_input, pair, rel_err

pytestmark = pytest.mark.gpu


@pytest.fixture(autouse=True)
def _name(request):
    print(f"\n[gpu case] {request.node.nodeid}", flush=True)
    yield


def dev(a, dtype):
    import torch

    return torch.tensor(np.asarray(a), dtype=torch.float64 if dtype == "f64" else torch.float32,
                        device="cuda:0").contiguous()


CASES = [dict(bc=(0, 0, 0)),
         dict(bc=(1, 0, 1), limiter=oracle.LIM_VANLEER, integrator=oracle.RK_SSP3,
              flags=oracle.SRC_FORCING | oracle.SRC_COOLING, ou_seed=3)]


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("case", range(len(CASES)))
def test_step_with_flux_correction(dtype, case):
    kw = dict(CASES[case])
    bc = kw.pop("bc")
    shape = (9, 11, 70)
    h = (1 / 70, 1 / 11, 1 / 9)
    U0 = as_input(wl.random_state(shape, seed=50, vmax=0.5), dtype)
    B = as_input(0.05 * np.random.default_rng(51).standard_normal((5,) + shape), dtype)
    s, oc = pair(shape, h, bc, dtype, **kw)
    oracle.set_flux_corr(oc, B)
    dt = 0.6 * oracle.cfl_dt(oc, U0)
    Bd = dev(B, dtype)
    s.set_flux_correction(Bd)
    s.set_state(U0)
    s.step(3, dt)
    sim = oracle.Simulation(oc, U0).advance(3, dt)
    assert rel_err(s.get_state(), sim.U) < TOL[dtype]


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("case", range(len(CASES)))
def test_adjoint_gradient_of_the_flux_correction(dtype, case):
    kw = dict(CASES[case])
    bc = kw.pop("bc")
    shape = (9, 11, 70)
    h = (1 / 70, 1 / 11, 1 / 9)
    U0 = as_input(wl.random_state(shape, seed=52, vmax=0.5), dtype)
    rng = np.random.default_rng(53)
    B = as_input(0.05 * rng.standard_normal((5,) + shape), dtype)
    lam = as_input(rng.standard_normal((5,) + shape), dtype)
    s, oc = pair(shape, h, bc, dtype, **kw)
    oracle.set_flux_corr(oc, B)
    dt = 0.6 * oracle.cfl_dt(oc, U0)
    nvec = oracle.ou_modes(oc.ou_kmin, oc.ou_kmax) if oc.flags & oracle.SRC_FORCING else \
        np.zeros((0, 3), np.int32)
    ahat = oracle.ou_init(oc, nvec) if len(nvec) else np.zeros(6)
    ref_lam, ref_g = oracle.step_vjp_flux(oc, U0, dt, 2, nvec, ahat, np.zeros(shape), lam)
    g = dev(np.zeros((5,) + shape), dtype)
    s.set_flux_correction(dev(B, dtype), g)
    got = s.adjoint_step(dev(U0, dtype), dt, 2, dev(lam, dtype),
                         ou_ahat=ahat if len(nvec) else None).cpu().numpy()
    assert rel_err(got, ref_lam) < TOL[dtype]
    gg = g.cpu().numpy()
    assert np.abs(gg - ref_g).max() < 10 * TOL[dtype] * np.abs(ref_g).max()


def test_learned_flux_field_lowers_the_misfit():
    import torch

    n, nsteps = 32, 10
    s = mh.Solver(mh.grid_desc((n, n, n), (1.0 / n,) * 3, dtype="f64"), mh.physics_desc())
    U0 = dev(wl.smooth_random_state((n, n, n), seed=54), "f64")
    B_true = dev(0.02 * wl.smooth_random_state((n, n, n), seed=55) -
                 0.02 * wl.smooth_random_state((n, n, n), seed=56), "f64")
    s.set_flux_correction(B_true)
    s.set_state(U0)
    dts = s.step(nsteps, 0.0, record=True)
    target = s.get_state_device()[0].clone()
    s.set_flux_correction(None)
    B, losses = inv.learn_flux_correction(s, U0, target, dts, iters=25, lr=2e-3, K=5)
    print("flux misfit", losses[0], "->", losses[-1], flush=True)
    assert all(np.isfinite(losses))
    assert losses[-1] < 0.2 * losses[0]
