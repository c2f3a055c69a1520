"""Store instead of recompute (Sec. 2.3): mh_step_keep keeps a step's first
stage and its state after the forcing kick, and mh_adjoint_step_kept uses
them, and with gravity the potential the step solved for, instead of
recomputing the two stages and the forward Poisson solve.  Both must be
bitwise the plain calls: the state, clock and next CFL dt after the step,
and the adjoint; the checkpointed rollout gradient with and without keeping;
argument errors."""
import numpy as np
import pytest

import oracle
import paper_2512_13403_amd as mh
import workloads as wl
from paper_2512_13403_amd import rollout as ro
from parity import as_input, pair

pytestmark = pytest.mark.gpu


@pytest.fixture(autouse=True)
def _name(request):
    print(f"\n[gpu case] {request.node.nodeid}", flush=True)
    yield


def torch_dev(a, dtype):
    import torch

    return torch.tensor(np.asarray(a), dtype=torch.float64 if dtype == "f64" else torch.float32,
                        device="cuda:0")


def grav_state(n, seed=5):
    U0 = wl.grf_density_state(n, seed=seed)
    U0[1:4] += 0.05 * np.random.default_rng(seed + 1).standard_normal((3, n, n, n)) * U0[0]
    return U0


F, C, G = oracle.SRC_FORCING, oracle.SRC_COOLING, oracle.SRC_GRAVITY
CASES = {
    "plain": dict(flags=0),
    "forcing+cooling": dict(flags=F | C, ou_seed=3),
    "cooling": dict(flags=C),
    "forcing": dict(flags=F, ou_seed=4),
    "gravity-mg+cooling": dict(flags=G | C, grav_G=wl.JEANS_G, mg_tol=0.0, mg_max_cycles=8),
    "gravity-fft+forcing": dict(flags=G | F, grav_G=wl.JEANS_G, grav_solver=oracle.GRAV_FFT,
                                ou_seed=5),
    "tabulated cooling": dict(flags=F | C, ou_seed=6, cool_model=oracle.COOL_TABLE,
                              cool_table=wl.synthetic_cie_table(),
                              cool_integrator=oracle.COOLINT_AUTO, cool_frac=0.05,
                              cool_nsub_max=50, **wl.COOLING_TABLE_MODEL),
}


def setup(case, dtype):
    kw = CASES[case]
    if kw["flags"] & G:
        n = 16
        shape, h, U0 = (n, n, n), (1 / n,) * 3, grav_state(n)
    elif case == "tabulated cooling":
        shape, h = (8, 10, 34), (1 / 34, 1 / 10, 1 / 8)
        U0 = wl.random_state(shape, seed=37, vmax=0.4, rho=(0.5, 2.0), p=(0.002, 1.0))
    else:
        shape, h = (9, 12, 40), (1 / 40, 1 / 12, 1 / 9)
        U0 = wl.random_state(shape, seed=21, vmax=0.5)
    return shape, h, as_input(U0, dtype), kw


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("case", list(CASES))
def test_keep_step_and_kept_adjoint_are_bitwise(case, dtype):
    import torch

    shape, h, Uin, kw = setup(case, dtype)
    s1, oc = pair(shape, h, dtype=dtype, **kw)
    s2, _ = pair(shape, h, dtype=dtype, **kw)
    U0 = torch_dev(Uin, dtype)
    for s in (s1, s2):
        s.set_state(U0)
    ahat = s1.ou_state() if kw["flags"] & F else None
    phi = s1.potential_device() if kw["flags"] & G else None
    d1 = s1.step(1, 0.0, record=True)
    U1, Ub = s2.new_state_tensor(), s2.new_state_tensor()
    d2 = s2.step_keep(0.0, U1, Ub, record=True)
    phi1 = s2.potential_device() if kw["flags"] & G else None
    assert d1[0] == d2[0] > 0
    assert torch.equal(s1.get_state_device(), s2.get_state_device())
    assert s1.clock() == s2.clock()
    # the epilogue's CFL speed and health check: the next step's dt agrees
    assert s1.check()[0] == s2.check()[0] == 0
    n1, n2 = s1.step(1, 0.0, record=True), s2.step(1, 0.0, record=True)
    assert n1[0] == n2[0]
    # the adjoint of the first step, recomputed and kept
    lam = torch_dev(np.random.default_rng(7).standard_normal(Uin.shape), dtype)
    a1 = s1.adjoint_step(U0, float(d1[0]), 0, lam, ou_ahat=ahat, phi_n=phi)
    a2 = s1.adjoint_step(U0, float(d1[0]), 0, lam, ou_ahat=ahat, phi_n=phi, kept=(U1, Ub))
    assert torch.equal(a1, a2), (a1 - a2).abs().max().item()
    if kw["flags"] & G:
        # and the potential the step solved for (the multigrid solve skipped;
        # ignored by the spectral solver)
        a3 = s1.adjoint_step(U0, float(d1[0]), 0, lam, ou_ahat=ahat, phi_n=phi,
                             kept=(U1, Ub, phi1))
        assert torch.equal(a1, a3), (a1 - a3).abs().max().item()


@pytest.mark.parametrize("case", ["forcing+cooling", "gravity-mg+cooling", "gravity-fft+forcing"])
def test_rollout_gradient_with_kept_stages(case):
    import torch

    n = 16
    kw = CASES[case]
    flags = kw["flags"]
    U0 = grav_state(n, seed=9) if flags & G else wl.random_state((n, n, n), seed=22, vmax=0.5)
    s, _ = pair((n, n, n), (1 / n,) * 3, dtype="f64", **kw)
    nsteps, K = 7, 3
    Uf, dts, cks = ro.rollout_forward(s, torch_dev(U0, "f64"), nsteps, K)
    lam = torch_dev(np.cos(np.arange(U0.size)).reshape(U0.shape), "f64")
    g0 = ro.rollout_backward(s, cks, dts, K, lam, keep=False)
    g1 = ro.rollout_backward(s, cks, dts, K, lam, keep=True)
    assert torch.equal(g0, g1)


def test_keep_argument_errors():
    import torch

    shape, h = (8, 8, 16), (1 / 16, 1 / 8, 1 / 8)
    s, _ = pair(shape, h, dtype="f32")
    s.set_state(torch_dev(wl.random_state(shape, seed=3), "f32"))
    U1 = s.new_state_tensor()
    with pytest.raises(mh.MHError):  # the same buffer twice
        s.step_keep(0.0, U1, U1)
    s3, _ = pair(shape, h, dtype="f32", integrator=oracle.RK_SSP3)
    s3.set_state(torch_dev(wl.random_state(shape, seed=3), "f32"))
    with pytest.raises(mh.MHError):  # SSPRK3 keeps no two-stage intermediates
        s3.step_keep(0.0, s3.new_state_tensor(), s3.new_state_tensor())
    lam = torch.zeros_like(U1)
    with pytest.raises(mh.MHError):
        s3.adjoint_step(s3.get_state_device(), 1e-3, 0, lam, kept=(U1, s3.new_state_tensor()))
    torch.cuda.synchronize()
