"""The corrector network in flux mode driving the learned flux hook (Sec. 8,
the solver-in-the-loop flux corrector): the parameter gradient of a one-step
misfit, chained through the adjoint step and the network's reverse pass,
against central differences in output-layer weights, and a network with a
perturbed output layer trained back towards a teacher's rollout."""
import numpy as np
import pytest

import oracle.corrector as oc
import paper_2512_13403_amd as mh
import workloads as wl
from paper_2512_13403_amd import fluxsil
from parity import as_input

pytestmark = pytest.mark.gpu

GAMMA = 5.0 / 3.0
N = 16


@pytest.fixture(autouse=True)
def _name(request):
    print(f"\n[gpu case] {request.node.nodeid}", flush=True)
    yield


def dev(a, dtype):
    import torch

    return torch.tensor(np.asarray(a), dtype=torch.float64 if dtype == "f64" else torch.float32,
                        device="cuda:0").contiguous()


def teacher_params(seed=5):
    theta = wl.corrector_init_params(seed=seed, out_scale=0.3)
    rng = np.random.default_rng(seed + 1)
    theta[-5:] = 0.2 * rng.standard_normal(5)
    return theta.astype(np.float32)


def setup(dtype, seed=140):
    shape = (N, N, N)
    s = mh.Solver(mh.grid_desc(shape, (1.0 / N,) * 3, dtype=dtype))
    U0 = as_input(wl.smooth_random_state(shape, seed=seed, kmax=3), dtype)
    mean = U0.mean(axis=(1, 2, 3))
    std = U0.std(axis=(1, 2, 3)) + 1e-3
    scale = (2e-2, 1e-2, 1e-2, 1e-2, 3e-2)
    corr = mh.Corrector(mh.corr_desc(N, 1, dtype, GAMMA, mean, std, scale, (1.0,) * 5, 1e-6,
                                     1e-3, mode=mh.CORR_FLUX))
    rho, P = U0[0], (GAMMA - 1.0) * (U0[4] - 0.5 * (U0[1:4] ** 2).sum(axis=0) / U0[0])
    vmax = (np.sqrt((U0[1:4] / rho) ** 2).max(axis=0) + np.sqrt(GAMMA * P / rho)).max()
    dt = 0.3 / N / vmax
    return s, corr, U0, dt


W3_OFF = 32 * 5 * 27 + 32 + 32 * 32 * 27 + 32  # W3[5][32][27] in the flat parameter order


def test_parameter_gradient_against_differences():
    """Central differences in single output-layer weights (pre-rounded to
    bf16, stepped by bf16-representable amounts, so the network sees the
    exact perturbation); the output biases add a uniform field, whose face
    differences cancel, so their gradient vanishes."""
    dtype = "f64"
    s, corr, U0, dt = setup(dtype)
    theta = oc.pack({k: oc.bf16_round(v) if k.startswith("W") else v
                     for k, v in oc.unpack(teacher_params()).items()}).astype(np.float32)
    Ud = dev(U0, dtype)
    dts = [dt]
    corr.set_params(theta)
    states, _ = fluxsil.rollout(s, corr, Ud, dts)
    rng = np.random.default_rng(141)
    targets = [states[1] + dev(1e-3 * rng.standard_normal(U0.shape), dtype)]
    corr.zero_grad()
    fluxsil.loss_and_grad(s, corr, Ud, dts, targets)
    g = corr.grad().astype(np.float64)
    gw3 = g[W3_OFF:W3_OFF + 5 * 32 * 27]
    # zero up to the bf16 rounding of the upstream gradient in the network's
    # reverse pass, which breaks the exact cancellation of the face sums
    assert np.abs(g[-5:]).max() < 1e-2 * np.abs(gw3).max()
    for c in range(5):
        # the weight of this output channel with the largest gradient
        j = W3_OFF + c * 32 * 27 + int(np.argmax(np.abs(gw3[c * 32 * 27:(c + 1) * 32 * 27])))
        w = float(theta[j])
        ulp = 2.0 ** (np.floor(np.log2(abs(w))) - 7)
        eps = 2.0 * ulp
        vals = []
        for sgn in (1.0, -1.0):
            th = theta.copy()
            th[j] = np.float32(w + sgn * eps)
            assert oc.bf16_round(np.float64(th[j])) == w + sgn * eps
            corr.set_params(th)
            st, _ = fluxsil.rollout(s, corr, Ud, dts)
            vals.append(fluxsil.misfit(st, targets))
        fd = (vals[0] - vals[1]) / (2.0 * eps)
        assert abs(fd - g[j]) <= 1e-2 * abs(g[j]), (c, fd, g[j])


def test_training_towards_a_teacher():
    dtype = "f32"
    s, corr, U0, dt = setup(dtype, seed=150)
    Ud = dev(U0, dtype)
    dts = [dt] * 3
    theta = teacher_params()
    corr.set_params(theta)
    states, _ = fluxsil.rollout(s, corr, Ud, dts)
    targets = [t.clone() for t in states[1:]]
    # the student: output layer perturbed
    rng = np.random.default_rng(151)
    th = theta.copy()
    nw3 = 5 * 32 * 27
    nb = mh.NPARAM_CORRECTOR - 5
    th[nb - nw3:nb] *= np.float32(1.0) + np.float32(0.5) * rng.standard_normal(nw3).astype(np.float32)
    corr.set_params(th)
    losses = np.array(fluxsil.train(s, corr, Ud, dts, targets, iters=30, lr=3e-4))
    assert np.all(np.isfinite(losses)) and losses[0] > 0
    assert np.all(losses[1:] < losses[:-1] * 1.05), losses
    assert losses[-1] < 0.15 * losses[0], losses
