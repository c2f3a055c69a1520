"""Pins of the corrector oracle (oracle/corrector.py) against independent
facts: bf16 rounding against torch's float32 -> bfloat16 conversion (round to
nearest even); the periodic 3x3x3 convolution against scipy.ndimage.correlate
in wrap mode, channel pair by channel pair; the adjoint identities of the
convolution's input and weight gradients; GELU's closed-form values; the full
backward pass against central finite differences of the forward in exact
arithmetic; the first ADAM step's closed form (-lr sign(g)); the floor."""
import math

import numpy as np
import pytest
import torch
from scipy.ndimage import correlate

import oracle.corrector as oc
import workloads as wl


def test_bf16_round_matches_torch():
    rng = np.random.default_rng(0)
    x = np.concatenate([rng.standard_normal(10000) * 10 ** rng.uniform(-6, 6, 10000),
                        np.array([1.0 + 2 ** -8, 1.0 + 3 * 2 ** -8, -1.0 - 2 ** -8, 0.0, 1e-40])])
    x32 = x.astype(np.float32)
    ref = torch.from_numpy(x32).to(torch.bfloat16).to(torch.float32).numpy().astype(np.float64)
    assert np.array_equal(oc.bf16_round(x32), ref)


def test_conv3_matches_scipy_correlate():
    rng = np.random.default_rng(1)
    x = rng.standard_normal((1, 5, 6, 7, 3))
    W = rng.standard_normal((4, 3, 27))
    y = oc.conv3(x, W)
    for co in range(4):
        ref = np.zeros(x.shape[1:4])
        for ci in range(3):
            k = np.zeros((3, 3, 3))
            for t, (dx, dy, dz) in enumerate(oc.TAPS):
                k[dz + 1, dy + 1, dx + 1] = W[co, ci, t]
            ref += correlate(x[0, :, :, :, ci], k, mode="wrap")
        assert np.allclose(y[0, :, :, :, co], ref, rtol=1e-12, atol=1e-12)


def test_conv3_gradients_are_adjoints():
    rng = np.random.default_rng(2)
    x = rng.standard_normal((2, 4, 5, 6, 3))
    W = rng.standard_normal((4, 3, 27))
    gy = rng.standard_normal((2, 4, 5, 6, 4))
    lhs = (oc.conv3(x, W) * gy).sum()
    assert lhs == pytest.approx((x * oc.conv3_input_grad(gy, W)).sum(), rel=1e-12)
    assert lhs == pytest.approx((W * oc.conv3_weight_grad(gy, x)).sum(), rel=1e-12)


def test_gelu_values():
    assert oc.gelu(np.array([0.0]))[0] == 0.0
    assert oc.gelu(np.array([10.0]))[0] == pytest.approx(10.0, rel=1e-15)
    assert oc.gelu(np.array([-10.0]))[0] == pytest.approx(0.0, abs=1e-20)
    # Phi(1) = 0.841344746...; GELU(1) = Phi(1)
    assert oc.gelu(np.array([1.0]))[0] == pytest.approx(0.8413447460685429, rel=1e-14)
    z = np.linspace(-4, 4, 33)
    fd = (oc.gelu(z + 1e-6) - oc.gelu(z - 1e-6)) / 2e-6
    assert np.allclose(oc.gelu_grad(z), fd, rtol=1e-8, atol=1e-10)


def _setup(n=6, B=2, seed=3):
    rng = np.random.default_rng(seed)
    U = np.stack([wl.smooth_random_state((n, n, n), seed=seed + b) for b in range(B)])
    T = U + 0.01 * rng.standard_normal(U.shape)
    theta = wl.corrector_init_params(seed=seed, out_scale=0.5)
    mean = U.mean(axis=(0, 2, 3, 4))
    std = U.std(axis=(0, 2, 3, 4)) + 1e-3
    scale = 0.02 * std
    return U, T, theta, mean, std, scale


def test_backward_matches_finite_differences():
    U, T, theta, mean, std, scale = _setup()
    w, sig = (4.0, 1.0, 1.0, 1.0, 1.0), std

    def loss(th):
        Uc, _ = oc.forward(U, th, mean, std, scale, rounding=False)
        return oc.loss_and_grad_y(Uc, T, w, sig)[0]

    Uc, cache = oc.forward(U, theta, mean, std, scale, rounding=False)
    _, gU = oc.loss_and_grad_y(Uc, T, w, sig)
    g = oc.backward(gU, cache, scale)
    rng = np.random.default_rng(4)
    for _ in range(3):
        d = rng.standard_normal(theta.size)
        eps = 1e-6
        fd = (loss(theta + eps * d) - loss(theta - eps * d)) / (2 * eps)
        assert float(g @ d) == pytest.approx(fd, rel=1e-6)
    # single entries in each parameter block
    offs = np.cumsum([0] + [int(np.prod(s)) for _, s in oc.SHAPES])
    for b in range(6):
        q = int(offs[b] + 3 % (offs[b + 1] - offs[b]))
        e = np.zeros(theta.size)
        e[q] = 1.0
        fd = (loss(theta + 1e-6 * e) - loss(theta - 1e-6 * e)) / 2e-6
        assert g[q] == pytest.approx(fd, rel=1e-5, abs=1e-12)


def test_input_gradient_matches_finite_differences():
    U, T, theta, mean, std, scale = _setup()
    w, sig = (4.0, 1.0, 1.0, 1.0, 1.0), std

    def loss(u):
        Uc, _ = oc.forward(u, theta, mean, std, scale, rounding=False)
        return oc.loss_and_grad_y(Uc, T, w, sig)[0]

    Uc, cache = oc.forward(U, theta, mean, std, scale, rounding=False)
    _, gUc = oc.loss_and_grad_y(Uc, T, w, sig)
    oc.backward(gUc, cache, scale)
    gU = oc.input_grad(gUc, cache, std)
    rng = np.random.default_rng(8)
    for _ in range(3):
        d = rng.standard_normal(U.shape)
        eps = 1e-6
        fd = (loss(U + eps * d) - loss(U - eps * d)) / (2 * eps)
        assert float((gU * d).sum()) == pytest.approx(fd, rel=1e-6)
    # the network path matters: without it the directional derivative is off
    d = rng.standard_normal(U.shape)
    fd = (loss(U + 1e-6 * d) - loss(U - 1e-6 * d)) / 2e-6
    assert abs(float((gUc * d).sum()) - fd) > 1e-3 * abs(fd)


def test_split_input_carries_sixteen_bits():
    rng = np.random.default_rng(7)
    x = np.concatenate([rng.standard_normal(20000) * 10 ** rng.uniform(-3, 1, 20000),
                        np.array([0.0, 1.0, -2.5, 1.0 + 2 ** -9 + 2 ** -20])])
    hi, lo = oc.split_parts(x)
    # each part is a bf16 value (torch's float32 -> bfloat16 rounding is exact on them)
    for part in (hi, lo):
        t = torch.from_numpy(part.astype(np.float32)).to(torch.bfloat16).to(torch.float32)
        assert np.array_equal(t.numpy().astype(np.float64), part)
    x32 = x.astype(np.float32).astype(np.float64)
    assert np.array_equal(hi, oc.bf16_round(x))
    # |x - (hi + lo)| <= 2^-16 |x| (two 8-bit significands, round to nearest)
    assert np.all(np.abs(x32 - (hi + lo)) <= 2.0 ** -16 * np.abs(x32))
    # the low part keeps 8 bits of the remainder: 1 + 2^-9 + 2^-20 -> 1 + 2^-9
    assert np.array_equal(oc.split_bf16(np.array([1.0 + 2 ** -9 + 2 ** -20])),
                          np.array([1.0 + 2 ** -9]))


def test_rounded_forward_close_to_exact():
    U, T, theta, mean, std, scale = _setup()
    a, _ = oc.forward(U, theta, mean, std, scale, rounding=True)
    b, _ = oc.forward(U, theta, mean, std, scale, rounding=False)
    # the correction is scale * y with |y| ~ 1: bf16 changes it by ~1 %
    assert np.abs(a - b).max() < 0.05 * np.abs(b - U).max()


def test_adam_first_step_is_signed_lr():
    g = np.array([3.0, -0.5, 1e-3])
    th, m, v = oc.adam(np.zeros(3), np.zeros(3), np.zeros(3), g, 1, 1e-3)
    assert np.allclose(th, -1e-3 * np.sign(g), rtol=1e-5)


def test_floor_only_touches_unphysical_cells():
    U, _, _, _, _, _ = _setup(n=4, B=1)
    Uc = U.copy()
    Uc[0, 0, 1, 2, 3] = -1.0          # negative density
    Uc[0, 4, 0, 0, 0] = 0.0           # negative pressure
    out, nfl, bad = oc.floor_and_check(U, Uc, 5 / 3)
    assert nfl == 2 and not bad
    assert out[0, 0, 1, 2, 3] == pytest.approx(1e-6 * U[0, 0].mean())
    keep = np.ones(U.shape[2:], bool)
    keep[1, 2, 3] = keep[0, 0, 0] = False
    assert np.array_equal(out[0][:, keep], Uc[0][:, keep])
    Uc[0, 2, 1, 1, 1] = np.nan
    assert oc.floor_and_check(U, Uc, 5 / 3)[2]
