"""GPU parity of the learned state corrector (mh_corr_*) against the oracle
of oracle/corrector.py, which takes the same bf16-rounded operands at the same
points and accumulates in float64.

Layer by layer, each GPU layer is compared with the oracle layer fed the GPU's
own input activations, so every comparison sees one layer's arithmetic only:
fp32-accumulated products within 1e-5 of the fp64 sum (relative to the
layer's largest value), and bf16-rounded activations equal except for
elements that sit on a rounding boundary, which may differ by one bf16 ulp
(at most 0.1 % of them).  The reverse pass is checked the same way, element
by element on the GPU's own activations and gradient activations: dY, dZ2
and dZ1 as bf16 activations, each weight and bias gradient and the first
layer's input gradient within 1e-5 of the sum of the magnitudes of its
products (the worst-case error of fp32 accumulation over the ~130 sequential
MFMA accumulations of one chunk of cells is about 130 * 2^-24 = 8e-6 of that
sum), and dL/dU within two fp32 roundings.  Only the end-to-end correction
and gradients against the oracle's own forward pass, where one-ulp flips
propagate, are compared in norm."""
import numpy as np
import pytest

import oracle.corrector as oc
import paper_2512_13403_amd as mh
import workloads as wl
from parity import as_input

pytestmark = pytest.mark.gpu

GAMMA = 5.0 / 3.0


@pytest.fixture(autouse=True)
def _name(request):
    print(f"\n[gpu case] {request.node.nodeid}", flush=True)
    yield


def torch_dev(a, dtype):
    import torch

    return torch.tensor(np.asarray(a), dtype=torch.float64 if dtype == "f64" else torch.float32,
                        device="cuda:0")


def batch_state(n, batch, seed, dtype):
    U = np.stack([wl.smooth_random_state((n, n, n), seed=seed + b, kmax=4) for b in range(batch)])
    return as_input(U, dtype)


def stats(U):
    mean = U.mean(axis=(0, 2, 3, 4))
    std = U.std(axis=(0, 2, 3, 4)) + 1e-3
    return mean, std


def params(seed=1, bias=0.1):
    theta = wl.corrector_init_params(seed=seed, out_scale=1.0)
    rng = np.random.default_rng(seed + 100)
    p = oc.unpack(theta)
    for k in ("b1", "b2", "b3"):
        p[k] = bias * rng.standard_normal(p[k].shape)
    return oc.pack(p).astype(np.float32).astype(np.float64)


def make(n, batch, dtype, U, scale=(1e-2,) * 5, loss_w=(4.0, 1.0, 1.0, 1.0, 1.0),
         fallback_frac=1e-3, theta=None):
    mean, std = stats(U)
    d = mh.corr_desc(n, batch, dtype, GAMMA, mean, std, scale, loss_w, 1e-6, fallback_frac)
    c = mh.Corrector(d)
    th = params() if theta is None else theta
    c.set_params(th)
    return c, th, mean, std, np.asarray(scale)


def rel_inf(a, b):
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


def check_bf16_activation(got, ref):
    """Equal except one-ulp flips on at most 0.1 % of the elements."""
    diff = got != ref
    assert diff.mean() <= 1e-3, diff.mean()
    if diff.any():
        assert np.all(np.abs(got[diff] - ref[diff]) <= 2.0 ** -7 * np.abs(ref[diff]) + 1e-30)


def check_bf16_recomputed(got, ref, err):
    """A bf16 activation that the oracle recomputes from the GPU's inputs to
    it (an fp32-accumulated convolution times GELU', then bf16): equal to the
    rounded oracle value except on at most 0.1 % of the elements, which may
    differ by one bf16 ulp plus the bound `err` of the GPU's own arithmetic
    before the rounding."""
    r = oc.bf16_round(ref)
    diff = got != r
    assert diff.mean() <= 1e-3, diff.mean()
    if diff.any():
        bound = 2.0 ** -7 * np.abs(r) + err
        assert np.all(np.abs(got - r)[diff] <= bound[diff] + 1e-300)


def dz_error_bound(S, z):
    """Error bound of dZ = (conv of the upstream bf16 gradient) * GELU'(z) on
    the GPU before its bf16 rounding, with S the sum of the magnitudes of the
    convolution's products: fp32 accumulation (1e-5 of S, as for the other
    products) times |GELU'|, plus S times the absolute error of the GPU's
    GELU' = Phi + z phi.  That derivative comes from the Numerical Recipes
    erfc fit (relative error 1.2e-7) and fp32 exp, a relative error well
    below 1e-6 in each of Phi and z phi; near its root (z = -0.75) the two
    cancel and only this absolute bound holds."""
    from scipy.special import erfc

    Phi = 0.5 * erfc(-z / np.sqrt(2.0))
    phi = np.exp(-0.5 * z * z) / np.sqrt(2.0 * np.pi)
    return S * (1e-5 * np.abs(oc.gelu_grad(z)) + 1e-6 * (Phi + np.abs(z) * phi))


def to_oracle(a, batch, n):
    return a.reshape(batch, n, n, n, a.shape[-1])


@pytest.mark.parametrize("dtype", ["f32", "f64"])
@pytest.mark.parametrize("n,batch", [(16, 2), (32, 1)])
def test_forward_layers(dtype, n, batch):
    U = batch_state(n, batch, 10, dtype)
    c, th, mean, std, scale = make(n, batch, dtype, U)
    Ud = torch_dev(U, dtype)
    out, nfl, fb = c.apply(Ud)
    out = out.cpu().numpy()
    h1_apply = c.activation(2)
    c.loss_grad(Ud, Ud)  # the training forward also stores z1, z2 and y
    assert np.array_equal(c.activation(2), h1_apply)
    p = {k: oc.bf16_round(v) if k.startswith("W") else v for k, v in oc.unpack(th).items()}
    # network input, both bf16 parts: bitwise
    x0 = c.activation(0)
    hi, lo = oc.split_parts((np.moveaxis(U, 1, -1) - mean) / std)
    assert np.array_equal(x0[:, :5], hi.reshape(-1, 5))
    assert np.array_equal(x0[:, 5:10], lo.reshape(-1, 5)) and not x0[:, 10:].any()
    # each layer from the GPU's own input activations
    z1 = c.activation(1)
    xin = to_oracle(x0[:, :5] + x0[:, 5:10], batch, n)
    assert rel_inf(z1, oc.conv3(xin, p["W1"], p["b1"]).reshape(-1, 32)) < 1e-5
    h1 = c.activation(2)
    check_bf16_activation(h1, oc.bf16_round(oc.gelu(z1)))
    z2 = c.activation(3)
    assert rel_inf(z2, oc.conv3(to_oracle(h1, batch, n), p["W2"], p["b2"]).reshape(-1, 32)) < 1e-5
    h2 = c.activation(4)
    check_bf16_activation(h2, oc.bf16_round(oc.gelu(z2)))
    y = c.activation(5)
    assert not y[:, 5:].any()
    yref = oc.conv3(to_oracle(h2, batch, n), p["W3"], p["b3"]).reshape(-1, 5)
    assert rel_inf(y[:, :5], yref) < 1e-5
    # residual update from the GPU's y, then the floor (none needed here)
    Uc = U + np.moveaxis(to_oracle(y[:, :5], batch, n), -1, 1) * scale.reshape(1, 5, 1, 1, 1)
    ref, nref, bad = oc.floor_and_check(U, Uc, GAMMA)
    assert nfl == nref == 0 and not fb and not bad
    tol = 1e-15 if dtype == "f64" else 2e-7
    assert rel_inf(out, ref) < tol
    # inference writes U + scale y from the last layer's epilogue, from the
    # same y as the training forward: in fp32 bitwise the residual kernel's
    # rounding (the product in fp64, rounded to fp32, then the sum); in fp64
    # the product and the sum may fuse into one rounding
    td = np.float64 if dtype == "f64" else np.float32
    d = (scale.reshape(1, 5, 1, 1, 1) * np.moveaxis(to_oracle(y[:, :5], batch, n), -1, 1)
         .astype(np.float64)).astype(td)
    if dtype == "f32":
        assert np.array_equal(out, U.astype(td) + d)
    else:
        assert np.all(np.abs(out - (U + d)) <= 2.3e-16 * (np.abs(U) + np.abs(d)))
    # end to end against the oracle's own forward: the correction agrees in norm
    oref, _ = oc.forward(U, th, mean, std, scale)
    dc, dr = out - U, oref - U
    assert np.linalg.norm(dc - dr) / np.linalg.norm(dr) < 1e-2


def test_batch_members_are_independent():
    n = 16
    U = batch_state(n, 2, 20, "f32")
    c2, th, mean, std, scale = make(n, 2, "f32", U)
    out2 = c2.apply(torch_dev(U, "f32"))[0].cpu().numpy()
    for b in range(2):
        d = mh.corr_desc(n, 1, "f32", GAMMA, mean, std, scale, (1.0,) * 5, 1e-6, 1e-3)
        c1 = mh.Corrector(d)
        c1.set_params(th)
        out1 = c1.apply(torch_dev(U[b:b + 1], "f32"))[0].cpu().numpy()
        assert np.array_equal(out1[0], out2[b])


def oracle_grad_from_gpu(c, U, T, th, std, scale, loss_w, batch, n):
    """The oracle's backward pass on the GPU's forward activations."""
    p = {k: oc.bf16_round(v) if k.startswith("W") else v for k, v in oc.unpack(th).items()}
    y = c.activation(5)[:, :5]
    x0 = c.activation(0)
    cache = dict(x=to_oracle(x0[:, :5] + x0[:, 5:10], batch, n),
                 z1=to_oracle(c.activation(1), batch, n), h1=to_oracle(c.activation(2), batch, n),
                 z2=to_oracle(c.activation(3), batch, n), h2=to_oracle(c.activation(4), batch, n),
                 y=to_oracle(y, batch, n), p=p, rd=oc.bf16_round)
    Uc = U + np.moveaxis(to_oracle(y, batch, n), -1, 1) * scale.reshape(1, 5, 1, 1, 1)
    L, gUc = oc.loss_and_grad_y(Uc, T, loss_w, std)
    return L, oc.backward(gUc, cache, scale)


BLOCKS = [("W1", 0, 4320), ("b1", 4320, 4352), ("W2", 4352, 32000), ("b2", 32000, 32032),
          ("W3", 32032, 36352), ("b3", 36352, 36357)]


def check_sum_bound(got, ref, absref, what, tol=1e-5):
    """|got - ref| <= tol * (sum of the magnitudes of the products) per element."""
    err = np.abs(np.asarray(got, dtype=np.float64) - ref)
    bound = tol * absref + 1e-300
    worst = float((err / bound).max())
    assert worst <= 1.0, (what, worst)
    return worst


def check_reverse_pass(c, th, gUc, scale, batch, n, grad=None, input_grad=False):
    """Element-wise checks of one GPU reverse pass, each step from the GPU's
    own inputs to it: dY from the upstream gradient gUc (dL/dU' of the oracle
    on the GPU's y), the layer-3 gradients from dY and h2, dZ2 from dY, W3
    and z2, the layer-2 gradients from dZ2 and h1, dZ1 from dZ2, W2 and z1,
    the layer-1 gradients from dZ1 and both input parts, and (input_grad) the
    transposed first layer from dZ1.  grad: the GPU's parameter gradient of
    this pass alone."""
    p = {k: oc.bf16_round(v) if k.startswith("W") else v for k, v in oc.unpack(th).items()}
    B = lambda a: to_oracle(a, batch, n)
    x0 = c.activation(0)
    xhi, xlo = B(x0[:, :5]), B(x0[:, 5:10])
    z1, h1, z2, h2 = (B(c.activation(k)) for k in (1, 2, 3, 4))
    dy = c.activation(6)
    assert not dy[:, 5:].any()
    dy = B(dy[:, :5])
    check_bf16_activation(dy.reshape(-1, 5),
                          oc.bf16_round(np.moveaxis(gUc, 1, -1) * scale).reshape(-1, 5))
    dz2 = B(c.activation(7))
    check_bf16_recomputed(dz2, oc.conv3_input_grad(dy, p["W3"]) * oc.gelu_grad(z2),
                          dz_error_bound(oc.conv3_input_grad(np.abs(dy), np.abs(p["W3"])), z2))
    dz1 = B(c.activation(8))
    check_bf16_recomputed(dz1, oc.conv3_input_grad(dz2, p["W2"]) * oc.gelu_grad(z1),
                          dz_error_bound(oc.conv3_input_grad(np.abs(dz2), np.abs(p["W2"])), z1))
    if grad is not None:
        g = oc.unpack(grad.astype(np.float64))
        wg = oc.conv3_weight_grad
        check_sum_bound(g["W3"], wg(dy, h2), wg(np.abs(dy), np.abs(h2)), "W3")
        check_sum_bound(g["b3"], dy.sum(axis=(0, 1, 2, 3)), np.abs(dy).sum(axis=(0, 1, 2, 3)), "b3")
        check_sum_bound(g["W2"], wg(dz2, h1), wg(np.abs(dz2), np.abs(h1)), "W2")
        check_sum_bound(g["b2"], dz2.sum(axis=(0, 1, 2, 3)), np.abs(dz2).sum(axis=(0, 1, 2, 3)),
                        "b2")
        check_sum_bound(g["W1"], wg(dz1, xhi) + wg(dz1, xlo),
                        wg(np.abs(dz1), np.abs(xhi)) + wg(np.abs(dz1), np.abs(xlo)), "W1")
        check_sum_bound(g["b1"], dz1.sum(axis=(0, 1, 2, 3)), np.abs(dz1).sum(axis=(0, 1, 2, 3)),
                        "b1")
    gx = None
    if input_grad:
        gx = c.activation(9)
        ref = oc.conv3_input_grad(dz1, p["W1"])
        aref = oc.conv3_input_grad(np.abs(dz1), np.abs(p["W1"]))
        check_sum_bound(gx[:, :5], ref.reshape(-1, 5), aref.reshape(-1, 5), "dX hi")
        check_sum_bound(gx[:, 5:10], ref.reshape(-1, 5), aref.reshape(-1, 5), "dX lo")
        gx = B(gx[:, :5])
    return gx


def check_input_grad(gU, gres, gx, std, dtype, gres_err=0.0):
    """dL/dU = residual path + dX / std, from the GPU's dX: within two
    roundings of the state dtype of the magnitudes involved, plus gres_err,
    the bound of the residual path's own rounding differences."""
    ref = gres + np.moveaxis(gx, -1, 1) / std.reshape(1, 5, 1, 1, 1)
    mag = np.abs(gres) + np.abs(np.moveaxis(gx, -1, 1) / std.reshape(1, 5, 1, 1, 1))
    u = 2.0 ** -52 if dtype == "f64" else 2.0 ** -23
    err = np.abs(gU - ref)
    assert np.all(err <= 2 * u * mag + gres_err + 1e-300), float(err.max())


def loss_grad_rounding(U, y, scale, loss_w, std, batch, n):
    """Bound of the rounding differences of the loss gradient
    2 w (U + scale y - T) / (std^2 cells) between two fp64 evaluations: the
    corrected state U + scale y may be formed with or without a fused
    multiply-add (one rounding of its magnitude each), and the rest of the
    expression is evaluated in the same order on both sides."""
    sy = np.moveaxis(to_oracle(y, batch, n), -1, 1) * scale.reshape(1, 5, 1, 1, 1)
    w = np.asarray(loss_w).reshape(1, 5, 1, 1, 1)
    s2 = (np.asarray(std) ** 2).reshape(1, 5, 1, 1, 1)
    return 4.0 * w * 2.0 ** -52 * (np.abs(U) + np.abs(sy)) / s2 / (batch * n ** 3)


@pytest.mark.parametrize("dtype", ["f32", "f64"])
def test_loss_and_gradient(dtype):
    n, batch = 16, 2
    U = batch_state(n, batch, 30, dtype)
    T = as_input(U + 0.02 * batch_state(n, batch, 40, "f64"), dtype)
    loss_w = np.array([4.0, 1.0, 1.0, 1.0, 1.0])
    c, th, mean, std, scale = make(n, batch, dtype, U, scale=(5e-2,) * 5, loss_w=loss_w)
    Ud, Td = torch_dev(U, dtype), torch_dev(T, dtype)
    L, g = c.loss_grad(Ud, Td)
    L2, g2 = c.loss_grad(Ud, Td)
    assert L == L2 and np.array_equal(g, g2)  # deterministic reductions
    Lref, gref = oracle_grad_from_gpu(c, U, T, th, std, scale, loss_w, batch, n)
    assert L == pytest.approx(Lref, rel=1e-9)
    # element by element, each step of the reverse pass on the GPU's inputs
    y = c.activation(5)[:, :5]
    Uc = U + np.moveaxis(to_oracle(y, batch, n), -1, 1) * scale.reshape(1, 5, 1, 1, 1)
    _, gUc = oc.loss_and_grad_y(Uc, T, loss_w, std)
    check_reverse_pass(c, th, gUc, scale, batch, n, grad=g)
    # and in norm against the oracle's chained reverse pass
    for name, a, b in BLOCKS:
        tol = 1e-4 if name in ("W3", "b3") else 2e-3
        err = np.linalg.norm(g[a:b] - gref[a:b]) / np.linalg.norm(gref[a:b])
        assert err < tol, (name, err)
    # against the oracle's own forward + backward: same direction
    Uc, cache = oc.forward(U, th, mean, std, scale)
    _, gUc = oc.loss_and_grad_y(Uc, T, loss_w, std)
    gown = oc.backward(gUc, cache, scale)
    cos = float(g @ gown / (np.linalg.norm(g) * np.linalg.norm(gown)))
    assert cos > 0.9999


@pytest.mark.parametrize("dtype", ["f32", "f64"])
def test_input_gradient_and_accumulation(dtype):
    n, batch = 16, 2
    U = batch_state(n, batch, 90, dtype)
    T = as_input(U + 0.02 * batch_state(n, batch, 91, "f64"), dtype)
    gup = as_input(1e-3 * np.random.default_rng(92).standard_normal(U.shape), dtype)
    loss_w = np.array([4.0, 1.0, 1.0, 1.0, 1.0])
    c, th, mean, std, scale = make(n, batch, dtype, U, scale=(5e-2,) * 5, loss_w=loss_w)
    Ud, Td, Gd = torch_dev(U, dtype), torch_dev(T, dtype), torch_dev(gup, dtype)
    c.zero_grad()
    L, gU = c.backward(Ud, Td, Gd, want_loss=True, input_grad=True)
    g1 = c.grad()
    # the oracle's reverse pass on the GPU's activations, upstream = loss + gup
    p = {k: oc.bf16_round(v) if k.startswith("W") else v for k, v in oc.unpack(th).items()}
    x0 = c.activation(0)
    y = c.activation(5)[:, :5]
    cache = dict(x=to_oracle(x0[:, :5] + x0[:, 5:10], batch, n),
                 z1=to_oracle(c.activation(1), batch, n), h1=to_oracle(c.activation(2), batch, n),
                 z2=to_oracle(c.activation(3), batch, n), h2=to_oracle(c.activation(4), batch, n),
                 y=to_oracle(y, batch, n), p=p, rd=oc.bf16_round)
    Uc = U + np.moveaxis(to_oracle(y, batch, n), -1, 1) * scale.reshape(1, 5, 1, 1, 1)
    Lref, gl = oc.loss_and_grad_y(Uc, T, loss_w, std)
    gref = oc.backward(gl + gup, cache, scale)
    gUref = oc.input_grad(gl + gup, cache, std)
    assert L == pytest.approx(Lref, rel=1e-9)
    gx = check_reverse_pass(c, th, gl + gup, scale, batch, n, grad=g1, input_grad=True)
    gU = gU.cpu().numpy()
    check_input_grad(gU, gl + gup, gx, std, dtype,
                     loss_grad_rounding(U, y, scale, loss_w, std, batch, n))
    assert np.linalg.norm(g1 - gref) / np.linalg.norm(gref) < 2e-3
    assert np.linalg.norm(gU - gUref) / np.linalg.norm(gUref) < 2e-3
    # the network path is a visible part of dL/dU
    assert np.linalg.norm(gUref - (gl + gup)) > 1e-2 * np.linalg.norm(gUref)
    # a second pass accumulates: exactly twice the gradient
    c.backward(Ud, Td, Gd)
    assert np.array_equal(c.grad(), 2 * g1)
    c.zero_grad()
    assert not c.grad().any()


def test_adam_step_and_training_reduces_loss():
    n, batch = 16, 2
    U = batch_state(n, batch, 50, "f32")
    T = as_input(U + 0.02 * batch_state(n, batch, 60, "f64"), "f32")
    c, th, mean, std, scale = make(n, batch, "f32", U, scale=(5e-2,) * 5)
    Ud, Td = torch_dev(U, "f32"), torch_dev(T, "f32")
    L0, g = c.loss_grad(Ud, Td)
    lr = 1e-3
    L0b = c.train_step(Ud, Td, lr)
    assert L0b == L0
    ref, _, _ = oc.adam(th, np.zeros_like(th), np.zeros_like(th), g.astype(np.float64), 1, lr)
    assert np.abs(c.params() - ref).max() < 1e-6
    losses = [c.train_step(Ud, Td, lr) for _ in range(30)]
    assert losses[-1] < 0.5 * L0


@pytest.mark.parametrize("dtype", ["f32", "f64"])
def test_floor_and_fallback(dtype):
    n, batch = 16, 2
    U = batch_state(n, batch, 70, dtype)
    scale = np.array([2.0, 0.0, 0.0, 0.0, 2.0])
    # no fallback: the floored state against the oracle floor on the GPU's y
    c, th, mean, std, _ = make(n, batch, dtype, U, scale=scale, fallback_frac=1.0)
    out, nfl, fb = c.apply(torch_dev(U, dtype))
    # y from the training forward (inference does not store it)
    c.loss_grad(torch_dev(U, dtype), torch_dev(U, dtype))
    y = c.activation(5)[:, :5]
    Uc = U + np.moveaxis(to_oracle(y, batch, n), -1, 1) * scale.reshape(1, 5, 1, 1, 1)
    Uc = as_input(Uc, dtype)
    ref, nref, bad = oc.floor_and_check(U, Uc, GAMMA)
    assert nref > 0 and nfl == nref and not fb and not bad
    tol = 1e-15 if dtype == "f64" else 2e-7
    assert rel_inf(out.cpu().numpy(), ref) < tol
    # too many floored cells: the plain state comes back unchanged
    c2, *_ = make(n, batch, dtype, U, scale=scale, fallback_frac=1e-3, theta=th)
    out2, nfl2, fb2 = c2.apply(torch_dev(U, dtype))
    assert fb2 and nfl2 == nref and np.array_equal(out2.cpu().numpy(), U)
    # the enqueue-only form makes the same choice on the device
    out2b, none1, none2 = c2.apply(torch_dev(U, dtype), stats=False)
    assert none1 is None and none2 is None and np.array_equal(out2b.cpu().numpy(), U)
    # non-finite parameters: fallback as well
    bad_th = th.copy()
    bad_th[-1] = np.nan
    c3, *_ = make(n, batch, dtype, U, fallback_frac=1.0, theta=bad_th)
    out3, _, fb3 = c3.apply(torch_dev(U, dtype))
    assert fb3 and np.array_equal(out3.cpu().numpy(), U)


@pytest.mark.parametrize("dtype", ["f32", "f64"])
@pytest.mark.parametrize("r", [2, 4])
def test_block_average(dtype, r):
    nf = 32
    F = as_input(wl.random_state((nf, nf, nf), seed=80), dtype)
    got = mh.block_average(torch_dev(F, dtype), r).cpu().numpy()
    nc = nf // r
    ref = F.reshape(5, nc, r, nc, r, nc, r).mean(axis=(2, 4, 6))
    assert rel_inf(got, ref) < (1e-15 if dtype == "f64" else 2e-7)
    # conservation: the coarse totals times r^3 are the fine totals
    assert np.allclose(got.astype(np.float64).sum(axis=(1, 2, 3)) * r ** 3, F.sum(axis=(1, 2, 3)),
                       rtol=1e-6)


@pytest.mark.parametrize("dtype", ["f32", "f64"])
def test_flux_mode_output_and_gradients(dtype):
    """Flux mode: the output is scale * Net(U) alone, and the reverse pass has
    no residual term in dL/dU."""
    n, batch = 16, 2
    U = batch_state(n, batch, 130, dtype)
    gup = as_input(1e-3 * np.random.default_rng(131).standard_normal(U.shape), dtype)
    mean, std = stats(U)
    scale = np.array([2e-2, 1e-2, 1e-2, 1e-2, 3e-2])
    d = mh.corr_desc(n, batch, dtype, GAMMA, mean, std, scale, (1.0,) * 5, 1e-6, 1e-3,
                     mode=mh.CORR_FLUX)
    c = mh.Corrector(d)
    th = params(seed=3)
    c.set_params(th)
    Ud, Gd = torch_dev(U, dtype), torch_dev(gup, dtype)
    out, nfl, fb = c.apply(Ud)
    assert nfl == 0 and not fb
    y = c.activation(5)[:, :5]
    ref = np.moveaxis(to_oracle(y, batch, n), -1, 1) * scale.reshape(1, 5, 1, 1, 1)
    assert np.array_equal(out.cpu().numpy(), as_input(ref, dtype))
    # the same network in state mode gives U + the same correction
    ds = mh.corr_desc(n, batch, dtype, GAMMA, mean, std, scale, (1.0,) * 5, 1e-6, 1e-3)
    cs = mh.Corrector(ds)
    cs.set_params(th)
    outs, _, _ = cs.apply(Ud)
    cs.loss_grad(Ud, Ud)  # the training forward stores y (inference does not)
    assert np.array_equal(cs.activation(5), c.activation(5))
    tol = 1e-15 if dtype == "f64" else 2e-7
    assert rel_inf(outs.cpu().numpy(), U + out.cpu().numpy()) < tol
    # reverse pass with an upstream gradient against the oracle's
    c.zero_grad()
    _, gU = c.backward(Ud, gUc=Gd, input_grad=True)
    p = {k: oc.bf16_round(v) if k.startswith("W") else v for k, v in oc.unpack(th).items()}
    x0 = c.activation(0)
    cache = dict(x=to_oracle(x0[:, :5] + x0[:, 5:10], batch, n),
                 z1=to_oracle(c.activation(1), batch, n), h1=to_oracle(c.activation(2), batch, n),
                 z2=to_oracle(c.activation(3), batch, n), h2=to_oracle(c.activation(4), batch, n),
                 y=to_oracle(c.activation(5)[:, :5], batch, n), p=p, rd=oc.bf16_round)
    gref = oc.backward(gup, cache, scale)
    gx = check_reverse_pass(c, th, gup, scale, batch, n, grad=c.grad(), input_grad=True)
    gU = gU.cpu().numpy()
    check_input_grad(gU, np.zeros_like(gup), gx, std, dtype)
    assert np.linalg.norm(c.grad() - gref) / np.linalg.norm(gref) < 2e-3
    gUref = oc.input_grad(gup, cache, std) - gup
    assert np.linalg.norm(gU - gUref) / np.linalg.norm(gUref) < 2e-3
    # training against a target is a state-mode operation
    with pytest.raises(mh.MHError):
        c.backward(Ud, Ud)
    with pytest.raises(mh.MHError):
        c.loss_grad(Ud, Ud)
