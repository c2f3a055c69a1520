"""Oracle of the learned state corrector (test infrastructure only).

The paper embeds a convolutional network in the solver loop and trains it
through the solver (Sec. 8, solver-in-the-loop: U^{n+1} = H(U^n, B_theta)),
with periodic padding and an MSE loss that weights density up.  The corrector
built here is a 3D state corrector applied after each coarse step:

    x  = (U - mean) / std                     (per channel, 5 -> 5)
    h1 = GELU(conv3(x;  W1) + b1)             (5 -> 32)
    h2 = GELU(conv3(h1; W2) + b2)             (32 -> 32)
    y  = conv3(h2; W3) + b3                   (32 -> 5)
    U' = U + scale * y

conv3 is a 3x3x3 cross-correlation with periodic padding; GELU is the erf
form x (1 + erf(x / sqrt 2)) / 2.  The GPU computes with bf16 operands and
fp32 accumulation; this oracle rounds the same operands to bf16 (round to
nearest even) at the same points -- the weights, the stored activations h1,
h2 -- and accumulates in float64.  The standardised input is carried as the
sum of two bf16 numbers, x = x_hi + x_lo with x_hi = bf16(x32) and x_lo =
bf16(x32 - x_hi), x32 the float32 value: about 16 significant bits, so the
first layer sees the state's small-scale structure (a single bf16 would round
it away at 2^-8 of the channel's spread).  Both parts go through the same
first-layer weights.

Tap order: t = 9 (dz + 1) + 3 (dy + 1) + (dx + 1), reading input at
(x + dx, y + dy, z + dz).  Arrays are [batch][z][y][x][channel].
Parameters, in their canonical flat order: W1[32][5][27], b1[32],
W2[32][32][27], b2[32], W3[5][32][27], b3[5] (36 357 values).
"""
from __future__ import annotations

import math

import numpy as np
from scipy.special import erf

SHAPES = [("W1", (32, 5, 27)), ("b1", (32,)), ("W2", (32, 32, 27)), ("b2", (32,)),
          ("W3", (5, 32, 27)), ("b3", (5,))]
NPARAM = sum(int(np.prod(s)) for _, s in SHAPES)

TAPS = [(dx, dy, dz) for dz in (-1, 0, 1) for dy in (-1, 0, 1) for dx in (-1, 0, 1)]


def bf16_round(x):
    """Round to the nearest bfloat16 (ties to even), returned as float64."""
    f = np.asarray(x, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    r = ((u + 0x7FFF + lsb) & 0xFFFF0000).astype(np.uint32)
    return r.view(np.float32).astype(np.float64)


def split_parts(x):
    """(x_hi, x_lo) of the two-part bf16 input: x_hi = bf16(x32), x_lo =
    bf16(x32 - x_hi) with x32 = float32(x) (the difference is exact in
    float32)."""
    x32 = np.asarray(x, dtype=np.float32).astype(np.float64)
    hi = bf16_round(x32)
    return hi, bf16_round(x32 - hi)


def split_bf16(x):
    hi, lo = split_parts(x)
    return hi + lo


def unpack(theta):
    out, o = {}, 0
    for name, shp in SHAPES:
        k = int(np.prod(shp))
        out[name] = np.asarray(theta[o:o + k], dtype=np.float64).reshape(shp)
        o += k
    return out


def pack(p):
    return np.concatenate([np.asarray(p[name], dtype=np.float64).ravel() for name, _ in SHAPES])


def gelu(z):
    return 0.5 * z * (1.0 + erf(z / math.sqrt(2.0)))


def gelu_grad(z):
    return 0.5 * (1.0 + erf(z / math.sqrt(2.0))) + z * np.exp(-0.5 * z * z) / math.sqrt(2.0 * math.pi)


def shift(x, dx, dy, dz):
    """x'[.., z, y, x, :] = x[.., z + dz, y + dy, x + dx, :] with periodic wrap."""
    return np.roll(x, shift=(-dz, -dy, -dx), axis=(1, 2, 3))


def conv3(x, W, b=None):
    """y[., c_out] = sum_t sum_ci W[c_out, ci, t] x[. + off_t, ci] (+ b)."""
    B, nz, ny, nx, _ = x.shape
    y = np.zeros((B, nz, ny, nx, W.shape[0]))
    for t, (dx, dy, dz) in enumerate(TAPS):
        y += shift(x, dx, dy, dz) @ W[:, :, t].T
    if b is not None:
        y += b
    return y


def conv3_input_grad(gy, W):
    """Adjoint of conv3 in its input: gx[p] = sum_t W[:, :, t]^T gy[p - off_t]."""
    gx = np.zeros(gy.shape[:4] + (W.shape[1],))
    for t, (dx, dy, dz) in enumerate(TAPS):
        gx += shift(gy, -dx, -dy, -dz) @ W[:, :, t]
    return gx


def conv3_weight_grad(gy, x):
    """dW[c_out, ci, t] = sum_p gy[p, c_out] x[p + off_t, ci]."""
    co, ci = gy.shape[-1], x.shape[-1]
    gW = np.zeros((co, ci, 27))
    g2 = gy.reshape(-1, co)
    for t, (dx, dy, dz) in enumerate(TAPS):
        gW[:, :, t] = g2.T @ shift(x, dx, dy, dz).reshape(-1, ci)
    return gW


def forward(U, theta, mean, std, scale, rounding=True):
    """U: [batch][5][z][y][x] float64.  Returns (U', cache).  rounding=False
    skips the bf16 roundings (exact arithmetic, for derivative checks)."""
    rd = bf16_round if rounding else (lambda a: np.asarray(a, dtype=np.float64))
    p = {k: rd(v) if k.startswith("W") else v for k, v in unpack(theta).items()}
    x = (np.moveaxis(U, 1, -1) - np.asarray(mean)) / np.asarray(std)
    if rounding:
        x = split_bf16(x)
    z1 = conv3(x, p["W1"], p["b1"])
    h1 = rd(gelu(z1))
    z2 = conv3(h1, p["W2"], p["b2"])
    h2 = rd(gelu(z2))
    y = conv3(h2, p["W3"], p["b3"])
    Uc = U + np.moveaxis(y * np.asarray(scale), -1, 1)
    return Uc, dict(x=x, z1=z1, h1=h1, z2=z2, h2=h2, y=y, p=p, rd=rd)


def loss_and_grad_y(Uc, T, weights, sigma):
    """L = sum_c w_c mean((Uc_c - T_c)^2) / sigma_c^2 and dL/dUc."""
    w = np.asarray(weights).reshape(1, 5, 1, 1, 1)
    s2 = (np.asarray(sigma) ** 2).reshape(1, 5, 1, 1, 1)
    ncell = Uc[:, 0].size
    d = Uc - T
    L = float((w * d * d / s2).sum() / ncell)
    return L, 2.0 * w * d / s2 / ncell


def backward(gUc, cache, scale):
    """Gradient of the loss w.r.t. the parameters (canonical flat order) from
    gUc = dL/dU'.  Activation gradients are rounded to bf16 where the GPU feeds
    them to its matrix cores (dY, dZ2, dZ1), weights as in the forward; dZ1 is
    left in the cache for input_grad."""
    p, rd = cache["p"], cache["rd"]
    gy = rd(np.moveaxis(gUc, 1, -1) * np.asarray(scale))
    g = {}
    g["W3"] = conv3_weight_grad(gy, cache["h2"])
    g["b3"] = gy.sum(axis=(0, 1, 2, 3))
    gh2 = conv3_input_grad(gy, p["W3"])
    gz2 = rd(gh2 * gelu_grad(cache["z2"]))
    g["W2"] = conv3_weight_grad(gz2, cache["h1"])
    g["b2"] = gz2.sum(axis=(0, 1, 2, 3))
    gh1 = conv3_input_grad(gz2, p["W2"])
    gz1 = rd(gh1 * gelu_grad(cache["z1"]))
    g["W1"] = conv3_weight_grad(gz1, cache["x"])
    g["b1"] = gz1.sum(axis=(0, 1, 2, 3))
    cache["gz1"] = gz1
    return pack(g)


def input_grad(gUc, cache, std):
    """dL/dU after backward(): the residual path gUc plus the network path
    (W1^T conv of dZ1) divided by the standardisation std.  The two-part bf16
    split of the input is passed through as the identity (its parts sum to x
    up to rounding)."""
    gx = conv3_input_grad(cache["gz1"], cache["p"]["W1"])
    return gUc + np.moveaxis(gx, -1, 1) / np.asarray(std).reshape(1, 5, 1, 1, 1)


def adam(theta, m, v, grad, it, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One ADAM update (Kingma & Ba 2015), iteration it >= 1 (paper Sec. 7)."""
    m = b1 * m + (1.0 - b1) * grad
    v = b2 * v + (1.0 - b2) * grad * grad
    mh = m / (1.0 - b1 ** it)
    vh = v / (1.0 - b2 ** it)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v


def floor_and_check(U, Uc, gamma, floor_rel=1e-6):
    """Positivity floor after the correction: rho >= floor_rel <rho>, then
    P >= floor_rel <P> by raising E at fixed momentum (means of the uncorrected
    state U, per sample).  Returns (floored state, number of floored cells,
    any non-finite value)."""
    out = np.array(Uc, dtype=np.float64, copy=True)
    nfl = 0
    for b in range(U.shape[0]):
        rho0 = U[b, 0]
        p0 = (gamma - 1.0) * (U[b, 4] - 0.5 * (U[b, 1] ** 2 + U[b, 2] ** 2 + U[b, 3] ** 2) / rho0)
        rf = floor_rel * rho0.mean()
        pf = floor_rel * p0.mean()
        r = out[b, 0]
        low = r < rf
        r[low] = rf
        ek = 0.5 * (out[b, 1] ** 2 + out[b, 2] ** 2 + out[b, 3] ** 2) / r
        p = (gamma - 1.0) * (out[b, 4] - ek)
        lowp = p < pf
        out[b, 4][lowp] = ek[lowp] + pf / (gamma - 1.0)
        nfl += int((low | lowp).sum())
    return out, nfl, bool(not np.all(np.isfinite(out)))
