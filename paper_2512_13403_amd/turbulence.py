"""Spectral turbulent initial conditions with the mode phases as control
variables (the construction of Sec. 3.1, used as the parametrisation of the
turbulence reconstruction of Sec. 7).

On the FFT grid of an n^3 periodic box (integer wavenumbers k in the order of
the state arrays, x fastest) each velocity component gets the coefficients
    X_i(k) = A(k) sum_j M_ij(k) exp(i phi_j(k)),
    A(k) = |k|^(p/2) for kmin <= |k| <= kmax, else 0   (the power-law band),
    M = zeta P + (1 - zeta) C,  C_ij = k_i k_j / |k|^2,  P = 1 - C
(the solenoidal / compressive mixture), the real part of the unnormalised
inverse transform gives u_i, and the field is rescaled to the target rms
Mach number, v = Mach c_s u / rms|u|, before the conserved state is assembled
at uniform density and pressure.  Only the phases phi_j(k) are free.

The transforms run in the library (``mh_fft3``); the reverse pass of the
phase-to-velocity map is written out: with g = dL/du and G_i = FFT(g_i)
(forward, unnormalised), dL/dphi_j = A (cos phi_j Im H_j - sin phi_j Re H_j),
H_j = sum_i M_ij G_i.  The Mach rescaling and the state assembly are
elementwise torch operations.
"""
from __future__ import annotations

import math

import numpy as np

from . import Adam, fft3
from .inversion import misfit
from .rollout import make_rollout_function


def spectral_basis(n, kmin, kmax, power, zeta, dtype, device):
    """A(k) [n][n][n] and the six entries of the symmetric M(k), as torch
    tensors (index order (kz, ky, kx))."""
    import torch

    k1 = np.fft.fftfreq(n, d=1.0 / n)
    kz, ky, kx = np.meshgrid(k1, k1, k1, indexing="ij")
    ks = (kx, ky, kz)
    k2 = kx * kx + ky * ky + kz * kz
    k = np.sqrt(k2)
    band = (k >= kmin) & (k <= kmax)
    A = np.zeros_like(k)
    A[band] = k[band] ** (power / 2.0)
    k2s = np.where(k2 > 0, k2, 1.0)
    M = {}
    for i in range(3):
        for j in range(i, 3):
            C = ks[i] * ks[j] / k2s
            M[(i, j)] = zeta * ((1.0 if i == j else 0.0) - C) + (1.0 - zeta) * C
    t = lambda a: torch.tensor(a, dtype=dtype, device=device)
    return t(A), {key: t(v) for key, v in M.items()}


def _m(M, i, j):
    return M[(i, j)] if i <= j else M[(j, i)]


def _velocity_from_phases(phases, A, M):
    """u_i = Re IFFT(X_i) for phases [3][n][n][n] (no autograd)."""
    import torch

    c, s = torch.cos(phases), torch.sin(phases)
    u = []
    for i in range(3):
        X = torch.zeros(phases.shape[1:] + (2,), dtype=phases.dtype, device=phases.device)
        for j in range(3):
            m = A * _m(M, i, j)
            X[..., 0] += m * c[j]
            X[..., 1] += m * s[j]
        u.append(fft3(X.contiguous(), inverse=True)[..., 0].clone())
    return torch.stack(u)


def _phase_gradient(phases, A, M, g):
    """dL/dphi for dL/du = g [3][n][n][n] (the written-out reverse pass)."""
    import torch

    G = []
    for i in range(3):
        Z = torch.zeros(g.shape[1:] + (2,), dtype=g.dtype, device=g.device)
        Z[..., 0] = g[i]
        G.append(fft3(Z.contiguous(), inverse=False))
    out = torch.empty_like(phases)
    for j in range(3):
        Hr = sum(_m(M, i, j) * G[i][..., 0] for i in range(3))
        Hi = sum(_m(M, i, j) * G[i][..., 1] for i in range(3))
        out[j] = A * (torch.cos(phases[j]) * Hi - torch.sin(phases[j]) * Hr)
    return out


def make_phase_velocity_function():
    """torch.autograd.Function phases -> u (before the Mach rescaling)."""
    import torch

    class PhaseVelocity(torch.autograd.Function):
        @staticmethod
        def forward(ctx, phases, A, M6):
            M = dict(zip(((0, 0), (0, 1), (0, 2), (1, 1), (1, 2), (2, 2)), M6))
            ctx.save_for_backward(phases)
            ctx.A, ctx.M = A, M
            return _velocity_from_phases(phases.detach(), A, M)

        @staticmethod
        def backward(ctx, g):
            (phases,) = ctx.saved_tensors
            return _phase_gradient(phases.detach(), ctx.A, ctx.M, g.contiguous()), None, None

    return PhaseVelocity


def initial_state(phases, basis, mach=1.0, rho0=1.0, p0=1.0, gamma=5.0 / 3.0):
    """Conserved state [5][n][n][n] of the phase-parametrised turbulent field
    (differentiable with respect to phases)."""
    import torch

    A, M = basis
    M6 = tuple(M[k] for k in ((0, 0), (0, 1), (0, 2), (1, 1), (1, 2), (2, 2)))
    u = make_phase_velocity_function().apply(phases, A, M6)
    cs = math.sqrt(gamma * p0 / rho0)
    v = u * (mach * cs / torch.sqrt((u * u).sum(dim=0).mean()))
    rho = torch.full_like(u[0], rho0)
    E = p0 / (gamma - 1.0) + 0.5 * rho0 * (v * v).sum(dim=0)
    return torch.cat([rho.unsqueeze(0), rho0 * v, E.unsqueeze(0)], dim=0).contiguous()


def invert_turbulent_phases(solver, phases_init, target, dts, basis, iters=30, lr=0.1, K=10,
                            kind="projected", mach=1.0, rho0=1.0, p0=1.0, callback=None):
    """ADAM on the phases so that len(dts) steps with the fixed time steps dts
    end with a density matching `target` (a z-projected map for "projected",
    a cube for "l2").  Returns (optimised phases, misfit before each
    iteration)."""
    import torch

    gamma = solver.grid.gamma
    phases = phases_init.detach().clone().contiguous().requires_grad_(True)
    opt = Adam(phases.data, lr=lr)
    F = make_rollout_function()
    dts = np.asarray(dts, dtype=np.float64)
    losses = []
    for it in range(iters):
        phases.grad = None
        U0 = initial_state(phases, basis, mach, rho0, p0, gamma)
        Uf = F.apply(U0, solver, len(dts), K, dts)
        loss = misfit(Uf[0], target, kind)
        loss.backward()
        losses.append(float(loss.detach()))
        opt.step(phases.grad)
        if callback is not None:
            callback(it, losses[-1])
    return phases.detach(), losses
