"""Seeded synthetic inputs for the diffhydro finite-volume workloads.

This module is shared by the tests, the benchmark, the oracle runs and the HIP
runs.  It only builds initial states from seeded random numbers and the
problem definitions; it holds none of the solver's arithmetic (no fluxes,
reconstruction, time stepping or sources).  The one formula it shares with the
solver is the initial-condition assembly E = P/(gamma-1) + rho |v|^2 / 2 of
the paper's Sec. 3.1 (eq:turbic), which defines the input, not the method.

States are float64 arrays of shape (5, nz, ny, nx), fields (rho, m_x, m_y,
m_z, E), x fastest.  Every generator takes an explicit seed and uses
``numpy.random.default_rng(seed)``.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

PERIODIC, OUTFLOW = 0, 1


@dataclass(frozen=True)
class Grid:
    """Uniform grid: shape = (nz, ny, nx), spacing h = (hx, hy, hz), boundary
    kind per axis (x, y, z)."""

    shape: tuple
    h: tuple
    bc: tuple = (PERIODIC, PERIODIC, PERIODIC)

    @property
    def cells(self) -> int:
        return int(np.prod(self.shape))


def cube(n: int, length: float = 1.0) -> Grid:
    return Grid((n, n, n), (length / n,) * 3)


def conserved(rho, vx, vy, vz, p, gamma):
    """Initial-condition assembly (paper Sec. 3.1, eq:turbic)."""
    rho = np.asarray(rho, dtype=np.float64)
    E = p / (gamma - 1.0) + 0.5 * rho * (vx * vx + vy * vy + vz * vz)
    return np.ascontiguousarray(np.stack([rho, rho * vx, rho * vy, rho * vz,
                                          np.broadcast_to(E, rho.shape)]).astype(np.float64))


def centres(n: int):
    return (np.arange(n) + 0.5) / n


# ---------------------------------------------------------------- Sod tube

def sod_grid(nx: int = 128, ny: int = 16, nz: int = 16) -> Grid:
    """Sod tube along x on [0,1] with dx = 1/nx, transmissive in x, periodic in
    y and z (the transverse extent uses the same spacing)."""
    h = 1.0 / nx
    return Grid((nz, ny, nx), (h, h, h), (OUTFLOW, PERIODIC, PERIODIC))


def sod_state(grid: Grid, gamma: float = 1.4, left=(1.0, 0.0, 1.0), right=(0.125, 0.0, 0.1),
              x0: float = 0.5):
    nz, ny, nx = grid.shape
    x = (np.arange(nx) + 0.5) * grid.h[0]
    L = x < x0
    rho = np.where(L, left[0], right[0])
    u = np.where(L, left[1], right[1])
    p = np.where(L, left[2], right[2])
    b = lambda a: np.broadcast_to(a, (nz, ny, nx)).copy()
    z = np.zeros((nz, ny, nx))
    return conserved(b(rho), b(u), z, z, b(p), gamma)


# ---------------------------------------------------------------- KH

def kh_state(n: int, gamma: float = 5.0 / 3.0, seed: int = 0, noise: float = 1e-3):
    """3D Kelvin-Helmholtz: rho=2, vx=+0.5 in the band |y-0.5|<0.25, else rho=1,
    vx=-0.5; p=2.5; vy = 0.01 sin(4 pi x); vx and vy get seeded uniform noise
    noise*(2U-1) (vx drawn first); vz = 0."""
    rng = np.random.default_rng(seed)
    x = centres(n)[None, None, :]
    y = centres(n)[None, :, None]
    band = np.abs(y - 0.5) < 0.25
    shape = (n, n, n)
    rho = np.broadcast_to(np.where(band, 2.0, 1.0), shape).copy()
    vx = np.broadcast_to(np.where(band, 0.5, -0.5), shape).copy()
    vy = np.broadcast_to(0.01 * np.sin(4.0 * np.pi * x), shape).copy()
    vx += noise * (2.0 * rng.random(shape) - 1.0)
    vy += noise * (2.0 * rng.random(shape) - 1.0)
    return conserved(rho, vx, vy, np.zeros(shape), np.full(shape, 2.5), gamma)


# ---------------------------------------------------------------- uniform / random

def rest_state(shape, rho: float = 1.0, p: float = 1.0, gamma: float = 5.0 / 3.0, v=(0.0, 0.0, 0.0)):
    z = np.zeros(shape)
    return conserved(np.full(shape, rho), z + v[0], z + v[1], z + v[2], np.full(shape, p), gamma)


def random_state(shape, seed: int, gamma: float = 5.0 / 3.0, rho=(0.5, 1.5), p=(0.5, 1.5),
                 vmax: float = 1.0):
    """Cell-wise independent random primitives: rough on purpose, so every
    limiter branch and every HLLC wave region occurs."""
    rng = np.random.default_rng(seed)
    r = rng.uniform(rho[0], rho[1], shape)
    v = rng.uniform(-vmax, vmax, (3,) + tuple(shape))
    pp = rng.uniform(p[0], p[1], shape)
    return conserved(r, v[0], v[1], v[2], pp, gamma)


def smooth_random_state(shape, seed: int, gamma: float = 5.0 / 3.0, kmax: int = 3,
                        amp_rho: float = 0.3, amp_v: float = 0.5, amp_p: float = 0.3):
    """Smooth periodic random primitives made of a few low Fourier modes."""
    rng = np.random.default_rng(seed)
    nz, ny, nx = shape
    z, y, x = np.meshgrid(centres(nz), centres(ny), centres(nx), indexing="ij")

    def field():
        f = np.zeros(shape)
        for _ in range(6):
            k = rng.integers(-kmax, kmax + 1, 3)
            ph = rng.uniform(0, 2 * np.pi)
            f += np.cos(2 * np.pi * (k[0] * x + k[1] * y + k[2] * z) + ph)
        return f / 6.0

    rho = 1.0 + amp_rho * field()
    v = [amp_v * field() for _ in range(3)]
    p = 1.0 + amp_p * field()
    return conserved(rho, v[0], v[1], v[2], p, gamma)


# ---------------------------------------------------------------- turbulence ICs

def _kgrid(n):
    k1 = np.fft.fftfreq(n, d=1.0 / n)
    kz, ky, kx = np.meshgrid(k1, k1, k1, indexing="ij")
    return kx, ky, kz


def turbulent_velocity_state(n: int, seed: int = 0, kmin: float = 2.0, kmax: float = 20.0,
                             power: float = -5.0 / 3.0, zeta: float = 1.0, mach: float = 1.0,
                             rho0: float = 1.0, p0: float = 1.0, gamma: float = 5.0 / 3.0):
    """Band-limited Gaussian velocity field (paper Sec. 3.1: mode band
    kmin <= |n| <= kmax, amplitude k^(p/2) (eq:turbpl), mixed projection
    zeta P + (1-zeta) C (eq:turbproj), rescaled to the rms Mach number
    (eq:turbscale), assembled by eq:turbic).  Hermitian symmetry comes from
    transforming real white noise."""
    rng = np.random.default_rng(seed)
    kx, ky, kz = _kgrid(n)
    k2 = kx * kx + ky * ky + kz * kz
    k = np.sqrt(k2)
    band = (k >= kmin) & (k <= kmax)
    amp = np.zeros_like(k)
    amp[band] = k[band] ** (power / 2.0)
    G = [np.fft.fftn(rng.standard_normal((n, n, n))) for _ in range(3)]
    ks = (kx, ky, kz)
    k2s = np.where(k2 > 0, k2, 1.0)
    uh = []
    for i in range(3):
        s = np.zeros_like(G[0])
        for j in range(3):
            C = ks[i] * ks[j] / k2s
            P = (1.0 if i == j else 0.0) - C
            s = s + (zeta * P + (1.0 - zeta) * C) * G[j]
        uh.append(s * amp)
    u = [np.real(np.fft.ifftn(x)) for x in uh]
    cs = math.sqrt(gamma * p0 / rho0)
    urms = math.sqrt(np.mean(u[0] ** 2 + u[1] ** 2 + u[2] ** 2))
    alpha = mach * cs / urms
    shape = (n, n, n)
    return conserved(np.full(shape, rho0), alpha * u[0], alpha * u[1], alpha * u[2],
                     np.full(shape, p0), gamma)


def grf_density_state(n: int, seed: int = 0, amp: float = 0.1, power: float = -3.0,
                      p0: float = 1.0, gamma: float = 5.0 / 3.0):
    """rho = 1 + amp*g with g a unit-rms Gaussian random field of power
    spectrum k^power (k = 0 removed), at rest with uniform pressure."""
    rng = np.random.default_rng(seed)
    kx, ky, kz = _kgrid(n)
    k = np.sqrt(kx * kx + ky * ky + kz * kz)
    filt = np.zeros_like(k)
    filt[k > 0] = k[k > 0] ** (power / 2.0)
    g = np.real(np.fft.ifftn(np.fft.fftn(rng.standard_normal((n, n, n))) * filt))
    g /= math.sqrt(np.mean(g * g))
    shape = (n, n, n)
    z = np.zeros(shape)
    return conserved(1.0 + amp * g, z, z, z, np.full(shape, p0), gamma)


# ---------------------------------------------------------------- workload presets

COOLING_CURVE = dict(lambda0=0.3, tc=1e-2, ts=1e-3, tfloor=1e-4)
"""Synthetic two-branch cooling curve for the driven-turbulence workload, in
code units with T = P/rho (T = 1e-2 corresponds to 1e4 K at T[K] = 1e6 P/rho):
Lambda = L0 (T/Tc)^(1/2) above Tc and L0 exp((T-Tc)/Ts) below; floor Tfloor."""

def synthetic_cie_table():
    """Synthetic stand-in for the tabulated CIE cooling curve of the paper's
    model (its SD93 table is not available), in code units T = P/rho (T = 1e-2
    is 1e4 K): 17 points log10 T = -2 .. 2, a peak of log10 Lambda near
    log10 T = -0.8 (about 1.6e5 K), a decline above it and a T^(1/2) rise
    above log10 T = 0.5.  Returns (log10 T, log10 Lambda)."""
    x = np.linspace(-2.0, 2.0, 17)
    y = (math.log10(0.3) + 1.0 * np.exp(-((x + 0.8) / 0.45) ** 2) - 0.3 * np.maximum(0.0, x + 0.8)
         + 0.8 * np.maximum(0.0, x - 0.5))
    return x, y


COOLING_TABLE_MODEL = dict(cool_ki=(3000.0, 2.0, 0.003, 0.5), cool_heat=0.0272)
"""Low-temperature branch L1 T^a1 + L2 T^a2 of the tabulated model and its
heating rate Gamma_0 (code units): at rho = 1 heating balances cooling near
T = 3e-3 (3000 K), so denser gas cools further (the two-phase medium)."""

OU_DRIVE = dict(seed=0, tau=0.5, arms=1.0, zeta=1.0, kmin=1.0, kmax=2.0)
"""Solenoidal OU forcing on 1 <= |n| <= 2 with correlation time 0.5."""

JEANS_G = 9.0 * math.pi * (5.0 / 3.0)
"""G for a Jeans length of one third of the unit box at rho=1, p=1,
gamma=5/3: lambda_J = c_s sqrt(pi/(G rho)) = 1/3  =>  G = 9 pi gamma p / rho^2."""


def corrector_init_params(seed: int = 0, out_scale: float = 1e-3):
    """Seeded initial parameters of the 5 -> 32 -> 32 -> 5 conv corrector in
    its canonical flat order W1[32][5][27], b1[32], W2[32][32][27], b2[32],
    W3[5][32][27], b3[5]: He-normal hidden layers, a last layer scaled by
    out_scale (the corrector starts close to the identity map), zero biases."""
    rng = np.random.default_rng(seed)
    w1 = rng.standard_normal((32, 5, 27)) * math.sqrt(2.0 / (5 * 27))
    w2 = rng.standard_normal((32, 32, 27)) * math.sqrt(2.0 / (32 * 27))
    w3 = rng.standard_normal((5, 32, 27)) * out_scale * math.sqrt(1.0 / (32 * 27))
    return np.concatenate([w1.ravel(), np.zeros(32), w2.ravel(), np.zeros(32), w3.ravel(),
                           np.zeros(5)])

