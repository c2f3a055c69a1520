"""Shared helpers of the GPU parity tests: paired configurations for the HIP
library and the oracle, the relative field norm, and windowed oracle
evaluation of sampled cells of large grids."""
from __future__ import annotations

import math

import numpy as np

import oracle
import paper_2512_13403_amd as mh

PHYS_KEYS = ("cool", "ou_seed", "ou_tau", "ou_arms", "ou_zeta", "ou_kmin", "ou_kmax", "ou_every",
             "grav_G", "mg_pre", "mg_post", "mg_max_cycles", "mg_coarsest", "mg_tol",
             "mg_coarse_sweeps", "mg_cycle", "mg_smoother", "grav_solver", "cool_model",
             "cool_integrator", "cool_nsub_max", "cool_frac", "cool_ccool", "cool_ki", "cool_heat",
             "cool_table")


def pair(shape, h, bc=(0, 0, 0), dtype="f64", gamma=5.0 / 3.0, cfl=0.4, limiter=0, flags=0,
         riemann=0, integrator=0, **phys):
    """(Solver, oracle Config) for the same grid, scheme and physics (the
    binding's default smoother, red-black Gauss-Seidel, on both sides)."""
    phys.setdefault("mg_smoother", mh.SMOOTH_RBGS)
    g = mh.grid_desc(shape, h, bc, dtype, gamma, cfl, limiter, riemann, integrator)
    p = mh.physics_desc(flags=flags, **phys)
    oc = oracle.make_config(shape, h, bc, gamma=gamma, cfl=cfl, limiter=limiter, riemann=riemann,
                            flags=flags, integrator=integrator, **phys)
    return mh.Solver(g, p), oc


def as_input(U, dtype):
    """The exact values both sides start from: rounded to the GPU precision,
    handed to the oracle in float64."""
    if dtype == "f32":
        return U.astype(np.float32).astype(np.float64)
    return np.array(U, dtype=np.float64)


def rel_err(a, b):
    """max over fields f of ||a_f - b_f||_inf / D_f with D_rho = ||rho||_inf,
    D_E = ||E||_inf, D_m = sqrt(D_rho D_E)."""
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    Dr = np.abs(b[0]).max()
    DE = np.abs(b[4]).max()
    Dm = math.sqrt(Dr * DE)
    D = [Dr, Dm, Dm, Dm, DE]
    return max(float(np.abs(a[f] - b[f]).max()) / D[f] for f in range(5))


TOL = {"f64": 1e-12, "f32": 1e-5}


def window(U, i, j, k, r):
    """Periodic (2r+1)^3 window of U centred on cell (i, j, k) (x index i)."""
    nz, ny, nx = U.shape[1:]
    zi = np.arange(k - r, k + r + 1) % nz
    yi = np.arange(j - r, j + r + 1) % ny
    xi = np.arange(i - r, i + r + 1) % nx
    return np.ascontiguousarray(U[:, zi][:, :, yi][:, :, :, xi])


def oracle_step_sampled(oc, U, cells, dt, ahat=None, nvec=None):
    """Oracle result of one step at the given cells of a periodic grid.

    One RK2 step of a cell depends on the cross-shaped stencil of radius 2 of
    radius-2 stencils, so the oracle steps a periodic 9^3 window around the
    cell and keeps its centre, which the wrap of the small window cannot
    reach.  Forcing (at the cell's global position) and cooling are then
    applied to that centre cell exactly as in a full step."""
    r = 4
    wc = oracle.make_config((2 * r + 1,) * 3, tuple(oc.h), (0, 0, 0), gamma=oc.gamma,
                            cfl=oc.cfl, limiter=oc.limiter)
    one = oracle.make_config((1, 1, 1), tuple(oc.h), (0, 0, 0), gamma=oc.gamma,
                             cool=(oc.cool_lambda0, oc.cool_tc, oc.cool_ts, oc.cool_tfloor))
    out = np.empty((5, len(cells)))
    for s, (i, j, k) in enumerate(cells):
        V = oracle.rk2(wc, window(U, i, j, k, r), dt)[:, r:r + 1, r:r + 1, r:r + 1].copy()
        if oc.flags & oracle.SRC_FORCING:
            acc = oracle.ou_accel_at(oc, nvec, ahat, i, j, k).reshape(3, 1, 1, 1)
            V = oracle.kick(one, V, acc, dt)
        if oc.flags & oracle.SRC_COOLING:
            V = oracle.cool(one, V, dt)
        out[:, s] = V[:, 0, 0, 0]
    return out
