"""Pins of the oracle's alternative limiters and Riemann solvers (paper App. A.1
names minmod, van Leer, MC and superbee; App. A.2 names HLL and Rusanov beside
HLLC; none of them is printed).  Each check goes through the whole semi-discrete
operator L(U) and compares with a fact that does not come from the oracle:

* limiters: on a contact (uniform velocity and pressure) HLLC transports
  density by exact upwinding (pinned in test_oracle_hydro), so the mass flux
  through face i+1/2 is u (rho_i + s_i / 2) and every cell's limited slope s_i
  can be read back from L(U).  The slopes must equal phi(r) * b in the
  flux-limiter (ratio) form of the published definitions, b = rho_i - rho_{i-1},
  r = (rho_{i+1} - rho_i) / b, with phi at the designed ratios taken from the
  hand-computed table in tests/golden/limiter_phi_table.json;
* Riemann solvers: at first order a contact (density jump at uniform velocity
  u, transverse velocities w and pressure p) gets, from any two-state flux of
  the form alpha F_L + beta F_R + delta (U_R - U_L), a mass flux
  u (rho_L + rho_R) / 2 - kappa (rho_R - rho_L) and the other fields follow
  from it (normal momentum u m + p, transverse w m, energy |v|^2 m / 2 +
  gamma u p / (gamma - 1)).  The numerical diffusion kappa identifies the
  solver: |u| / 2 for HLLC (exact upwinding), max(c, |u|) / 2 for HLL with the
  Davis speeds u -/+ c (c the larger sound speed), (|u| + c) / 2 for Rusanov.
  A pressure jump at rest gives the mean pressure as momentum flux and
  -c (p_R - p_L) / (2 (gamma - 1)) as energy flux for both HLL and Rusanov.
"""
import json
import math
import os

import numpy as np
import pytest

import oracle
import workloads as wl

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
LIMS = {"minmod": oracle.LIM_MINMOD, "vanleer": oracle.LIM_VANLEER, "mc": oracle.LIM_MC,
        "superbee": oracle.LIM_SUPERBEE}


def phi_ratio(name, r):
    """The published ratio forms (LeVeque 2002, eq. 6.39a-d)."""
    if name == "minmod":
        return max(0.0, min(1.0, r))
    if name == "vanleer":
        return (r + abs(r)) / (1.0 + abs(r))
    if name == "mc":
        return max(0.0, min(2.0 * r, 0.5 * (1.0 + r), 2.0))
    if name == "superbee":
        return max(0.0, min(2.0 * r, 1.0), min(r, 2.0))
    raise ValueError(name)


def pencil(axis, n, h):
    """(shape, spacing) of a one-dimensional grid of n cells along axis."""
    shape = [1, 1, 1]
    shape[2 - axis] = n
    hh = [0.5, 0.5, 0.5]
    hh[axis] = h
    return tuple(shape), tuple(hh)


def state_along(axis, rho, vn, wt, p, gamma):
    """Conserved state of a pencil along axis: normal velocity vn, the two
    transverse velocities wt = (w1, w2) in cyclic order after axis."""
    n = len(rho)
    shape, _ = pencil(axis, n, 1.0)
    v = [0.0, 0.0, 0.0]
    v[axis] = vn
    v[(axis + 1) % 3] = wt[0]
    v[(axis + 2) % 3] = wt[1]
    r = np.asarray(rho, dtype=np.float64).reshape(shape)
    f = lambda a: np.full(shape, a)
    return wl.conserved(r, f(v[0]), f(v[1]), f(v[2]), f(p), gamma)


def fields_along(axis, L):
    """(mass, normal momentum, t1, t2, energy) rows of a pencil's L(U)."""
    flat = [L[f].ravel() for f in range(5)]
    return [flat[0], flat[1 + axis], flat[1 + (axis + 1) % 3], flat[1 + (axis + 2) % 3], flat[4]]


# ------------------------------------------------------------------------- limiters

def designed_profile(rs, sign):
    """Density pencil holding, for every ratio r in rs, a cell with backward
    difference b = sign/8 and forward difference r b (all values exact in
    binary), separated by flat stretches of the background value 1.  Returns
    the profile and the indices of the designed cells."""
    rho, cells = [1.0] * 4, []
    for r in rs:
        b = sign * 0.125
        rho += [1.0 + b, 1.0 + b + r * b]
        cells.append(len(rho) - 2)
        rho += [1.0] * 3
    return np.array(rho), cells


def recover_slopes(limiter, rho, axis=0, u=0.5, p=1.0, gamma=1.4):
    """Every cell's limited density slope, read back from the mass row of L(U)
    of an upwind-transported contact (u > 0): face i+1/2 carries u f_{i+1/2},
    f_{i+1/2} = rho_i + s_i / 2, and L_i = -u (f_{i+1/2} - f_{i-1/2}) / h.
    Cells 0-2 are flat, so f_{1+1/2} = rho_1 starts the recursion."""
    n = len(rho)
    h = 1.0 / n
    shape, hh = pencil(axis, n, h)
    U = state_along(axis, rho, u, (0.0, 0.0), p, gamma)
    c = oracle.make_config(shape, hh, gamma=gamma, limiter=limiter)
    mass = fields_along(axis, oracle.rhs(c, U))[0]
    assert rho[0] == rho[1] == rho[2]
    f = np.empty(n)
    f[1] = rho[1]
    for i in list(range(2, n)) + [0]:
        f[i] = f[i - 1] - h * mass[i] / u
    return 2.0 * (f - rho)


def expected_slopes(name, rho):
    n = len(rho)
    out = np.empty(n)
    for i in range(n):
        a = rho[(i + 1) % n] - rho[i]
        b = rho[i] - rho[i - 1]
        out[i] = 0.0 if b == 0.0 else phi_ratio(name, a / b) * b
    return out


@pytest.mark.parametrize("name", sorted(LIMS))
@pytest.mark.parametrize("sign", [1.0, -1.0])
def test_limiter_matches_published_phi_table(name, sign):
    g = json.load(open(os.path.join(GOLDEN, "limiter_phi_table.json")))
    rho, cells = designed_profile(g["r"], sign)
    s = recover_slopes(LIMS[name], rho)
    for r, i, phi in zip(g["r"], cells, g["phi"][name]):
        b = rho[i] - rho[i - 1]
        assert s[i] / b == pytest.approx(phi, abs=1e-12), (name, r)


@pytest.mark.parametrize("name", sorted(LIMS))
@pytest.mark.parametrize("axis", [0, 1, 2])
def test_limiter_slopes_of_a_random_profile(name, axis):
    """All slopes of a random profile (every branch of each limiter is taken)
    against the ratio form, along every axis."""
    rng = np.random.default_rng(11 + axis)
    rho = np.concatenate([np.ones(4), rng.uniform(0.5, 2.0, 60), np.ones(3)])
    s = recover_slopes(LIMS[name], rho, axis=axis)
    e = expected_slopes(name, rho)
    assert np.abs(s - e).max() < 1e-12


def test_limiter_ratio_forms_are_symmetric():
    """phi(r) / r = phi(1 / r) for the symmetric limiters (a check of the
    ratio forms this file uses, over both branches of each)."""
    for name in LIMS:
        for r in (0.1, 0.3, 0.5, 0.8, 1.0, 1.7, 3.0, 9.0):
            assert phi_ratio(name, r) / r == pytest.approx(phi_ratio(name, 1.0 / r), rel=1e-14)


def test_limiters_differ_where_the_table_says():
    """Guards the table against a limiter coded as another: at r = 1/4 and
    r = 2 the four published functions take different values."""
    g = json.load(open(os.path.join(GOLDEN, "limiter_phi_table.json")))
    k1, k2 = g["r"].index(0.25), g["r"].index(2.0)
    seen = {(g["phi"][n][k1], g["phi"][n][k2]) for n in LIMS}
    assert len(seen) == 4
    for n in LIMS:
        for r, phi in zip(g["r"], g["phi"][n]):
            assert phi_ratio(n, r) == pytest.approx(phi, abs=1e-15)


# ------------------------------------------------------------------- Riemann solvers

def recovered_face_flux(solver, axis, rhoL, rhoR, u, wt, p, gamma, n=8):
    """First-order (no slopes) pencil with rho_L in cells [0, n/2) and rho_R in
    [n/2, n): the flux through the face between cells n/2-1 and n/2 in the
    face frame, from L of cell n/2-1, whose other face sees rho_L on both
    sides and carries the physical flux of the left state."""
    h = 1.0 / n
    shape, hh = pencil(axis, n, h)
    rho = np.array([rhoL] * (n // 2) + [rhoR] * (n // 2))
    U = state_along(axis, rho, u, wt, p, gamma)
    c = oracle.make_config(shape, hh, gamma=gamma, limiter=oracle.LIM_NONE, riemann=solver)
    L = fields_along(axis, oracle.rhs(c, U))
    i = n // 2 - 1
    E = p / (gamma - 1.0) + 0.5 * rhoL * (u * u + wt[0] ** 2 + wt[1] ** 2)
    phys = [rhoL * u, rhoL * u * u + p, rhoL * u * wt[0], rhoL * u * wt[1], u * (E + p)]
    return np.array([phys[f] - h * L[f][i] for f in range(5)])


def contact_flux(kappa, rhoL, rhoR, u, wt, p, gamma):
    m = 0.5 * u * (rhoL + rhoR) - kappa * (rhoR - rhoL)
    v2 = u * u + wt[0] ** 2 + wt[1] ** 2
    return np.array([m, u * m + p, wt[0] * m, wt[1] * m,
                     0.5 * v2 * m + gamma * u * p / (gamma - 1.0)])


@pytest.mark.parametrize("solver", ["hllc", "hll", "rusanov"])
@pytest.mark.parametrize("u", [0.0, 0.3, -0.45, 2.5, -2.5])
@pytest.mark.parametrize("axis", [0, 1, 2])
def test_contact_flux_has_the_solver_s_numerical_diffusion(solver, u, axis):
    gamma, p, wt = 1.4, 0.6, (0.2, -0.1)
    rhoL, rhoR = 1.0, 0.25
    c = math.sqrt(gamma * p / min(rhoL, rhoR))  # the larger sound speed
    kappa = {"hllc": abs(u) / 2, "hll": max(c, abs(u)) / 2, "rusanov": (abs(u) + c) / 2}[solver]
    rs = {"hllc": oracle.RS_HLLC, "hll": oracle.RS_HLL, "rusanov": oracle.RS_RUSANOV}[solver]
    for (a, b) in ((rhoL, rhoR), (rhoR, rhoL)):
        got = recovered_face_flux(rs, axis, a, b, u, wt, p, gamma)
        want = contact_flux(kappa, a, b, u, wt, p, gamma)
        scale = np.abs(want).max()
        assert np.abs(got - want).max() < 1e-13 * scale, (solver, u, a, b, got, want)


@pytest.mark.parametrize("solver", [oracle.RS_HLL, oracle.RS_RUSANOV])
def test_pressure_jump_at_rest(solver):
    """v = 0, uniform density, p_L != p_R: both two-state solvers give zero
    mass flux, the mean pressure as momentum flux and -c (p_R - p_L) / (2 (gamma-1))
    as energy flux, c = sqrt(gamma max(p) / rho) (Davis speeds -c, +c)."""
    gamma, rho, pL, pR, n = 5.0 / 3.0, 0.8, 2.0, 0.5, 8
    h = 1.0 / n
    p = np.array([pL] * (n // 2) + [pR] * (n // 2))
    shape, hh = pencil(0, n, h)
    z = np.zeros(shape)
    U = wl.conserved(np.full(shape, rho), z, z, z, p.reshape(shape), gamma)
    cfg = oracle.make_config(shape, hh, gamma=gamma, limiter=oracle.LIM_NONE, riemann=solver)
    L = oracle.rhs(cfg, U)
    i = n // 2 - 1
    got = np.array([0.0 - h * L[0].ravel()[i], pL - h * L[1].ravel()[i],
                    0.0 - h * L[4].ravel()[i]])
    c = math.sqrt(gamma * max(pL, pR) / rho)
    want = np.array([0.0, 0.5 * (pL + pR), -c * (pR - pL) / (2.0 * (gamma - 1.0))])
    assert np.abs(got - want).max() < 1e-13 * np.abs(want).max()
