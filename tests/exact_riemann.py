"""Exact solution of the 1D Riemann problem for the ideal-gas Euler equations.

Independent of the solver under test: it follows the classical construction
(Toro, Riemann Solvers and Numerical Methods for Fluid Dynamics, 3rd ed.,
ch. 4): Newton iteration on the pressure function f(p) = f_L(p) + f_R(p) + du
for the star pressure, then sampling of the self-similar wave fan at x/t.
Used to pin the oracle on the Sod shock tube.
"""
from __future__ import annotations

import math

import numpy as np


def _fK(p, rho, pK, cK, g):
    """Pressure function of one side and its derivative (shock if p > pK,
    rarefaction otherwise)."""
    if p > pK:
        A = 2.0 / ((g + 1.0) * rho)
        B = (g - 1.0) / (g + 1.0) * pK
        q = math.sqrt(A / (p + B))
        return (p - pK) * q, q * (1.0 - 0.5 * (p - pK) / (B + p))
    r = p / pK
    f = 2.0 * cK / (g - 1.0) * (r ** ((g - 1.0) / (2.0 * g)) - 1.0)
    df = 1.0 / (rho * cK) * r ** (-(g + 1.0) / (2.0 * g))
    return f, df


def star_state(left, right, gamma):
    """left/right = (rho, u, p).  Returns (p*, u*, residual)."""
    rl, ul, pl = left
    rr, ur, pr = right
    g = gamma
    cl, cr = math.sqrt(g * pl / rl), math.sqrt(g * pr / rr)
    du = ur - ul
    # primitive-variable guess, kept positive
    p = max(1e-12, 0.5 * (pl + pr) - 0.125 * du * (rl + rr) * (cl + cr))
    for _ in range(100):
        fl, dfl = _fK(p, rl, pl, cl, g)
        fr, dfr = _fK(p, rr, pr, cr, g)
        pn = p - (fl + fr + du) / (dfl + dfr)
        pn = max(pn, 1e-14)
        if abs(pn - p) <= 1e-15 * (pn + p):
            p = pn
            break
        p = pn
    fl, _ = _fK(p, rl, pl, cl, g)
    fr, _ = _fK(p, rr, pr, cr, g)
    u = 0.5 * (ul + ur) + 0.5 * (fr - fl)
    return p, u, fl + fr + du


def sample(left, right, gamma, s):
    """Solution (rho, u, p) at similarity coordinate s = (x - x0)/t."""
    rl, ul, pl = left
    rr, ur, pr = right
    g = gamma
    cl, cr = math.sqrt(g * pl / rl), math.sqrt(g * pr / rr)
    ps, us, _ = star_state(left, right, gamma)
    gm = (g - 1.0) / (g + 1.0)
    if s <= us:  # left of the contact
        if ps > pl:  # left shock
            sl = ul - cl * math.sqrt((g + 1.0) / (2.0 * g) * ps / pl + (g - 1.0) / (2.0 * g))
            if s <= sl:
                return rl, ul, pl
            return rl * (ps / pl + gm) / (gm * ps / pl + 1.0), us, ps
        cls = cl * (ps / pl) ** ((g - 1.0) / (2.0 * g))
        if s <= ul - cl:
            return rl, ul, pl
        if s >= us - cls:
            return rl * (ps / pl) ** (1.0 / g), us, ps
        c = 2.0 / (g + 1.0) * (cl + 0.5 * (g - 1.0) * (ul - s))
        u = 2.0 / (g + 1.0) * (cl + 0.5 * (g - 1.0) * ul + s)
        rho = rl * (c / cl) ** (2.0 / (g - 1.0))
        return rho, u, pl * (c / cl) ** (2.0 * g / (g - 1.0))
    if ps > pr:  # right shock
        sr = ur + cr * math.sqrt((g + 1.0) / (2.0 * g) * ps / pr + (g - 1.0) / (2.0 * g))
        if s >= sr:
            return rr, ur, pr
        return rr * (ps / pr + gm) / (gm * ps / pr + 1.0), us, ps
    crs = cr * (ps / pr) ** ((g - 1.0) / (2.0 * g))
    if s >= ur + cr:
        return rr, ur, pr
    if s <= us + crs:
        return rr * (ps / pr) ** (1.0 / g), us, ps
    c = 2.0 / (g + 1.0) * (cr - 0.5 * (g - 1.0) * (ur - s))
    u = 2.0 / (g + 1.0) * (-cr + 0.5 * (g - 1.0) * ur + s)
    rho = rr * (c / cr) ** (2.0 / (g - 1.0))
    return rho, u, pr * (c / cr) ** (2.0 * g / (g - 1.0))


def profile(left, right, gamma, x, x0, t):
    out = np.array([sample(left, right, gamma, (xi - x0) / t) for xi in x])
    return out[:, 0], out[:, 1], out[:, 2]


def cell_average_profile(left, right, gamma, nx, x0, t, sub=64):
    """Cell averages of (rho, u, p) over [i h, (i+1) h] by midpoint quadrature
    with `sub` points per cell (rho, m, E averaged, then converted back)."""
    h = 1.0 / nx
    xs = (np.arange(nx * sub) + 0.5) * h / sub
    r, u, p = profile(left, right, gamma, xs, x0, t)
    m = r * u
    E = p / (gamma - 1.0) + 0.5 * r * u * u
    ra = r.reshape(nx, sub).mean(1)
    ma = m.reshape(nx, sub).mean(1)
    Ea = E.reshape(nx, sub).mean(1)
    ua = ma / ra
    pa = (gamma - 1.0) * (Ea - 0.5 * ra * ua * ua)
    return ra, ua, pa
