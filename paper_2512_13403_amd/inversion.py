"""Gradient-based reconstruction of initial conditions (the paper's inverse
workflow, Sec. 2.3 and Sec. 7): an initial density field is optimised with
ADAM so that the simulated final state matches a target, the gradient of the
misfit coming from the checkpointed adjoint rollout (``rollout.py``, the
library's hand-written adjoint step).

The control is the initial density; the initial velocity and pressure stay
fixed, and the conserved state is assembled from them as in the paper's
initial-condition equation (Sec. 3.1: m = rho v, E = P/(gamma-1) + rho|v|^2/2).
The ADAM update of the control runs in the library (``mh_adam``).
Two misfits are offered:

* ``"l2"``:        1/2 sum (rho_final - rho_target)^2 over the cube;
* ``"projected"``: the mean-square error of the density projected along z
  against a target map (Sec. 7, the projected-density likelihood).

The time steps are frozen to a given schedule (the adjoint treats dt as
fixed), so every iteration differentiates the same discrete map.  All hydro,
source and adjoint arithmetic runs in the HIP library; the misfit, the state
assembly and the ADAM update of the control are elementwise torch operations
on device tensors.
"""
from __future__ import annotations

import numpy as np

from . import Adam
from .rollout import make_rollout_function


def assemble_state(rho, v, p, gamma):
    """Conserved state [5][nz][ny][nx] from density (differentiable), fixed
    velocity [3][...] and pressure [...]."""
    import torch

    m = rho.unsqueeze(0) * v
    E = p / (gamma - 1.0) + 0.5 * rho * (v * v).sum(dim=0)
    return torch.cat([rho.unsqueeze(0), m, E.unsqueeze(0)], dim=0).contiguous()


def misfit(rho_final, target, kind="l2"):
    if kind == "l2":
        return 0.5 * ((rho_final - target) ** 2).sum()
    if kind == "projected":
        return ((rho_final.sum(dim=0) - target) ** 2).mean()
    raise ValueError(f"unknown misfit {kind!r}")


def invert_initial_density(solver, U_init, target, dts, iters=50, lr=1e-2, K=10, kind="l2",
                           rho_floor=1e-6, callback=None):
    """Optimises the initial density of ``U_init`` (device tensor [5][...];
    its velocity and pressure are kept) for ``iters`` ADAM iterations so that
    ``len(dts)`` steps with the fixed time steps ``dts`` end close to
    ``target`` (a density cube for "l2", a z-projected map for "projected").
    Densities are clamped at ``rho_floor`` after each update.  Returns (the
    optimised initial state, the misfit before each iteration)."""
    import torch

    gamma = solver.grid.gamma
    rho0 = U_init[0]
    v = (U_init[1:4] / rho0).detach()
    p = ((gamma - 1.0) * (U_init[4] - 0.5 * (U_init[1:4] ** 2).sum(dim=0) / rho0)).detach()
    rho = rho0.detach().clone().contiguous().requires_grad_(True)
    opt = Adam(rho.data, lr=lr)
    F = make_rollout_function()
    dts = np.asarray(dts, dtype=np.float64)
    losses = []
    for it in range(iters):
        rho.grad = None
        U0 = assemble_state(rho, v, p, gamma)
        Uf = F.apply(U0, solver, len(dts), K, dts)
        loss = misfit(Uf[0], target, kind)
        loss.backward()
        losses.append(float(loss.detach()))
        opt.step(rho.grad)
        with torch.no_grad():
            rho.clamp_(min=rho_floor)
        if callback is not None:
            callback(it, losses[-1])
    with torch.no_grad():
        return assemble_state(rho, v, p, gamma).detach(), losses


def learn_flux_correction(solver, U0, target, dts, iters=30, lr=1e-3, K=10, kind="l2",
                          field_init=None, callback=None):
    """Solver-in-the-loop training of a learned flux term (Sec. 8): a
    correction field B [5][...] added to each cell's upper-face fluxes
    (``Solver.set_flux_correction``) is fitted with ADAM so that len(dts)
    steps from U0 with the fixed time steps dts end with a density close to
    ``target``; the gradient of the misfit with respect to B is accumulated
    by the adjoint steps of the checkpointed rollout.  Here B is a free field
    (the parameters themselves); a network producing B from the state would
    chain its own reverse pass onto the same gradient.  Returns (B, misfit
    before each iteration)."""
    import torch

    from .rollout import rollout_backward, rollout_forward

    B = (torch.zeros_like(U0) if field_init is None else field_init.detach().clone()).contiguous()
    gB = torch.zeros_like(U0)
    opt = Adam(B, lr=lr)
    dts = np.asarray(dts, dtype=np.float64)
    losses = []
    for it in range(iters):
        field = B.detach().contiguous()
        gB.zero_()
        solver.set_flux_correction(field, gB)
        Uf, used, cks = rollout_forward(solver, U0, len(dts), K, dts)
        rho = Uf[0].detach().requires_grad_(True)
        loss = misfit(rho, target, kind)
        loss.backward()
        lam = torch.zeros_like(Uf)
        lam[0] = rho.grad
        rollout_backward(solver, cks, used, K, lam)
        losses.append(float(loss.detach()))
        opt.step(gB)
        if callback is not None:
            callback(it, losses[-1])
    solver.set_flux_correction(None, None)
    return B.detach(), losses
