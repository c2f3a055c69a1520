"""Differentiable multi-step rollout with checkpoint-every-K recomputation.

The paper differentiates through the time loop in reverse mode, storing a
sparse set of states and recomputing the segments between them (Sec. 2.3).
``HydroRollout`` does the same with the library's hand-written adjoint step
(``mh_adjoint_step``): the forward pass runs ``nsteps`` steps and keeps the
state, OU amplitudes, potential and clock every ``K`` steps; the backward pass
walks the segments from last to first, replays each segment from its
checkpoint with the recorded (frozen) dt values, keeping every step's inputs,
and applies the adjoint steps in reverse.  All arithmetic runs in the HIP
library; this module only orders the calls.
"""
from __future__ import annotations

import numpy as np

from . import Solver


class Checkpoint:
    def __init__(self, U, ahat, phi, t, step):
        self.U, self.ahat, self.phi, self.t, self.step = U, ahat, phi, t, step


def _gravity_on(s: Solver) -> bool:
    from . import SRC_GRAVITY

    return bool(s.phys.flags & SRC_GRAVITY)


def _forcing_on(s: Solver) -> bool:
    from . import SRC_FORCING

    return bool(s.phys.flags & SRC_FORCING)


def _snapshot(s: Solver) -> Checkpoint:
    t, step = s.clock()
    return Checkpoint(s.get_state_device(), s.ou_state() if _forcing_on(s) else None,
                      s.potential_device() if _gravity_on(s) else None, t, step)


def _restore(s: Solver, ck: Checkpoint):
    s.set_state(ck.U)
    if ck.ahat is not None:
        s.set_ou_state(ck.ahat)
    if ck.phi is not None:
        s.set_potential(ck.phi)
    s.set_clock(ck.t, ck.step)


def rollout_forward(s: Solver, U0, nsteps: int, K: int, dts=None):
    """Runs nsteps from U0 (CUDA tensor).  dts: per-step fixed dt values, or
    None for CFL steps (recorded).  Returns (U_final, dts, checkpoints)."""
    K = max(1, int(K))
    s.set_state(U0)
    cks = []
    used = []
    for k in range(nsteps):
        if k % K == 0:
            cks.append(_snapshot(s))
        d = s.step(1, float(dts[k]) if dts is not None else 0.0, record=True)
        used.append(float(d[0]))
    return s.get_state_device(), np.array(used), cks


def rollout_backward(s: Solver, cks, dts, K: int, lam, keep=None):
    """lam_0 = (dU_final/dU_0)^T lam for the run recorded by rollout_forward.

    keep: the segment replay also keeps each step's first stage and its state
    after the forcing kick (mh_step_keep), two more states per step of a
    segment, and the adjoint steps use them, and with gravity the potential
    each step solved for (the next step's snapshot), instead of recomputing
    the stages and the forward Poisson solve (the gradient is bitwise the
    same).  Default: on for SSP-RK2."""
    from . import RK_SSP2

    K = max(1, int(K))
    nsteps = len(dts)
    if keep is None:
        keep = s.grid.integrator == RK_SSP2
    lam = lam.contiguous().clone()
    for seg in range(len(cks) - 1, -1, -1):
        k0 = seg * K
        k1 = min(k0 + K, nsteps)
        _restore(s, cks[seg])
        inputs = []
        kept = []
        for k in range(k0, k1):
            snap = _snapshot(s)
            inputs.append(snap)
            if keep:
                U1, Ub = s.new_state_tensor(), s.new_state_tensor()
                s.step_keep(float(dts[k]), U1, Ub)
                kept.append((U1, Ub))
            else:
                s.step(1, float(dts[k]))
        # the potential each replayed step solved for: the next step's
        # starting one, and the solver's after the last
        phi_after = ([snap.phi for snap in inputs[1:]] +
                     [s.potential_device() if _gravity_on(s) else None]) if keep else None
        for k in range(k1 - 1, k0 - 1, -1):
            snap = inputs[k - k0]
            kk = (kept[k - k0] + (phi_after[k - k0],)) if keep else None
            s.adjoint_step(snap.U, float(dts[k]), snap.step, lam, ou_ahat=snap.ahat,
                           phi_n=snap.phi, out=lam, kept=kk)
            if keep:
                kept[k - k0] = None  # free the step's kept stages
    return lam


def make_rollout_function():
    """torch.autograd.Function over the rollout: forward(U0, solver, nsteps, K,
    dts) -> U_final; backward gives dL/dU0 through the hand-written adjoint."""
    import torch

    class HydroRollout(torch.autograd.Function):
        @staticmethod
        def forward(ctx, U0, solver, nsteps, K, dts=None):
            Uf, used, cks = rollout_forward(solver, U0.detach(), nsteps, K, dts)
            ctx.solver, ctx.cks, ctx.dts, ctx.K = solver, cks, used, K
            return Uf.clone()

        @staticmethod
        def backward(ctx, grad_out):
            lam0 = rollout_backward(ctx.solver, ctx.cks, ctx.dts, ctx.K, grad_out)
            return lam0, None, None, None, None

    return HydroRollout
