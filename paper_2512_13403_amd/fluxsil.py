"""Solver-in-the-loop training of a learned flux network (Sec. 8, the
Kelvin-Helmholtz flux corrector): the corrector network in flux mode produces
B_theta(U^n), which ``Solver.set_flux_correction`` adds to each cell's
upper-face fluxes in every stage of step n; a rollout of m steps is compared
with target states, and the gradient of the misfit flows back through each
step's adjoint (which accumulates dL/dB^n) and through the network (whose
reverse pass gives the parameter gradient and the input-gradient path back
into lambda^n).  No sources; fixed time steps.  All arithmetic runs in the
library (network, step, adjoint); this module orders the calls and forms the
misfit.
"""
from __future__ import annotations


def _field(corr, U):
    """B_theta(U) for one state [5][n][n][n] (the corrector has batch 1)."""
    out, _, _ = corr.apply(U.unsqueeze(0), stats=False)
    return out[0]


def rollout(solver, corr, U0, dts):
    """States U^0 .. U^m and fields B^0 .. B^{m-1} of m steps with the
    network flux."""
    solver.set_state(U0)
    states, fields = [U0.clone()], []
    for dt in dts:
        B = _field(corr, states[-1]).contiguous()
        solver.set_flux_correction(B)
        solver.step(1, float(dt))
        fields.append(B)
        states.append(solver.get_state_device().clone())
    solver.set_flux_correction(None)
    return states, fields


WEIGHTS = (4.0, 1.0, 1.0, 1.0, 1.0)


def misfit(states, targets, weights=WEIGHTS):
    """L = sum_k sum_c w_c mean((U^k_c - T^k_c)^2) over k = 1..m against
    targets[k-1]."""
    loss = 0.0
    for k in range(1, len(states)):
        d = states[k] - targets[k - 1]
        for c in range(5):
            loss += weights[c] * float((d[c] * d[c]).mean())
    return loss


def loss_and_grad(solver, corr, U0, dts, targets, weights=WEIGHTS):
    """The unrolled misfit of the rollout from U0, accumulating dL/dtheta in
    the corrector (call corr.zero_grad() first).  Returns L."""
    import torch

    _, step0 = solver.clock()
    states, fields = rollout(solver, corr, U0, dts)
    w = torch.tensor(weights, dtype=U0.dtype, device=U0.device).view(5, 1, 1, 1)
    ncell = U0[0].numel()
    lam = torch.zeros_like(U0)
    g = torch.zeros_like(U0)
    for k in range(len(dts), 0, -1):
        lam = lam + 2.0 * w * (states[k] - targets[k - 1]) / ncell
        # step k-1: lambda^{k-1} and dL/dB^{k-1} from its adjoint
        g.zero_()
        solver.set_flux_correction(fields[k - 1], g)
        lam = solver.adjoint_step(states[k - 1], float(dts[k - 1]), step0 + k - 1,
                                  lam.contiguous())
        solver.set_flux_correction(None)
        # through the network: parameters, and its input-gradient path
        _, gU = corr.backward(states[k - 1].unsqueeze(0), gUc=g.unsqueeze(0), input_grad=True)
        lam = lam + gU[0]
    return misfit(states, targets, weights)


def train(solver, corr, U0, dts, targets, iters=30, lr=1e-3, callback=None):
    """ADAM on the network parameters through the unrolled misfit; returns the
    misfit before each iteration."""
    losses = []
    for it in range(iters):
        corr.zero_grad()
        losses.append(loss_and_grad(solver, corr, U0, dts, targets))
        corr.adam_step(lr)
        if callback is not None:
            callback(it, losses[-1])
    return losses
