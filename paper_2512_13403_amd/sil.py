"""Solver-in-the-loop study of the learned corrector on driven turbulence.

A fine run (256^3 by default) and coarse runs (64^3, a factor r = 4 coarser)
share one clock and one forcing path; the corrector is trained so that a
coarse step followed by the correction reproduces the block average of the
fine run (the paper's Sec. 8 setting, here in 3D on the conserved state).

Alignment.  The fine run computes its CFL step dt_f at the first of each
group of r substeps and holds it for the group; its OU amplitudes advance once
per group with r dt_f (``ou_every = r``).  A coarse step of dt_c = r dt_f then
covers one fine group at identical times, and the coarse run (``ou_every =
1``) draws the same OU noise for coarse step k as the fine run for group k,
because both index the draw by the group.  Targets are conservative r^3
block averages of the fine conserved state after each group.

Training (500 ADAM iterations, learning rate decaying geometrically from 1e-3
to 1e-4 as in the paper's Sec. 8): each iteration takes a batch of (trajectory,
time) pairs k, starts a coarse step from the block-averaged fine state T_k
with the fine run's OU amplitudes, and fits U' = P_{k+1} + s Net(P_{k+1}) to
T_{k+1}, where P_{k+1} is the plain coarse step.  Evaluation runs plain and
corrected coarse rollouts from T_0 of held-out seeds and reports the density
L2 error against the block-averaged fine run, and the wall-clock cost of each.

Every arithmetic step runs in the HIP library (mh_step, mh_corr_*,
mh_block_average); this module orders the calls.
"""
from __future__ import annotations

import math
import time
from dataclasses import dataclass, field

import numpy as np

from . import (BC_PERIODIC, Corrector, SRC_FORCING, Solver, block_average, corr_desc, grid_desc,
               physics_desc)

DRIVE = dict(ou_tau=0.5, ou_arms=1.0, ou_zeta=1.0, ou_kmin=1.0, ou_kmax=2.0)
GAMMA = 5.0 / 3.0


def make_solver(n: int, seed: int, every: int, dtype="f32") -> Solver:
    g = grid_desc((n, n, n), (1.0 / n,) * 3, (BC_PERIODIC,) * 3, dtype, GAMMA, 0.4)
    p = physics_desc(flags=SRC_FORCING, ou_seed=seed, ou_every=every, **DRIVE)
    return Solver(g, p)


def rest_state_device(n: int, torch_dtype):
    """rho = 1, v = 0, P = 1 (E = 1/(gamma - 1)), made on the device."""
    import torch

    U = torch.zeros((5, n, n, n), dtype=torch_dtype, device="cuda:0")
    U[0].fill_(1.0)
    U[4].fill_(1.0 / (GAMMA - 1.0))
    return U


def fine_group(s: Solver, r: int) -> float:
    """One group of r fine substeps at the group's CFL step; returns dt_f."""
    dt = float(s.step(1, 0.0, record=True)[0])
    if r > 1:
        s.step(r - 1, dt)
    return dt


@dataclass
class Trajectory:
    seed: int
    T: object                      # [nsteps+1][5][nc][nc][nc] block-averaged fine states
    dts: np.ndarray                # coarse steps dt_c = r dt_f
    ahat: list                     # OU amplitudes before each coarse step
    t: np.ndarray                  # clock before each coarse step
    step: np.ndarray               # coarse step index (= fine group index)
    fine_seconds: float = 0.0      # wall clock of the recorded fine groups
    fine_steps: int = 0


def record_trajectory(seed: int, nf: int = 256, r: int = 4, t_spinup: float = 1.0,
                      nsteps: int = 100) -> Trajectory:
    import torch

    s = make_solver(nf, seed, r)
    s.set_state(rest_state_device(nf, s.torch_dtype))
    t, fstep = s.clock()
    while t < t_spinup:
        fine_group(s, r)
        t, fstep = s.clock()
    T, dts, ahat, ts, steps = [], [], [], [], []

    def snap():
        T.append(block_average(s.get_state_device(), r))
        ahat.append(s.ou_state())
        tt, st = s.clock()
        ts.append(tt)
        steps.append(st // r)

    snap()
    torch.cuda.synchronize()
    fine_time = 0.0
    for _ in range(nsteps):
        t0 = time.perf_counter()
        dts.append(r * fine_group(s, r))
        torch.cuda.synchronize()
        fine_time += time.perf_counter() - t0
        snap()
    s.close()
    return Trajectory(seed, torch.stack(T), np.array(dts), ahat, np.array(ts),
                      np.array(steps, dtype=np.int64), fine_time, nsteps * r)


def coarse_step_from(c: Solver, traj: Trajectory, k: int):
    """The plain coarse step from T_k with the fine run's forcing state."""
    c.set_state(traj.T[k])
    c.set_ou_state(traj.ahat[k])
    c.set_clock(float(traj.t[k]), int(traj.step[k]))
    c.step(1, float(traj.dts[k]))
    return c.get_state_device()


@dataclass
class TrainResult:
    theta: np.ndarray
    losses: list = field(default_factory=list)
    stats: dict = field(default_factory=dict)
    seconds: float = 0.0


def train(trajs, nc: int, iters: int = 500, batch: int = 8, lr0: float = 1e-3, lr1: float = 1e-4,
          loss_w=(4.0, 1.0, 1.0, 1.0, 1.0), seed: int = 0, init_scale: float = 1e-2,
          schedule=((1.0, 1),)) -> TrainResult:
    """Fits the corrector in `iters` ADAM iterations; `schedule` lists
    (fraction of the iterations, unroll m) phases in order.  m = 1 uses
    single-step pairs (the plain coarse step from T_k against T_{k+1}); m > 1
    runs m corrected coarse steps from T_k and back-propagates the summed loss
    against T_{k+1..k+m} through the corrector (mh_corr_backward) and the
    hydro step (mh_adjoint_step): the solver in the loop.  The learning rate
    decays geometrically over all iterations."""
    import torch

    from workloads import corrector_init_params

    P, T = [], []
    solvers = {}
    for tr in trajs:
        cs = solvers.setdefault(tr.seed, make_solver(nc, tr.seed, 1))
        for k in range(len(tr.dts)):
            P.append(coarse_step_from(cs, tr, k))
            T.append(tr.T[k + 1])
    P = torch.stack(P)
    T = torch.stack(T)
    d = (T - P).double()
    Pd = P.double()
    mean = Pd.mean(dim=(0, 2, 3, 4)).cpu().numpy()
    std = Pd.std(dim=(0, 2, 3, 4)).cpu().numpy() + 1e-12
    scale = d.std(dim=(0, 2, 3, 4)).cpu().numpy() + 1e-12
    del d, Pd
    # relative MSE: the library divides channel c's squared error by std_c^2;
    # weights w_c std_c^2 / scale_c^2 make it sum_c w_c mean(d_c^2) / scale_c^2,
    # i.e. relative to the spread of the residual the network has to predict
    lw = np.asarray(loss_w, dtype=np.float64) * std ** 2 / scale ** 2
    stats = dict(mean=mean, std=std, scale=scale, loss_w=lw)
    corr = Corrector(corr_desc(nc, batch, "f32", GAMMA, mean, std, scale, lw, 1e-6, 1.0))
    corr.set_params(corrector_init_params(seed=seed, out_scale=init_scale))
    rng = np.random.default_rng(seed)
    losses = []
    nk = [len(tr.dts) for tr in trajs]
    offs = np.cumsum([0] + nk)
    phase_m = []
    for frac, m in schedule:
        phase_m += [int(m)] * int(round(frac * iters))
    phase_m = (phase_m + [phase_m[-1]] * iters)[:iters]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for it in range(iters):
        lr = lr0 * (lr1 / lr0) ** (it / max(iters - 1, 1))
        m = phase_m[it]
        if m == 1:
            idx = torch.as_tensor(rng.integers(0, P.shape[0], batch), device=P.device)
            losses.append(corr.train_step(P[idx], T[idx], lr))
            continue
        # solver in the loop: m corrected steps from T_k of `batch` windows
        picks = []
        for _ in range(batch):
            i = int(rng.integers(0, len(trajs)))
            picks.append((i, int(rng.integers(0, nk[i] - m + 1))))
        states = []      # U_{j-1} per step j (list over j of [batch] tensors)
        preds = []       # P_j = H(U_{j-1})
        U = torch.stack([trajs[i].T[k] for i, k in picks])
        for j in range(1, m + 1):
            states.append(U)
            Pj = torch.empty_like(U)
            for b, (i, k) in enumerate(picks):
                tr = trajs[i]
                cs = solvers[tr.seed]
                cs.set_state(U[b])
                cs.set_ou_state(tr.ahat[k + j - 1])
                cs.set_clock(float(tr.t[k + j - 1]), int(tr.step[k + j - 1]))
                cs.step(1, float(tr.dts[k + j - 1]))
                cs.get_state_into(Pj[b])
            preds.append(Pj)
            U, _, _ = corr.apply(Pj, stats=False)
        corr.zero_grad()
        lam = None
        total = 0.0
        for j in range(m, 0, -1):
            tgt = torch.stack([trajs[i].T[k + j] for i, k in picks])
            L, gP = corr.backward(preds[j - 1], tgt, lam, want_loss=True, input_grad=j > 1)
            total += L
            if j > 1:
                lam = torch.empty_like(gP)
                for b, (i, k) in enumerate(picks):
                    tr = trajs[i]
                    solvers[tr.seed].adjoint_step(states[j - 1][b], float(tr.dts[k + j - 1]),
                                                  int(tr.step[k + j - 1]), gP[b],
                                                  ou_ahat=tr.ahat[k + j - 1], out=lam[b])
        corr.adam_step(lr)
        losses.append(total / m)
    torch.cuda.synchronize()
    for cs in solvers.values():
        cs.close()
    return TrainResult(corr.params(), losses, stats, time.perf_counter() - t0)


def rel_l2(a, b) -> float:
    return float(((a - b).double().norm() / b.double().norm()).item())


def evaluate(trajs, nc: int, res: TrainResult, nsteps: int | None = None) -> dict:
    """Plain and corrected coarse rollouts from T_0 of each held-out trajectory
    against its fine run.  The trajectories advance together, one coarse solver
    each; the corrected rollout is one call of the library's corrected step
    (mh_step_corrected: the plain steps and one batched corrector pass per
    step, replayed from a captured HIP graph, the step sizes from a device
    schedule).  Cost = wall clock of the batched rollout (after one untimed
    step of each kind); the fine cost is the summed wall clock of the same
    trajectories' fine groups."""
    import torch

    from . import step_corrected

    B = len(trajs)
    n = min(len(t.dts) for t in trajs) if nsteps is None else nsteps
    st = res.stats
    corr = Corrector(corr_desc(nc, B, "f32", GAMMA, st["mean"], st["std"], st["scale"],
                               st["loss_w"], 1e-6, 1e-3))
    corr.set_params(res.theta)
    solvers = [make_solver(nc, t.seed, 1) for t in trajs]
    stage = torch.empty(2 * B * 5 * nc ** 3, dtype=solvers[0].torch_dtype,
                        device=solvers[0].device)
    dts = torch.tensor(np.stack([t.dts[:n] for t in trajs], axis=1), dtype=torch.float64,
                       device=solvers[0].device).contiguous()

    def reset():
        for c, t in zip(solvers, trajs):
            c.set_state(t.T[0])
            c.set_ou_state(t.ahat[0])
            c.set_clock(float(t.t[0]), int(t.step[0]))

    def advance(k, corrected, stats):
        if not corrected:
            for c, t in zip(solvers, trajs):
                c.step(1, float(t.dts[k]))
            return 0
        fb = step_corrected(solvers, corr, 1, dts[k:k + 1].contiguous(), use_graph=False,
                            stage=stage, count_fallbacks=stats)
        return int(fb) if stats else 0

    out = {}
    for mode in ("plain", "corrected"):
        corrected = mode == "corrected"
        # one untimed step first (code objects loaded, the capture path run
        # once), then the timed rollout from the start
        reset()
        if corrected:
            step_corrected(solvers, corr, 1, dts[0:1].contiguous(), use_graph=True, stage=stage)
        else:
            advance(0, False, False)
        reset()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        if corrected:
            step_corrected(solvers, corr, n, dts, use_graph=True, stage=stage)
        else:
            for k in range(n):
                advance(k, False, False)
        torch.cuda.synchronize()
        secs = time.perf_counter() - t0
        final = [c.get_state_device() for c in solvers]
        # errors and fallback counts from a step-by-step replay (kept out of
        # the timed loop); it ends in the same states as the timed rollout
        reset()
        errs = [[] for _ in trajs]
        fallbacks = 0
        for k in range(n):
            fallbacks += advance(k, corrected, True)
            for i, (c, t) in enumerate(zip(solvers, trajs)):
                errs[i].append(rel_l2(c.get_state_device()[0], t.T[k + 1][0]))
        for c, u in zip(solvers, final):
            if not torch.equal(c.get_state_device(), u):
                raise RuntimeError("the replayed rollout differs from the timed one")
        out[mode] = dict(rho_rel_l2=errs, seconds=secs, fallbacks=fallbacks)
    for c in solvers:
        c.close()
    fine = sum(t.fine_seconds * n / len(t.dts) for t in trajs)
    out["fine_seconds"] = fine
    out["cost_ratio"] = fine / out["corrected"]["seconds"]
    out["seeds"] = [t.seed for t in trajs]
    return out


def run_study(train_seeds=range(0, 12), eval_seeds=range(12, 16), nf: int = 256, r: int = 4,
              t_spinup: float = 1.0, nsteps: int = 100, iters: int = 500, batch: int = 4,
              schedule=((0.1, 1), (0.3, 16), (0.6, 64)), log=print, lr0: float = 1e-3,
              lr1: float = 1e-4, loss_w=(16.0, 1.0, 1.0, 1.0, 1.0)) -> dict:
    nc = nf // r
    t0 = time.perf_counter()
    trajs = [record_trajectory(s, nf, r, t_spinup, nsteps) for s in train_seeds]
    log(f"[sil] recorded {len(trajs)} training trajectories in {time.perf_counter() - t0:.1f} s")
    res = train(trajs, nc, iters, batch, lr0=lr0, lr1=lr1, loss_w=loss_w, schedule=schedule)
    log(f"[sil] trained {iters} iterations in {res.seconds:.1f} s: loss {res.losses[0]:.4g} -> "
        f"{np.mean(res.losses[-20:]):.4g}")
    del trajs
    evt = [record_trajectory(s, nf, r, t_spinup, nsteps) for s in eval_seeds]
    ev = evaluate(evt, nc, res)
    fin_p = [e[-1] for e in ev["plain"]["rho_rel_l2"]]
    fin_c = [e[-1] for e in ev["corrected"]["rho_rel_l2"]]
    for sd, a, b in zip(ev["seeds"], fin_p, fin_c):
        log(f"[sil] seed {sd}: rho L2 after {nsteps} coarse steps: plain {a:.4e} corrected {b:.4e}")
    plain = float(np.mean(fin_p))
    corrected = float(np.mean(fin_c))
    plain_avg = float(np.mean(ev["plain"]["rho_rel_l2"]))
    corr_avg = float(np.mean(ev["corrected"]["rho_rel_l2"]))
    log(f"[sil] cost: fine {ev['fine_seconds']:.3f} s, corrected coarse "
        f"{ev['corrected']['seconds']:.3f} s, plain coarse {ev['plain']['seconds']:.3f} s "
        f"(ratio {ev['cost_ratio']:.1f})")
    # per curriculum phase: the loss of its first iteration and the mean of
    # its last min(20, length) iterations, each the mean per unrolled step of
    # that phase's objective (so first and last of a phase are comparable)
    phases, it0 = [], 0
    for frac, m in schedule:
        k = int(round(frac * iters))
        seg = res.losses[it0:it0 + k]
        if seg:
            phases.append(dict(unroll=int(m), iters=len(seg), loss_first=float(seg[0]),
                               loss_last=float(np.mean(seg[-min(20, len(seg)):]))))
        it0 += k
    return dict(
        fine=nf, coarse=nc, steps=nsteps, iters=iters, batch=batch, lr=[lr0, lr1],
        loss_w=list(loss_w), schedule=[list(p) for p in schedule], train_phases=phases,
        rho_rel_l2_plain=plain, rho_rel_l2_corrected=corrected,
        error_ratio=corrected / plain,
        rho_rel_l2_plain_mean_over_steps=plain_avg,
        rho_rel_l2_corrected_mean_over_steps=corr_avg,
        cost_ratio=float(ev["cost_ratio"]),
        fine_seconds=float(ev["fine_seconds"]),
        corrected_seconds=float(ev["corrected"]["seconds"]),
        plain_seconds=float(ev["plain"]["seconds"]),
        fallbacks=int(ev["corrected"]["fallbacks"]),
        train_loss_first=float(res.losses[0]), train_loss_last=float(np.mean(res.losses[-20:])),
        seconds=time.perf_counter() - t0,
    )


if __name__ == "__main__":
    import argparse
    import json

    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--fine", type=int, default=256)
    ap.add_argument("--ratio", type=int, default=4)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--iters", type=int, default=500)
    ap.add_argument("--batch", type=int, default=4)
    ap.add_argument("--train-seeds", type=int, default=12)
    ap.add_argument("--eval-seeds", type=int, default=4)
    ap.add_argument("--spinup", type=float, default=1.0)
    ap.add_argument("--lr0", type=float, default=1e-3, help="first learning rate")
    ap.add_argument("--lr1", type=float, default=1e-4, help="last learning rate")
    ap.add_argument("--wrho", type=float, default=16.0, help="density weight of the loss")
    ap.add_argument("--unroll", type=int, default=64,
                    help="longest unroll: 10 %% of the iterations on pairs, 30 %% at "
                         "unroll/4, 60 %% at unroll")
    a = ap.parse_args()
    out = run_study(range(a.train_seeds), range(a.train_seeds, a.train_seeds + a.eval_seeds),
                    a.fine, a.ratio, a.spinup, a.steps, a.iters, a.batch,
                    ((0.1, 1), (0.3, max(a.unroll // 4, 1)), (0.6, a.unroll))
                    if a.unroll > 1 else ((1.0, 1),),
                    log=lambda m: print(m, flush=True), lr0=a.lr0, lr1=a.lr1,
                    loss_w=(a.wrho, 1.0, 1.0, 1.0, 1.0))
    print(json.dumps(out))
