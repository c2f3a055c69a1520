"""Benchmark of the hot path: one MI355X, the driven-turbulence workload at
512^3 in fp32 (OU forcing on 1 <= |n| <= 2 with tau = 0.5, exact optically
thin cooling, CFL 0.4, from rest with rho = 1, p = 1, gamma = 5/3).

A step is one full pass of the method: per-step dt/OU kernel, RK stage 1,
RK stage 2 with forcing, cooling and the CFL reduction fused.  The timed
region holds exactly --steps steps, bracketed by device synchronisation, with
no per-launch events in it; the state is resident in HBM before it starts.
A second pass of the same number of steps records HIP events around every
launch on the library's stream, for the per-kernel durations.  Prints one
JSON line.

value            cell-updates/s = cells * steps / seconds of the timed region
roofline         the dominant kernel (RK stage 2 with the sources and the CFL
                 reduction): algorithmic HBM bytes per launch (60 per cell:
                 read U1 and U^n, write U^{n+1}) over its mean launch duration,
                 against the 8 TB/s HBM peak; `traffic` = HBM bytes per launch
                 from the committed counter summary (null when the kernel
                 source changed since); `alu` = the same launch's algorithmic
                 FLOPs (489 per cell) against the 78.6 TFLOP/s fp32 vector
                 peak without packed instructions
extra            the same step on a second input (band-limited turbulent
                 velocity field, Mach 1) and the paper's fiducial van Leer +
                 HLLC scheme on the headline input
cpu_baseline     the FP64 oracle on the same physics at 256^3 for 2 steps on
                 all of the job's threads, with the CPU model and the rate of
                 one thread (128^3, 2 steps)
corrector        the solver-in-the-loop study: density L2 error of the plain and
                 the corrected 64^3 runs against the block-averaged 256^3 run,
                 and the cost ratio (fine run time / corrected coarse run time)
"""
import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
HBM_TARGET_FRAC = 0.6
# MI355X fp32 vector peak: 256 CUs x 4 SIMDs x 16 lanes x 2 (FMA) x 2.4 GHz =
# 78.6 TFLOP/s with one-lane-per-op instructions (157.3 with packed FP32
# instructions, which this build does not emit)
FP32_VECTOR_PEAK_TFLOPS = 78.6
# algorithmic floating-point operations per cell of one RK stage of the fp32
# method (primitive recovery, 3 faces of limited slopes + face states + HLLC,
# conservative update; stage 2 adds the RK combination, OU kick, exact cooling
# and the CFL signal speed): add, subtract, multiply, reciprocal, square root,
# exp and log count 1, an FMA 2; compares, selects, min/max and the
# median-of-three of minmod count 0 (the convention of the hardware FP32 FLOP
# counter, which reads 405 and 498 per cell executed, the excess being the
# tile-edge faces and halo primitives computed twice)
FLOP_STAGE1 = 396
FLOP_STAGE2 = 489
PMC_FILE = os.path.join(ROOT, "profiles", "pmc_k_stage_512_fp32.md")
KERNEL_SRCS = [os.path.join(ROOT, "paper_2512_13403_amd", "csrc", f)
               for f in ("hydro_kernels.hip", "mh_device.h")]


def kernel_hash():
    """Hash of the sources the stage kernels are compiled from."""
    h = hashlib.sha256()
    for f in KERNEL_SRCS:
        h.update(open(f, "rb").read())
    return h.hexdigest()[:16]


def measured_traffic():
    """HBM bytes per stage-2 launch from the committed rocprofv3 PMC summary,
    or None when missing or when the kernel source changed since."""
    if not os.path.exists(PMC_FILE):
        return None
    rec = {}
    for line in open(PMC_FILE):
        if line.startswith("traffic-record:"):
            for kv in line.split(":", 1)[1].split():
                k, v = kv.split("=")
                rec[k] = v
    if rec.get("kernel_sha256_16") != kernel_hash() or "stage2_bytes" not in rec:
        return None
    return float(rec["stage2_bytes"])


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    import platform

    return platform.processor() or "unknown"


def _oracle_rate(n, steps):
    import oracle
    import workloads as wl

    shape = (n, n, n)
    c = oracle.make_config(shape, (1.0 / n,) * 3, gamma=5.0 / 3.0, cfl=0.4,
                           flags=oracle.SRC_FORCING | oracle.SRC_COOLING)
    sim = oracle.Simulation(c, wl.rest_state(shape))
    t0 = time.perf_counter()
    sim.advance(steps)
    dt = time.perf_counter() - t0
    return n ** 3 * steps / dt, dt


def cpu_baseline(n=256, steps=6, n1=128, steps1=2):
    """The FP64 oracle on the headline physics (forcing + cooling from rest):
    n^3 for `steps` steps on all of the job's OpenMP threads, and n1^3 for
    `steps1` steps on one thread."""
    import oracle

    threads = oracle.num_threads()
    rate, secs = _oracle_rate(n, steps)
    oracle.set_num_threads(1)
    try:
        rate1, secs1 = _oracle_rate(n1, steps1)
    finally:
        oracle.set_num_threads(threads)
    return {"value": rate, "unit": "cell-updates/s", "cores": threads, "kind": "oracle",
            "sample": f"same physics (forcing + cooling, from rest) at {n}^3 for {steps} steps, "
                      f"fp64, OpenMP over {threads} threads, {secs:.1f} s",
            "cpu_model": cpu_model(),
            "one_core_value": rate1,
            "one_core_sample": f"{n1}^3 for {steps1} steps on 1 thread, {secs1:.1f} s"}


def corrector_study():
    """Second half of the metric: 16 driven-turbulence trajectories (forcing
    only, seeds 0..15), fine 256^3 block-averaged to 64^3 as targets; the
    corrector is trained on seeds 0..11 (500 ADAM iterations) and the plain and
    corrected 64^3 runs are compared over 100 coarse steps on seeds 12..15."""
    from paper_2512_13403_amd import sil

    out = sil.run_study(log=lambda m: print("# " + m, file=sys.stderr, flush=True))
    out["metric"] = "density rel. L2 error vs block-averaged 256^3 after 100 coarse steps"
    return out


def adjoint_probe(n=256, reps=10):
    """Adjoint steps of the hydro step with forcing and cooling (no gravity)
    from a smooth random state, recomputing the step's stages and from the
    stages kept by mh_step_keep, against forward steps of the same solver."""
    import torch

    import paper_2512_13403_amd as mh
    import workloads as wl

    s = mh.Solver(mh.grid_desc((n,) * 3, (1.0 / n,) * 3, dtype="f32"),
                  mh.physics_desc(flags=mh.SRC_FORCING | mh.SRC_COOLING))
    s.set_state(torch.tensor(wl.smooth_random_state((n,) * 3, seed=3, kmax=4),
                             dtype=torch.float32, device="cuda"))
    _, k0 = s.clock()
    ahat = s.ou_state()
    Un = s.get_state_device().clone()
    dt = float(s.step(1, 0.0, record=True)[0])
    lam = torch.randn(Un.shape, generator=torch.Generator(device="cuda").manual_seed(1),
                      device="cuda")
    for _ in range(2):
        s.adjoint_step(Un, dt, k0, lam, ou_ahat=ahat)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        s.adjoint_step(Un, dt, k0, lam, ou_ahat=ahat)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    # the same adjoint step from the stages kept by the forward step
    s.set_state(Un)
    s.set_clock(0.0, k0)
    s.set_ou_state(ahat)
    U1, Ub = s.new_state_tensor(), s.new_state_tensor()
    s.step_keep(dt, U1, Ub)
    for _ in range(2):
        s.adjoint_step(Un, dt, k0, lam, ou_ahat=ahat, kept=(U1, Ub))
    torch.cuda.synchronize()
    t4 = time.perf_counter()
    for _ in range(reps):
        s.adjoint_step(Un, dt, k0, lam, ou_ahat=ahat, kept=(U1, Ub))
    torch.cuda.synchronize()
    t5 = time.perf_counter()
    s.set_state(Un)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    s.step(reps, dt)
    torch.cuda.synchronize()
    t3 = time.perf_counter()
    print(f"adjoint probe {n}^3 f32: adjoint step {1e3 * (t1 - t0) / reps:.3f} ms, "
          f"from kept stages {1e3 * (t5 - t4) / reps:.3f} ms, "
          f"forward step {1e3 * (t3 - t2) / reps:.3f} ms", flush=True)


def stage_probe(n=512, steps=20, extra_schemes=False):
    """Short runs of the 512^3 fp32 step in configurations that differ by one
    phase of the method (slopes off, each source on or off, the van Leer
    limiter; with extra_schemes also MC, superbee, HLL and Rusanov), timed
    side by side and for per-kernel instruction counters: one text line
    each."""
    import torch

    import paper_2512_13403_amd as mh

    base = dict(cool=(0.3, 1e-2, 1e-3, 1e-4), ou_seed=0, ou_tau=0.5, ou_arms=1.0, ou_zeta=1.0,
                ou_kmin=1.0, ou_kmax=2.0)
    F, C = mh.SRC_FORCING, mh.SRC_COOLING
    H = mh.RS_HLLC
    cases = (("minmod, forcing + cooling", mh.LIM_MINMOD, H, F | C),
             ("first order, forcing + cooling", mh.LIM_NONE, H, F | C),
             ("minmod, no sources", mh.LIM_MINMOD, H, 0),
             ("minmod, forcing", mh.LIM_MINMOD, H, F),
             ("minmod, cooling", mh.LIM_MINMOD, H, C),
             ("van Leer, forcing + cooling", mh.LIM_VANLEER, H, F | C))
    if extra_schemes:
        # the kernels that take the limiter and the solver at run time
        cases += (("MC + HLLC, forcing + cooling", mh.LIM_MC, H, F | C),
                  ("superbee + HLLC, forcing + cooling", mh.LIM_SUPERBEE, H, F | C),
                  ("minmod + HLL, forcing + cooling", mh.LIM_MINMOD, mh.RS_HLL, F | C),
                  ("minmod + Rusanov, forcing + cooling", mh.LIM_MINMOD, mh.RS_RUSANOV, F | C))
    for name, lim, rs, flags in cases:
        s = mh.Solver(mh.grid_desc((n,) * 3, (1.0 / n,) * 3, dtype="f32", gamma=GAMMA, cfl=0.4,
                                   limiter=lim, riemann=rs), mh.physics_desc(flags=flags, **base))
        s.set_state(rest_state_device(n, "f32"))
        s.step(1, 0.0)
        s.set_timing(True)
        ms, _ = timed_steps(s, steps)
        t, launches = s.timing()
        print(f"stage probe {n}^3 f32 [{name}]: {ms / steps:.3f} ms/step, stage 1 "
              f"{t[mh.TIME_STAGE1] / launches[mh.TIME_STAGE1]:.3f} ms, stage 2 "
              f"{t[mh.TIME_STAGE2] / launches[mh.TIME_STAGE2]:.3f} ms", flush=True)
        del s
        torch.cuda.empty_cache()


def corrector_probe(n=64, batch=4, reps=10):
    """The corrector's kernels at the solver-in-the-loop size (batch 4 x 64^3,
    fp32 states): forward passes, then training steps (forward, loss,
    reverse pass with the input gradient, ADAM); one text line."""
    import numpy as np
    import torch

    import paper_2512_13403_amd as mh
    import workloads as wl

    U = torch.tensor(np.stack([wl.smooth_random_state((n,) * 3, seed=s, kmax=4)
                               for s in range(batch)]), dtype=torch.float32, device="cuda")
    T = U + 0.01 * torch.randn(U.shape, generator=torch.Generator(device="cuda").manual_seed(0),
                               device="cuda")
    Ud = U.double().cpu().numpy()
    mean, std = Ud.mean(axis=(0, 2, 3, 4)), Ud.std(axis=(0, 2, 3, 4)) + 1e-3
    c = mh.Corrector(mh.corr_desc(n, batch, "f32", GAMMA, mean, std, (1e-2,) * 5, (1.0,) * 5))
    c.set_params(wl.corrector_init_params(seed=0, out_scale=1.0).astype(np.float32))
    out = torch.empty_like(U)
    for _ in range(2):
        c.apply(U, out, stats=False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        c.apply(U, out, stats=False)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for _ in range(reps):
        c.zero_grad()
        c.backward(U, T, None, input_grad=True)
        c.adam_step(1e-4)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    print(f"corrector probe {batch} x {n}^3 f32: apply {1e3 * (t1 - t0) / reps:.3f} ms, "
          f"training step {1e3 * (t2 - t1) / reps:.3f} ms", flush=True)


def c4_probe(n=128, nsteps=20, K=20):
    """The self-gravitating cooling box at 128^3 (GRF density, multigrid
    gravity with the default V-cycle and red-black Gauss-Seidel smoother):
    per dtype, the forward CFL steps of a checkpointed rollout, the mean
    multigrid cycles per step, and the adjoint rollout over them; one text
    line per dtype."""
    import numpy as np
    import torch

    import paper_2512_13403_amd as mh
    import workloads as wl
    from paper_2512_13403_amd import rollout as ro

    for dtype, tol in (("f64", 1e-10), ("f32", 1e-5)):
        s = mh.Solver(mh.grid_desc((n,) * 3, (1.0 / n,) * 3, dtype=dtype),
                      mh.physics_desc(flags=mh.SRC_GRAVITY | mh.SRC_COOLING, grav_G=wl.JEANS_G,
                                      mg_tol=tol))
        U0 = torch.tensor(wl.grf_density_state(n, seed=0), dtype=s.torch_dtype, device="cuda")
        ro.rollout_forward(s, U0, 2, K)  # graphs captured, caches warm
        s.set_clock(0.0, 0)
        s.set_potential(np.zeros((n,) * 3))
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        cycles = 0
        s.set_state(U0)
        cks = []
        dts = []
        for k in range(nsteps):
            if k % K == 0:
                cks.append(ro._snapshot(s))
            dts.append(float(s.step(1, 0.0, record=True)[0]))
            cycles += s.mg_cycles()
        Uf = s.get_state_device()
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        lam = torch.zeros_like(Uf)
        lam[0] = Uf[0] - 1.0
        ro.rollout_backward(s, cks, np.array(dts), K, lam)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        print(f"c4 probe {n}^3 {dtype}: forward {1e3 * (t1 - t0) / nsteps:.3f} ms/step "
              f"({cycles / nsteps:.1f} cycles/step), adjoint rollout "
              f"{1e3 * (t2 - t1) / nsteps:.3f} ms/step", flush=True)
        del s


def fft_gravity_probe(n=512):
    """Three checkpointed steps with spectral gravity and cooling on a
    Gaussian-random-field density, then ten standalone 3D transforms."""
    import torch

    import paper_2512_13403_amd as mh
    import workloads as wl
    from paper_2512_13403_amd import rollout as ro

    s = mh.Solver(mh.grid_desc((n,) * 3, (1.0 / n,) * 3, dtype="f32"),
                  mh.physics_desc(flags=mh.SRC_GRAVITY | mh.SRC_COOLING, grav_G=wl.JEANS_G,
                                  grav_solver=mh.GRAV_FFT))
    U0 = torch.tensor(wl.grf_density_state(n, seed=0), dtype=torch.float32, device="cuda")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ro.rollout_forward(s, U0, 3, 20)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    del U0
    x = torch.randn((n, n, n, 2), dtype=torch.float32, device="cuda")
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    for _ in range(10):
        mh.fft3(x)
    torch.cuda.synchronize()
    t3 = time.perf_counter()
    print(f"fft gravity probe {n}^3 f32: {1e3 * (t1 - t0) / 3:.3f} ms per step (first steps), "
          f"{1e3 * (t3 - t2) / 10:.3f} ms per 3D transform", flush=True)


GAMMA = 5.0 / 3.0


def make_solver(n, dtype, limiter=None):
    """The headline configuration: forcing + cooling, CFL 0.4, gamma 5/3."""
    import paper_2512_13403_amd as mh

    lim = mh.LIM_MINMOD if limiter is None else limiter
    grid = mh.grid_desc((n,) * 3, (1.0 / n,) * 3, dtype=dtype, gamma=GAMMA, cfl=0.4,
                        limiter=lim, riemann=mh.RS_HLLC)
    phys = mh.physics_desc(flags=mh.SRC_FORCING | mh.SRC_COOLING, cool=(0.3, 1e-2, 1e-3, 1e-4),
                           ou_seed=0, ou_tau=0.5, ou_arms=1.0, ou_zeta=1.0, ou_kmin=1.0,
                           ou_kmax=2.0)
    return mh.Solver(grid, phys)


def rest_state_device(n, dtype):
    import torch

    tdt = torch.float32 if dtype == "f32" else torch.float64
    U0 = torch.zeros((5, n, n, n), dtype=tdt, device="cuda:0")
    U0[0] = 1.0
    U0[4] = 1.0 / (GAMMA - 1.0)  # rest, rho = 1, p = 1
    return U0


def turbulent_state_device(n, dtype, seed=0, kmin=2.0, kmax=20.0, power=-5.0 / 3.0, mach=1.0):
    """Band-limited solenoidal velocity field of the Sec. 3.1 construction at
    uniform rho = 1, p = 1: coefficients A(k) P(k) exp(i phi(k)) with
    A = |k|^(power/2) on kmin <= |k| <= kmax, P the solenoidal projector and
    seeded uniform phases, the real part of the library's inverse transform,
    rescaled to rms Mach `mach` (a synthetic input built on the device)."""
    import torch

    import paper_2512_13403_amd as mh

    dev = "cuda:0"
    tdt = torch.float32 if dtype == "f32" else torch.float64
    k1 = torch.arange(n, device=dev, dtype=tdt)
    k1 = torch.where(k1 > n // 2, k1 - n, k1)
    kx, ky, kz = k1.view(1, 1, n), k1.view(1, n, 1), k1.view(n, 1, 1)
    k2 = kx * kx + ky * ky + kz * kz
    k = torch.sqrt(k2)
    A = torch.where((k >= kmin) & (k <= kmax), k.clamp(min=1.0) ** (power / 2.0),
                    torch.zeros_like(k))
    k2s = torch.where(k2 > 0, k2, torch.ones_like(k2))
    gen = torch.Generator(device=dev).manual_seed(seed)
    ph = torch.rand((3, n, n, n), generator=gen, device=dev, dtype=tdt) * (2.0 * math.pi)
    er, ei = torch.cos(ph), torch.sin(ph)
    del ph
    dr = (kx * er[0] + ky * er[1] + kz * er[2]) / k2s
    di = (kx * ei[0] + ky * ei[1] + kz * ei[2]) / k2s
    u = []
    for i, ki in enumerate((kx, ky, kz)):
        X = torch.empty((n, n, n, 2), dtype=tdt, device=dev)
        X[..., 0] = A * (er[i] - ki * dr)
        X[..., 1] = A * (ei[i] - ki * di)
        mh.fft3(X, inverse=True)
        u.append(X[..., 0].clone())
        del X
    del er, ei, dr, di
    v = torch.stack(u)
    del u
    cs = math.sqrt(GAMMA)
    v *= mach * cs / torch.sqrt((v * v).sum(dim=0).mean())
    U = torch.empty((5, n, n, n), dtype=tdt, device=dev)
    U[0] = 1.0
    U[1:4] = v
    U[4] = 1.0 / (GAMMA - 1.0) + 0.5 * (v * v).sum(dim=0)
    del v
    torch.cuda.empty_cache()
    return U


def timed_steps(s, steps):
    """(GPU ms from events on the solver's stream, wall seconds) of `steps`
    CFL steps, bracketed by device synchronisation."""
    import torch

    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    w0 = time.perf_counter()
    ev0.record(s.stream)
    s.step(steps, 0.0)
    ev1.record(s.stream)
    torch.cuda.synchronize()
    return ev0.elapsed_time(ev1), time.perf_counter() - w0


def extra_inputs(n, dtype, steps, warmup):
    """The step on C3's second input (the turbulent velocity field) and the
    paper's fiducial van Leer + HLLC scheme on the headline input, each timed
    like the headline (warm-up, then `steps` steps without per-launch events)."""
    import torch

    import paper_2512_13403_amd as mh

    es = 4 if dtype == "f32" else 8
    out = {}
    cases = (("turbulent_ic", "minmod + HLLC, band-limited solenoidal velocity 2<=|k|<=20, "
                              "E(k) ~ k^-5/3, Mach 1, seed 0, forcing + cooling", None),
             ("vanleer_hllc", "van Leer + HLLC (the paper's fiducial scheme), from rest, "
                              "forcing + cooling", mh.LIM_VANLEER))
    for name, what, lim in cases:
        print(f"# extra input: {name}", file=sys.stderr, flush=True)
        s = make_solver(n, dtype, limiter=lim)
        U0 = turbulent_state_device(n, dtype) if name == "turbulent_ic" else rest_state_device(n, dtype)
        s.set_state(U0)
        torch.cuda.synchronize()
        del U0
        s.step(warmup, 0.0)
        ms, _ = timed_steps(s, steps)
        bad, _ = s.check()
        t_sim, _ = s.clock()
        rate = n ** 3 * steps / (ms / 1e3)
        out[name] = {"workload": f"{n}^3 {dtype}: {what}", "steps": steps,
                     "ms_per_step": ms / steps, "value": rate, "unit": "cell-updates/s",
                     "hbm_frac_step_algorithmic": 25 * es * rate / 1e9 / HBM_PEAK_GBS,
                     "t_end": t_sim, "bad_cells": bad}
        del s
        torch.cuda.empty_cache()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--n", type=int, default=512)
    ap.add_argument("--dtype", default="f32", choices=["f32", "f64"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extra", action="store_true",
                    help="skip the second input and the van Leer scheme")
    ap.add_argument("--no-corrector-study", action="store_true",
                    help="skip the solver-in-the-loop study (fine 256^3 vs corrected 64^3)")
    ap.add_argument("--copy-probe", action="store_true",
                    help="first run one plain 1 GiB device copy (torch copy_ of 2^28 fp32), "
                         "the reference for scaling HBM counters")
    ap.add_argument("--adjoint-probe", action="store_true",
                    help="instead: time adjoint steps at 256^3 fp32 (forcing + cooling) for "
                         "the kernel profiles, one text line")
    ap.add_argument("--stage-probe", action="store_true",
                    help="instead: the 512^3 fp32 step in six configurations that differ by "
                         "one phase (timed side by side, and for instruction counters), one "
                         "text line each")
    ap.add_argument("--probe-steps", type=int, default=20,
                    help="timed steps per configuration of --stage-probe")
    ap.add_argument("--probe-schemes", action="store_true",
                    help="--stage-probe also times MC, superbee, HLL and Rusanov (the "
                         "run-time scheme kernels)")
    ap.add_argument("--corrector-probe", action="store_true",
                    help="instead: corrector forward passes and training steps at 4 x 64^3, "
                         "one text line")
    ap.add_argument("--c4-probe", action="store_true",
                    help="instead: forward and adjoint steps of the 128^3 self-gravitating "
                         "cooling box in fp64 and fp32, one text line each")
    ap.add_argument("--fft-gravity-probe", action="store_true",
                    help="instead: 3 steps with spectral gravity at 512^3 fp32 and 10 "
                         "standalone 3D transforms, for the kernel profiles, one text line")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(--gpus must be 1)", file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_2512_13403_amd as mh

    if args.copy_probe:
        src = torch.ones(1 << 28, dtype=torch.float32, device="cuda:0")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    if args.adjoint_probe:
        return adjoint_probe()
    if args.fft_gravity_probe:
        return fft_gravity_probe()
    if args.c4_probe:
        return c4_probe()
    if args.stage_probe:
        return stage_probe(steps=args.probe_steps, extra_schemes=args.probe_schemes)
    if args.corrector_probe:
        return corrector_probe()

    n = args.n
    shape = (n, n, n)
    N = n ** 3
    es = 4 if args.dtype == "f32" else 8
    s = make_solver(n, args.dtype)
    s.set_state(rest_state_device(n, args.dtype))
    torch.cuda.synchronize()
    print(f"# warmup {args.warmup} steps at {n}^3 {args.dtype}", file=sys.stderr, flush=True)
    s.step(args.warmup, 0.0)
    torch.cuda.synchronize()

    # the timed region: exactly --steps steps, no per-launch events
    gpu_ms, wall = timed_steps(s, args.steps)
    bad, first = s.check()
    t_sim, nstep = s.clock()
    print(f"# timed {args.steps} steps: {gpu_ms:.1f} ms (wall {wall * 1e3:.1f} ms), t = {t_sim:.4f}, "
          f"bad cells {bad}", file=sys.stderr, flush=True)
    if bad:
        raise SystemExit(f"unphysical cells after the run (first at {first})")
    # per-kernel durations: the same number of steps again with HIP events
    # recorded around every launch on the library's stream
    s.set_timing(True)
    pass_ms, _ = timed_steps(s, args.steps)
    ms, launches = s.timing()
    s.set_timing(False)

    seconds = gpu_ms / 1e3
    value = N * args.steps / seconds
    st2_ms = ms[mh.TIME_STAGE2] / max(launches[mh.TIME_STAGE2], 1)
    st1_ms = ms[mh.TIME_STAGE1] / max(launches[mh.TIME_STAGE1], 1)
    bytes2 = 15 * es * N  # read U1, read U^n, write U^{n+1}: 3 x 5 fields
    bytes1 = 10 * es * N  # read U^n, write U1
    ach2 = bytes2 / (st2_ms / 1e3) / 1e9
    ach1 = bytes1 / (st1_ms / 1e3) / 1e9
    traffic = measured_traffic() if args.dtype == "f32" and n == 512 else None
    flops2 = FLOP_STAGE2 * N / (st2_ms / 1e3) / 1e12
    step_frac = 25 * es * value / 1e9 / HBM_PEAK_GBS
    rec = {
        "metric": "cell-updates/s & %HBM BW at 512^3 fp32; corrected-64^3 L2 err vs plain",
        "value": value,
        "unit": "cell-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": gpu_ms / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": args.dtype,
        "data": "synthetic",
        "config": {
            "workload": f"driven turbulence {n}^3 {args.dtype}: PLM minmod + HLLC + SSP-RK2, "
                        "CFL 0.4, solenoidal OU forcing 1<=|n|<=2 tau=0.5, exact cooling, "
                        "from rest rho=1 p=1 gamma=5/3",
            "cells": N,
            "bytes_per_cell_update": 25 * es,
            "effective_GBps": 25 * es * value / 1e9,
            "hbm_frac_step_algorithmic": step_frac,
            "hbm_target_frac": HBM_TARGET_FRAC,
            "hbm_target_met": step_frac >= HBM_TARGET_FRAC,
            "stage1_ms": st1_ms,
            "stage2_ms": st2_ms,
            "prologue_ms": ms[mh.TIME_PROLOGUE] / max(launches[mh.TIME_PROLOGUE], 1),
            "timing_pass_ms_per_step": pass_ms / args.steps,
            "stage1_GBps": ach1,
            "stage2_GBps": ach2,
            "hbm_frac_stage1_algorithmic": ach1 / HBM_PEAK_GBS,
            "hbm_frac_stage2_measured": (traffic / (st2_ms / 1e3) / 1e9 / HBM_PEAK_GBS
                                         if traffic else None),
            "t_end": t_sim,
        },
        "roofline": {
            "bound": "hbm",
            "kernel": "k_stage<2> (RK stage 2 + forcing + cooling + CFL max)",
            "achieved": ach2,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": ach2 / HBM_PEAK_GBS,
            "traffic": traffic,
            "bytes_per_cell": 15 * es,
            "cells_per_launch": N,
            "alu": {"achieved": flops2, "peak": FP32_VECTOR_PEAK_TFLOPS, "unit": "TFLOP/s",
                    "frac": flops2 / FP32_VECTOR_PEAK_TFLOPS, "flop_per_cell": FLOP_STAGE2},
        },
    }
    del s
    torch.cuda.empty_cache()
    if not args.no_extra:
        rec["extra"] = extra_inputs(n, args.dtype, args.steps, args.warmup)
    if not args.no_corrector_study:
        print("# solver-in-the-loop study: fine 256^3, coarse 64^3", file=sys.stderr, flush=True)
        rec["corrector"] = corrector_study()
    if not args.no_cpu_baseline:
        print("# cpu baseline (oracle)", file=sys.stderr, flush=True)
        rec["cpu_baseline"] = cpu_baseline()
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
