"""Benchmark of the hot path: one MI355X, the driven-turbulence workload at
512^3 in fp32 (OU forcing on 1 <= |n| <= 2 with tau = 0.5, exact optically
thin cooling, CFL 0.4, from rest with rho = 1, p = 1, gamma = 5/3).

A step is one full pass of the method: per-step dt/OU kernel, RK stage 1,
RK stage 2 with forcing, cooling and the CFL reduction fused.  The timed
region holds exactly --steps steps, bracketed by device synchronisation; the
state is resident in HBM before it starts.  Prints one JSON line.

value            cell-updates/s = cells * steps / seconds of the timed region
roofline         the dominant kernel (RK stage 2), which is bound by the fp32
                 vector ALU: algorithmic FLOPs per launch (489 per cell) over
                 its mean duration from HIP events recorded around every launch
                 on the library's stream, against the fp32 vector peak;
                 `traffic` = HBM bytes per launch from the committed counter
                 summary (null when the kernel source changed since); the HBM
                 fractions of the metric are in `config`
cpu_baseline     the FP64 oracle on the same physics at 192^3 for 16 steps
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
# MI355X fp32 vector peak: 256 CUs x 4 SIMDs x 16 lanes x 2 (FMA) x 2.4 GHz =
# 78.6 TFLOP/s with one-lane-per-op instructions, 157.3 with packed FP32
FP32_VECTOR_PEAK_TFLOPS = 157.3
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


def cpu_baseline(n=192, steps=16):
    import numpy as np

    import oracle
    import workloads as wl

    shape = (n, n, n)
    c = oracle.make_config(shape, (1.0 / n,) * 3, gamma=5.0 / 3.0, cfl=0.4,
                           flags=oracle.SRC_FORCING | oracle.SRC_COOLING)
    sim = oracle.Simulation(c, wl.rest_state(shape))
    t0 = time.perf_counter()
    sim.advance(steps)
    dt = time.perf_counter() - t0
    threads = oracle.num_threads()
    return {"value": n ** 3 * steps / dt, "unit": "cell-updates/s", "cores": threads,
            "kind": "oracle",
            "sample": f"same physics (forcing + cooling, from rest) at {n}^3 for {steps} steps, "
                      f"fp64, OpenMP over {threads} threads, {dt:.1f} s"}


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
    from a smooth random state, against forward steps of the same solver."""
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
    s.set_state(Un)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    s.step(reps, dt)
    torch.cuda.synchronize()
    t3 = time.perf_counter()
    print(f"adjoint probe {n}^3 f32: adjoint step {1e3 * (t1 - t0) / reps:.3f} ms, "
          f"forward step {1e3 * (t3 - t2) / reps:.3f} ms", flush=True)


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


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--n", type=int, default=512)
    ap.add_argument("--dtype", default="f32", choices=["f32", "f64"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-corrector-study", action="store_true",
                    help="skip the solver-in-the-loop study (fine 256^3 vs corrected 64^3)")
    ap.add_argument("--copy-probe", action="store_true",
                    help="first run one plain 1 GiB device copy (torch copy_ of 2^28 fp32), "
                         "the reference for scaling HBM counters")
    ap.add_argument("--adjoint-probe", action="store_true",
                    help="instead: time adjoint steps at 256^3 fp32 (forcing + cooling) for "
                         "the kernel profiles, one text line")
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

    if args.adjoint_probe:
        return adjoint_probe()
    if args.fft_gravity_probe:
        return fft_gravity_probe()

    if args.copy_probe:
        src = torch.ones(1 << 28, dtype=torch.float32, device="cuda:0")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    n = args.n
    shape = (n, n, n)
    N = n ** 3
    gamma = 5.0 / 3.0
    grid = mh.grid_desc(shape, (1.0 / n,) * 3, dtype=args.dtype, gamma=gamma, cfl=0.4)
    phys = mh.physics_desc(flags=mh.SRC_FORCING | mh.SRC_COOLING, cool=(0.3, 1e-2, 1e-3, 1e-4),
                           ou_seed=0, ou_tau=0.5, ou_arms=1.0, ou_zeta=1.0, ou_kmin=1.0,
                           ou_kmax=2.0)
    s = mh.Solver(grid, phys)
    tdt = torch.float32 if args.dtype == "f32" else torch.float64
    U0 = torch.zeros((5,) + shape, dtype=tdt, device="cuda:0")
    U0[0] = 1.0
    U0[4] = 1.0 / (gamma - 1.0)  # rest, rho = 1, p = 1
    s.set_state(U0)
    torch.cuda.synchronize()
    del U0
    print(f"# warmup {args.warmup} steps at {n}^3 {args.dtype}", file=sys.stderr, flush=True)
    s.step(args.warmup, 0.0)
    torch.cuda.synchronize()

    s.set_timing(True)
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    w0 = time.perf_counter()
    ev0.record(s.stream)
    s.step(args.steps, 0.0)
    ev1.record(s.stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - w0
    gpu_ms = ev0.elapsed_time(ev1)
    ms, launches = s.timing()
    s.set_timing(False)
    bad, first = s.check()
    t_sim, nstep = s.clock()
    print(f"# timed {args.steps} steps: {gpu_ms:.1f} ms (wall {wall * 1e3:.1f} ms), t = {t_sim:.4f}, "
          f"bad cells {bad}", file=sys.stderr, flush=True)
    if bad:
        raise SystemExit(f"unphysical cells after the run (first at {first})")

    seconds = gpu_ms / 1e3
    value = N * args.steps / seconds
    es = 4 if args.dtype == "f32" else 8
    st2_ms = ms[mh.TIME_STAGE2] / max(launches[mh.TIME_STAGE2], 1)
    st1_ms = ms[mh.TIME_STAGE1] / max(launches[mh.TIME_STAGE1], 1)
    bytes2 = 15 * es * N  # read U1, read U^n, write U^{n+1}: 3 x 5 fields
    bytes1 = 10 * es * N  # read U^n, write U1
    ach2 = bytes2 / (st2_ms / 1e3) / 1e9
    ach1 = bytes1 / (st1_ms / 1e3) / 1e9
    traffic = measured_traffic() if args.dtype == "f32" and n == 512 else None
    flops2 = FLOP_STAGE2 * N / (st2_ms / 1e3) / 1e12
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
            "stage1_ms": st1_ms,
            "stage2_ms": st2_ms,
            "prologue_ms": ms[mh.TIME_PROLOGUE] / max(launches[mh.TIME_PROLOGUE], 1),
            "stage1_GBps": ach1,
            "stage2_GBps": ach2,
            "hbm_frac_stage2_algorithmic": ach2 / HBM_PEAK_GBS,
            "hbm_frac_stage2_measured": (traffic / (st2_ms / 1e3) / 1e9 / HBM_PEAK_GBS
                                         if traffic else None),
            "hbm_frac_step_algorithmic": 25 * es * value / 1e9 / HBM_PEAK_GBS,
            "t_end": t_sim,
        },
        "roofline": {
            "bound": "alu",
            "kernel": "k_stage<2> (RK stage 2 + forcing + cooling + CFL max)",
            "achieved": flops2,
            "peak": FP32_VECTOR_PEAK_TFLOPS,
            "unit": "TFLOP/s",
            "frac": flops2 / FP32_VECTOR_PEAK_TFLOPS,
            "traffic": traffic,
            "flop_per_cell": FLOP_STAGE2,
        },
    }
    del s
    torch.cuda.empty_cache()
    if not args.no_corrector_study:
        print("# solver-in-the-loop study: fine 256^3, coarse 64^3", file=sys.stderr, flush=True)
        rec["corrector"] = corrector_study()
    if not args.no_cpu_baseline:
        print("# cpu baseline (oracle)", file=sys.stderr, flush=True)
        rec["cpu_baseline"] = cpu_baseline()
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
