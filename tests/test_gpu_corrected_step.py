"""The corrector inside the step (mh_step_corrected, the solver-in-the-loop
update of Sec. 8): B coarse contexts advanced together, each step their plain
steps, one batched corrector pass and the scatter back, enqueued by the
library alone (kernel by kernel or replayed from a captured HIP graph).
Checked bitwise against the same sequence driven from the host (mh_step,
mh_get_state, mh_corr_apply, mh_set_state), for fixed steps from a device
schedule and for CFL steps, with forcing; fallbacks counted; argument errors."""
import numpy as np
import pytest

import paper_2512_13403_amd as mh
import workloads as wl

pytestmark = pytest.mark.gpu

GAMMA = 5.0 / 3.0


@pytest.fixture(autouse=True)
def _name(request):
    print(f"\n[gpu case] {request.node.nodeid}", flush=True)
    yield


def make_case(n, B, dtype, fallback_frac=1e-3, scale=(1e-2,) * 5, flags=mh.SRC_FORCING):
    import torch

    td = torch.float64 if dtype == "f64" else torch.float32
    U0 = [torch.tensor(wl.smooth_random_state((n, n, n), seed=40 + b, kmax=3), dtype=td,
                       device="cuda:0") for b in range(B)]
    Ud = torch.stack(U0).double().cpu().numpy()
    mean = Ud.mean(axis=(0, 2, 3, 4))
    std = Ud.std(axis=(0, 2, 3, 4)) + 1e-3
    corr = mh.Corrector(mh.corr_desc(n, B, dtype, GAMMA, mean, std, scale, (1.0,) * 5, 1e-6,
                                     fallback_frac))
    corr.set_params(wl.corrector_init_params(seed=5, out_scale=1.0).astype(np.float32))

    def solvers():
        out = []
        for b in range(B):
            s = mh.Solver(mh.grid_desc((n, n, n), (1.0 / n,) * 3, dtype=dtype, gamma=GAMMA),
                          mh.physics_desc(flags=flags, ou_seed=b))
            s.set_state(U0[b])
            out.append(s)
        return out

    return corr, solvers


def host_loop(solvers, corr, nsteps, dts):
    """The same corrected steps driven from the host."""
    import torch

    B = len(solvers)
    buf = torch.empty((B, 5) + solvers[0].shape, dtype=solvers[0].torch_dtype, device="cuda:0")
    out = torch.empty_like(buf)
    fallbacks = 0
    for k in range(nsteps):
        for b, s in enumerate(solvers):
            s.step(1, float(dts[k, b]) if dts is not None else 0.0)
        for b, s in enumerate(solvers):
            s.get_state_into(buf[b])
        _, _, fb = corr.apply(buf, out)
        fallbacks += int(fb)
        for b, s in enumerate(solvers):
            s.set_state(out[b].clone())
    return [s.get_state_device() for s in solvers], fallbacks


@pytest.mark.parametrize("dtype", ["f32", "f64"])
@pytest.mark.parametrize("cfl", [False, True])
def test_corrected_step_equals_host_loop(dtype, cfl):
    import torch

    n, B, nsteps = 16, 3, 6
    corr, solvers = make_case(n, B, dtype)
    dts = None if cfl else torch.tensor(
        1e-3 * (1.0 + np.arange(nsteps * B).reshape(nsteps, B) % 5), dtype=torch.float64,
        device="cuda:0")
    ref, fb_ref = host_loop(solvers(), corr, nsteps, dts.cpu().numpy() if dts is not None else None)
    for use_graph in (False, True):
        ss = solvers()
        fb = mh.step_corrected(ss, corr, nsteps, dts, use_graph=use_graph, count_fallbacks=True)
        assert fb == fb_ref == 0
        for b, s in enumerate(ss):
            got = s.get_state_device()
            assert torch.equal(got, ref[b]), (use_graph, b, (got - ref[b]).abs().max().item())
            t, k = s.clock()
            assert k == nsteps and t > 0
        # a second call continues from where the first stopped (schedule restarts)
        if not cfl:
            mh.step_corrected(ss, corr, 2, dts[:2].contiguous(), use_graph=use_graph)
            assert ss[0].clock()[1] == nsteps + 2


def test_corrected_step_counts_fallbacks():
    import torch

    # a large output scale drives densities below the floor: every step falls back
    n, B, nsteps = 16, 2, 3
    corr, solvers = make_case(n, B, "f32", fallback_frac=1e-3, scale=(5.0, 0.0, 0.0, 0.0, 5.0))
    ref, fb_ref = host_loop(solvers(), corr, nsteps, None)
    ss = solvers()
    fb = mh.step_corrected(ss, corr, nsteps, None, use_graph=True, count_fallbacks=True)
    assert fb == fb_ref == nsteps
    for b, s in enumerate(ss):
        assert torch.equal(s.get_state_device(), ref[b])


def test_corrected_step_rejects_bad_arguments():
    import torch

    n, B = 16, 2
    corr, solvers = make_case(n, B, "f32")
    ss = solvers()
    with pytest.raises(mh.MHError):  # batch mismatch
        mh.step_corrected(ss[:1], corr, 1)
    with pytest.raises(mh.MHError):  # repeated context
        mh.step_corrected([ss[0], ss[0]], corr, 1)
    other = mh.Solver(mh.grid_desc((n, n, n), (1.0 / n,) * 3, dtype="f64", gamma=GAMMA))
    with pytest.raises(mh.MHError):  # dtype mismatch
        mh.step_corrected([ss[0], other], corr, 1)
    grav = mh.Solver(mh.grid_desc((n, n, n), (1.0 / n,) * 3, dtype="f32", gamma=GAMMA),
                     mh.physics_desc(flags=mh.SRC_GRAVITY, grav_G=1.0))
    grav.set_state(ss[1].get_state_device())
    with pytest.raises(mh.MHError):  # gravity in a captured step
        mh.step_corrected([ss[0], grav], corr, 1, use_graph=True)
    # without a graph the gravity context steps
    mh.step_corrected([ss[0], grav], corr, 1, use_graph=False)
    torch.cuda.synchronize()
