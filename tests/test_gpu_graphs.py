"""The multigrid V-cycles replayed from captured HIP graphs give bitwise the
same states as the kernel-by-kernel launches, replay after replay, with eager
work (state uploads, host reads, synchronisation) between the replays; the
adjoint's solves likewise."""
import numpy as np
import pytest

import paper_2512_13403_amd as mh
import workloads as wl
from parity import as_input

pytestmark = pytest.mark.gpu


@pytest.fixture(autouse=True)
def _name(request):
    print(f"\n[gpu case] {request.node.nodeid}", flush=True)
    yield


def make(n, dtype, graphs, cycle=mh.MG_V, smoother=mh.SMOOTH_JACOBI):
    g = mh.grid_desc((n, n, n), (1.0 / n,) * 3, dtype=dtype)
    p = mh.physics_desc(flags=mh.SRC_GRAVITY | mh.SRC_COOLING, grav_G=wl.JEANS_G,
                        mg_tol=1e-9 if dtype == "f64" else 1e-5, mg_max_cycles=12,
                        mg_cycle=cycle, mg_smoother=smoother)
    s = mh.Solver(g, p)
    s.set_graphs(graphs)
    return s


@pytest.mark.parametrize("dtype,cycle,smoother", [("f64", mh.MG_V, mh.SMOOTH_JACOBI),
                                                  ("f32", mh.MG_V, mh.SMOOTH_JACOBI),
                                                  ("f64", mh.MG_W, mh.SMOOTH_RBGS)])
def test_graph_replays_match_eager_launches(dtype, cycle, smoother):
    import torch

    n = 32 if cycle == mh.MG_V else 64
    U0 = as_input(wl.grf_density_state(n, seed=7), dtype)
    sg, se = make(n, dtype, True, cycle, smoother), make(n, dtype, False, cycle, smoother)
    for s in (sg, se):
        s.set_state(U0)
    for k in range(6):
        if k == 3:
            # eager work between replays: a new state from the host
            U1 = sg.get_state()
            U1[0] *= 1.0 + 0.01 * np.cos(np.arange(n) * 2 * np.pi / n)[None, None, :]
            for s in (sg, se):
                s.set_state(U1)
        dg = sg.step(1, 0.0, record=True)
        de = se.step(1, 0.0, record=True)
        assert np.array_equal(dg, de)
        assert sg.mg_cycles() == se.mg_cycles() > 0
        assert np.array_equal(sg.get_state(), se.get_state())
        assert np.array_equal(sg.potential(), se.potential())
        torch.cuda.synchronize()
    # the adjoint step's second solve
    t = torch.float64 if dtype == "f64" else torch.float32
    U = torch.tensor(sg.get_state(), dtype=t, device="cuda:0")
    lam = torch.tensor(np.random.default_rng(3).standard_normal((5, n, n, n)), dtype=t,
                       device="cuda:0")
    phi = sg.potential_device()
    outs = []
    for s in (sg, se, sg):
        outs.append(s.adjoint_step(U, float(dg[0]), 6, lam, phi_n=phi).cpu().numpy())
    assert np.array_equal(outs[0], outs[1]) and np.array_equal(outs[0], outs[2])
