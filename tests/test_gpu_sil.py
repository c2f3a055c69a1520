"""GPU checks of the solver-in-the-loop study's plumbing at small sizes: the
coarse run's forcing path equals the fine run's group by group (bitwise OU
amplitudes), the targets are exact block averages, and a short training run
lowers the loss."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(autouse=True)
def _name(request):
    print(f"\n[gpu case] {request.node.nodeid}", flush=True)
    yield


def test_coarse_forcing_path_matches_fine_groups():
    from paper_2512_13403_amd import sil

    tr = sil.record_trajectory(seed=3, nf=32, r=4, t_spinup=0.02, nsteps=4)
    assert np.all(np.diff(tr.step) == 1) and tr.fine_steps == 16
    c = sil.make_solver(8, 3, 1)
    c.set_state(tr.T[0])
    c.set_ou_state(tr.ahat[0])
    c.set_clock(float(tr.t[0]), int(tr.step[0]))
    for k in range(4):
        c.step(1, float(tr.dts[k]))
        assert np.array_equal(c.ou_state(), tr.ahat[k + 1])
        t, st = c.clock()
        assert st == tr.step[k + 1] and t == pytest.approx(tr.t[k + 1], rel=1e-14)
    # the coarse step tracks the block-averaged fine run (same forcing, same times)
    U = c.get_state_device()
    err = float((U[0] - tr.T[4][0]).abs().max())
    assert err < 0.05


def test_short_study_trains_and_evaluates():
    from paper_2512_13403_amd import sil

    trajs = [sil.record_trajectory(seed=s, nf=64, r=4, t_spinup=0.05, nsteps=4) for s in (0, 1)]
    res = sil.train(trajs, 16, iters=40, batch=2)
    assert np.isfinite(res.losses).all()
    assert np.mean(res.losses[-5:]) < res.losses[0]
    ev = sil.evaluate(trajs, 16, res)
    for mode in ("plain", "corrected"):
        errs = np.array(ev[mode]["rho_rel_l2"])
        assert errs.shape == (2, 4) and np.isfinite(errs).all()
    assert ev["cost_ratio"] > 0 and ev["seeds"] == [0, 1]
    # the batched corrected rollout equals trajectory-by-trajectory rollouts
    one = sil.evaluate(trajs[1:], 16, res)
    assert np.array_equal(np.array(one["corrected"]["rho_rel_l2"][0]),
                          np.array(ev["corrected"]["rho_rel_l2"][1]))


def test_unrolled_training_through_the_adjoint():
    """Solver-in-the-loop iterations (3 corrected steps, back-propagated through
    the corrector and mh_adjoint_step) run and keep the loss finite."""
    from paper_2512_13403_amd import sil

    trajs = [sil.record_trajectory(seed=s, nf=64, r=4, t_spinup=0.05, nsteps=5) for s in (2, 3)]
    res = sil.train(trajs, 16, iters=12, batch=2, schedule=((0.5, 1), (0.5, 3)))
    assert len(res.losses) == 12 and np.isfinite(res.losses).all()
    assert np.isfinite(res.theta).all()


def test_trained_corrector_beats_the_plain_coarse_run():
    """What the learned part gains: a corrector trained through the solver
    (pairs, then unrolls of 4 and 16 steps back-propagated through
    mh_adjoint_step) lowers the density L2 error of held-out 32^3 runs against
    the block-averaged 128^3 run, over 50 coarse steps, below the plain 32^3
    run's.  Everything is seeded and the kernels are deterministic."""
    from paper_2512_13403_amd import sil

    train = [sil.record_trajectory(s, 128, 4, 1.0, 50) for s in range(6)]
    held = [sil.record_trajectory(s, 128, 4, 1.0, 50) for s in (100, 101)]
    res = sil.train(train, 32, iters=300, batch=4, schedule=((0.1, 1), (0.3, 4), (0.6, 16)))
    ev = sil.evaluate(held, 32, res)
    plain = np.array(ev["plain"]["rho_rel_l2"])
    corr = np.array(ev["corrected"]["rho_rel_l2"])
    print(f"rho rel. L2 after 50 steps: plain {plain[:, -1]}, corrected {corr[:, -1]}")
    assert ev["corrected"]["fallbacks"] == 0
    assert corr[:, -1].mean() < 0.95 * plain[:, -1].mean()
    assert corr.mean() < plain.mean()
