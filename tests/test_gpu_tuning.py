"""Launch shapes from the autotuner's table change the blocks, not the
arithmetic: every shape gives bitwise the same results (each point's
stencil, restriction and prolongation sums are formed in the same order
whatever z chunk a block marches).  And the launch timer counts what it
should: one k_pjac launch per fine-level V-cycle of a batched solve."""
import numpy as np
import pytest

from paper_1307_7867_amd import inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch as t
    if not t.cuda.is_available():
        pytest.skip("no GPU")
    return t


def _mlsdc(hs, torch, nsteps=2):
    pb = hs.Problem(n=63, order=4, nnodes=5, coarse=(31, 2, 3), nu=0.1, dt=0.02, nsteps=nsteps, sweeps=2,
                    tol=1e-12, max_cycles=60, batch=3, nslices=1)
    plan = hs.Plan(pb)
    u0 = np.concatenate([inputs.random_smooth(63, 40 + i).ravel() for i in range(3)])
    plan.set_state(torch.from_numpy(u0).cuda())
    plan.solve()
    st, stats = plan.stats()
    assert st == 0
    return plan.get_state().cpu().numpy(), stats


def _uneven(hs, torch):
    ns = [31, 63, 15, 63, 31]
    pb = hs.Problem(n=31, order=2, nnodes=3, nu=0.1, dt=0.02, nsteps=2, sweeps=2, tol=1e-12, max_cycles=60,
                    batch=len(ns), lane_n=ns, precision=hs.HS_MIXED)
    plan = hs.Plan(pb)
    u0 = np.concatenate([inputs.random_smooth(n, 60 + i).ravel() for i, n in enumerate(ns)])
    plan.set_state(torch.from_numpy(u0).cuda())
    plan.solve()
    st, _ = plan.stats()
    assert st == 0
    return plan.get_state().cpu().numpy()


@pytest.mark.parametrize("shape", [(1, 2), (4, 8), (16, 16), (32, 32)])
def test_tuned_shapes_are_bitwise_equal(torch, shape):
    from paper_1307_7867_amd import heatst as hs
    hs.tune_clear()
    try:
        ref, rstats = _mlsdc(hs, torch)
        uref = _uneven(hs, torch)
        zb, zr = shape
        for n in (63, 31, 15):
            for order in (2, 4):
                for prec in (0, 1):
                    for batch in (1, 2, 3):
                        hs.tune_set(n, order, prec, batch, zb, zr)
        assert hs.tune_lookup(63, 4, 0, 3) == (zb, zr)
        got, gstats = _mlsdc(hs, torch)
        assert np.array_equal(got, ref)
        assert [s["total_cycles"] for s in gstats] == [s["total_cycles"] for s in rstats]
        assert np.array_equal(_uneven(hs, torch), uref)
    finally:
        hs.tune_clear()


def test_launch_timer_counts_fine_cycles(torch):
    from paper_1307_7867_amd import heatst as hs
    pb = hs.Problem(n=63, order=4, nnodes=5, coarse=(31, 2, 3), nu=0.1, dt=0.01, nsteps=4, sweeps=2, tol=1e-12,
                    max_cycles=60, batch=4, nslices=4)
    plan = hs.Plan(pb)
    plan.set_state(torch.from_numpy(inputs.sine_product(63).ravel()).cuda())
    plan.timer(hs.HS_TIMER_PJAC, 4096)
    plan.pfasst_run()
    launches, ms = plan.timer_read()
    st, stats = plan.stats()
    assert st == 0
    # a batched cycle launches k_pjac once for all lanes, as many times per
    # solve as the lane that needs the most cycles
    fine = [s["level_cycles"][0] for s in stats]
    assert launches >= max(fine) > 0
    assert 0.0 < ms / launches < 10.0
    plan.timer(0, 0)
    plan.set_state(torch.from_numpy(inputs.sine_product(63).ravel()).cuda())
    plan.pfasst_run()
    assert plan.timer_read() == (0, 0.0)
