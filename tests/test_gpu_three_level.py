"""Three-level MLSDC and PFASST on the GPU against the oracle (section 1.1:
MLSDC iterations over a hierarchy of levels with fewer nodes and points, tied
together by the FAS correction).  Levels: 4th-order fine grid with 5 nodes,
2nd-order grids with 3 and 2 nodes below it.  FP64 tolerance as in the other
parity tests: 1e-12 relative in the max norm."""
import numpy as np
import pytest

import oracle
from paper_1307_7867_amd import inputs

pytestmark = pytest.mark.gpu

TOL = 1e-12


@pytest.fixture(scope="module")
def torch():
    import torch as t
    if not t.cuda.is_available():
        pytest.skip("no GPU")
    return t


def hs_mod():
    from paper_1307_7867_amd import heatst
    return heatst


def dev(torch, a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64).ravel()).cuda()


def rel(a, b):
    return np.abs(np.asarray(a) - np.asarray(b)).max() / max(np.abs(b).max(), 1e-300)


def sizes(nf):
    n1 = (nf - 1) // 2
    return n1, (n1 - 1) // 2


def gpu_problem(hs, nf, **kw):
    n1, n2 = sizes(nf)
    return hs.Problem(n=nf, order=4, nnodes=5, coarse=(n1, 2, 3), coarse2=(n2, 2, 2), **kw)


def or_problem(nf, **kw):
    n1, n2 = sizes(nf)
    mg = oracle.mg_params(tol=kw.pop("tol", 1e-12))
    return oracle.problem([(nf, 4, 5), (n1, 2, 3), (n2, 2, 2)], mg=mg, **kw)


def run_gpu(torch, hs, pb, u0, pfasst=False):
    plan = hs.Plan(pb)
    plan.set_state(dev(torch, u0))
    if pfasst:
        plan.pfasst_run()
    else:
        plan.solve()
    n = pb.n
    got = plan.get_state().cpu().numpy().reshape(n, n, n)
    st, stats = plan.stats()
    del plan
    return got, st, stats


@pytest.mark.parametrize("interp", [1, 3])
def test_mlsdc3_fixed_parity(torch, interp):
    hs = hs_mod()
    nf = 31
    u0 = inputs.random_smooth(nf, 21)
    print(f"mlsdc3 fixed nf={nf} interp={interp}", flush=True)
    got, st, stats = run_gpu(torch, hs, gpu_problem(hs, nf, nu=0.1, dt=0.05, nsteps=2, sweeps=3, tol=1e-12,
                                                    fas_interp=interp), u0)
    assert st == 0
    ref, s, _ = oracle.run(or_problem(nf, nu=0.1, dt=0.05, nsteps=2, sweeps=3, fas_interp=interp), u0)
    assert s == oracle.OK
    assert rel(got, ref) <= TOL
    lc = stats[0]["level_cycles"]
    assert lc[0] > 0 and lc[1] > 0 and lc[2] > 0


def test_mlsdc3_tolerance_parity(torch):
    """Iterations until the 1e-10 residual: the oracle's iteration count and result."""
    hs = hs_mod()
    nf = 31
    u0 = inputs.sine_product(nf)
    print(f"mlsdc3 tolerance nf={nf}", flush=True)
    got, st, stats = run_gpu(torch, hs, gpu_problem(hs, nf, nu=0.1, dt=0.01, nsteps=2, sweeps=0, sdc_tol=1e-10,
                                                    max_sweeps=40, tol=1e-12, fas_interp=3), u0)
    assert st == 0
    ref, s, ost = oracle.run(or_problem(nf, nu=0.1, dt=0.01, nsteps=2, sweeps=0, sdc_tol=1e-10, max_sweeps=40,
                                        fas_interp=3), u0)
    assert s == oracle.OK
    assert stats[0]["total_sweeps"] == ost.total_sweeps
    assert rel(got, ref) <= TOL


@pytest.mark.parametrize("pred", [0, 1])
def test_pfasst3_parity(torch, pred):
    """Three-level PFASST over two blocks of 4 slices: the oracle's result."""
    hs = hs_mod()
    nf, P = 15, 4
    u0 = inputs.random_smooth(nf, 11)
    print(f"pfasst3 nf={nf} P={P} pred={pred}", flush=True)
    got, st, _ = run_gpu(torch, hs, gpu_problem(hs, nf, nu=0.1, dt=0.02, nsteps=2 * P, sweeps=3, tol=1e-12,
                                                batch=P, nslices=P, pfasst_pred_sweeps=pred, fas_interp=3),
                         u0, pfasst=True)
    assert st == 0
    ref, s, _ = oracle.pfasst(or_problem(nf, nu=0.1, dt=0.02, nsteps=2 * P, sweeps=3, fas_interp=3), P, u0,
                              pred_sweeps=pred)
    assert s == oracle.OK
    assert rel(got, ref) <= TOL


def test_pfasst3_tolerance_parity(torch):
    """Three-level PFASST iterated to the 1e-9 residual: the oracle's iteration
    count and result."""
    hs = hs_mod()
    nf, P = 15, 4
    u0 = inputs.random_smooth(nf, 12)
    print(f"pfasst3 tolerance nf={nf} P={P}", flush=True)
    got, st, stats = run_gpu(torch, hs, gpu_problem(hs, nf, nu=0.1, dt=0.02, nsteps=P, sweeps=0, sdc_tol=1e-9,
                                                    max_sweeps=40, tol=1e-12, batch=P, nslices=P,
                                                    pfasst_pred_sweeps=1, fas_interp=3), u0, pfasst=True)
    assert st == 0
    ref, s, ost = oracle.pfasst(or_problem(nf, nu=0.1, dt=0.02, nsteps=P, sweeps=0, sdc_tol=1e-9, max_sweeps=40,
                                           fas_interp=3), P, u0, pred_sweeps=1)
    assert s == oracle.OK
    assert stats[0]["total_sweeps"] == ost.sweeps
    assert rel(got, ref) <= TOL


def test_mlsdc3_63_parity(torch):
    """A larger hierarchy (63^3 / 31^3 / 15^3: several tiles per plane, ragged
    tile edges, a multigrid tail on every level), one step of 2 iterations."""
    hs = hs_mod()
    nf = 63
    u0 = inputs.random_smooth(nf, 5)
    print(f"mlsdc3 nf={nf}", flush=True)
    got, st, _ = run_gpu(torch, hs, gpu_problem(hs, nf, nu=0.1, dt=0.02, nsteps=1, sweeps=2, tol=1e-12,
                                                fas_interp=3), u0)
    assert st == 0
    ref, s, _ = oracle.run(or_problem(nf, nu=0.1, dt=0.02, nsteps=1, sweeps=2, fas_interp=3), u0)
    assert s == oracle.OK
    assert rel(got, ref) <= TOL
