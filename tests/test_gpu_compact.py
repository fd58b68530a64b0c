"""The compact fourth-order pair on the GPU (hs_compact_apply) against the
oracle (or_compact_apply) and against its closed-form eigenvalues at full
size.  Single-operator tolerance: 1e-13 relative in the max norm, as for the
other operators."""
import math

import numpy as np
import pytest

import oracle
from paper_1307_7867_amd import inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch as t
    if not t.cuda.is_available():
        pytest.skip("no GPU")
    return t


def rel(a, b):
    return np.abs(np.asarray(a) - np.asarray(b)).max() / max(np.abs(b).max(), 1e-300)


@pytest.mark.parametrize("n", [1, 3, 7, 15, 31, 63, 127])
@pytest.mark.parametrize("alpha,beta", [(1.0, 0.0), (0.0, 1.0), (1.0, -0.004)])
def test_compact_apply_parity(torch, n, alpha, beta):
    from paper_1307_7867_amd import heatst as hs
    us = [inputs.random_field(n, 20 + b) for b in range(2)]
    u = torch.from_numpy(np.concatenate([x.ravel() for x in us])).cuda()
    y = torch.empty_like(u)
    print(f"compact_apply n={n} alpha={alpha} beta={beta}", flush=True)
    hs.compact_apply(u, y, n, 2, alpha, beta)
    got = y.cpu().numpy()
    for b in range(2):
        ref = oracle.compact_apply(us[b], alpha, beta)
        assert rel(got[b * n ** 3:(b + 1) * n ** 3].reshape(n, n, n), ref) <= 1e-13, (n, b)


def test_compact_apply_eigenvalues_at_255(torch):
    """On a sine mode of a 255^3 grid both matrices act as their closed-form
    eigenvalues (an identity that holds at any size)."""
    from paper_1307_7867_amd import heatst as hs
    n, k = 255, (3, 200, 7)
    h = 1.0 / (n + 1)
    x = np.arange(1, n + 1) / (n + 1)
    phi = (np.sin(k[2] * np.pi * x)[:, None, None] * np.sin(k[1] * np.pi * x)[None, :, None]
           * np.sin(k[0] * np.pi * x)[None, None, :])
    c = [math.cos(kk * math.pi * h) for kk in k]
    la = (4 * sum(c) + 4 * (c[0] * c[1] + c[0] * c[2] + c[1] * c[2]) - 24) / (6 * h * h)
    lb = 0.5 + sum(c) / 6
    u = torch.from_numpy(phi.ravel()).cuda()
    y = torch.empty_like(u)
    print(f"compact_apply eigen n={n}", flush=True)
    hs.compact_apply(u, y, n, 1, 0.0, 1.0)
    assert np.abs(y.cpu().numpy() - la * phi.ravel()).max() <= 1e-11 * abs(la)
    hs.compact_apply(u, y, n, 1, 1.0, 0.0)
    assert np.abs(y.cpu().numpy() - lb * phi.ravel()).max() <= 1e-13


# ----------------------------------------------------------------------------
# single-level SDC with the compact pair (plans with order HS_ORDER_COMPACT)
# ----------------------------------------------------------------------------

# FP64 SDC tolerance: the two sides run the same operations except that the
# GPU takes B f of the forcing's sine mode as its eigenvalue times f where the
# oracle applies the stencil, and kernels contract multiply-adds; each solve
# stops at a relative residual of 1e-12, so the states agree to about that
SDC_TOL = 1e-11


def _compact_pair(torch, n, M, u0s, nsteps=1, sweeps=2, sdc_tol=1e-10, max_sweeps=30, lane_n=None, **mgkw):
    from paper_1307_7867_amd import heatst as hs
    kw = dict(nu=0.1, dt=0.05, nsteps=nsteps, sweeps=sweeps, sdc_tol=sdc_tol, max_sweeps=max_sweeps)
    ns = lane_n if lane_n is not None else [n] * len(u0s)
    print(f"compact sdc n={ns} M={M} sweeps={sweeps} nsteps={nsteps} mg={mgkw}", flush=True)
    plan = hs.Plan(hs.Problem(n=n, order=hs.HS_ORDER_COMPACT, nnodes=M, batch=len(u0s), lane_n=lane_n,
                              tol=mgkw.get("tol", 1e-12), fixed_cycles=mgkw.get("fixed_cycles", 0),
                              nu1=mgkw.get("nu1", 2), nu2=mgkw.get("nu2", 1),
                              n_coarsest=mgkw.get("n_coarsest", 3), **kw))
    plan.set_state(torch.from_numpy(np.concatenate([u.ravel() for u in u0s])).cuda())
    plan.solve()
    flat = plan.get_state().cpu().numpy()
    st, stats = plan.stats()
    got, o = [], 0
    for m in ns:
        got.append(flat[o:o + m ** 3].reshape(m, m, m))
        o += m ** 3
    refs = []
    for b, m in enumerate(ns):
        mg = oracle.mg_params(**{k: v for k, v in mgkw.items()})
        refs.append(oracle.run(oracle.problem([(m, oracle.COMPACT, M)], mg=mg, **kw), u0s[b]))
    return st, stats, got, refs


@pytest.mark.parametrize("n", [1, 3, 7, 15, 31])
@pytest.mark.parametrize("M", [2, 3, 5])
def test_compact_sdc_parity(torch, n, M):
    u0 = inputs.random_smooth(n, 4)
    st, stats, got, refs = _compact_pair(torch, n, M, [u0], nsteps=2, sweeps=2)
    ref, s, ost = refs[0]
    assert st == 0 and s == oracle.OK
    assert rel(got[0], ref) <= SDC_TOL
    assert stats[0]["total_cycles"] == ost.total_cycles
    assert stats[0]["total_solves"] == ost.total_solves
    assert stats[0]["steps_done"] == 2


@pytest.mark.parametrize("nu1,nu2,n_coarsest", [(1, 1, 1), (3, 2, 3)])
def test_compact_sdc_cycle_shapes_parity(torch, nu1, nu2, n_coarsest):
    n = 31
    u0 = inputs.random_smooth(n, 6)
    st, stats, got, refs = _compact_pair(torch, n, 3, [u0], sweeps=2, nu1=nu1, nu2=nu2, n_coarsest=n_coarsest)
    ref, s, ost = refs[0]
    assert st == 0 and s == oracle.OK
    assert rel(got[0], ref) <= SDC_TOL
    assert stats[0]["total_cycles"] == ost.total_cycles


def test_compact_sdc_fixed_cycles_parity(torch):
    n = 15
    u0 = inputs.random_smooth(n, 7)
    st, stats, got, refs = _compact_pair(torch, n, 3, [u0], sweeps=3, fixed_cycles=3)
    ref, s, ost = refs[0]
    assert st == 0 and s == oracle.OK
    assert rel(got[0], ref) <= SDC_TOL
    assert stats[0]["total_cycles"] == ost.total_cycles == 3 * 2 * 3


def test_compact_sdc_tolerance_mode_parity(torch):
    """Sweeps until the B-weighted collocation residual meets sdc_tol."""
    n = 15
    u0 = inputs.random_smooth(n, 8)
    st, stats, got, refs = _compact_pair(torch, n, 5, [u0], nsteps=2, sweeps=0, sdc_tol=1e-9)
    ref, s, ost = refs[0]
    assert st == 0 and s == oracle.OK
    assert stats[0]["total_sweeps"] == ost.total_sweeps > 2
    assert rel(got[0], ref) <= SDC_TOL
    assert stats[0]["last_sdc_res"] <= 1e-9


def test_compact_sdc_sweep_cap_reported(torch):
    n = 15
    u0 = inputs.random_smooth(n, 8)
    st, stats, got, refs = _compact_pair(torch, n, 5, [u0], sweeps=0, sdc_tol=1e-13, max_sweeps=2)
    ref, s, ost = refs[0]
    assert s == oracle.ENOCONV
    assert st == hs_status("HS_ENOCONV")
    assert rel(got[0], ref) <= SDC_TOL


def hs_status(name):
    from paper_1307_7867_amd import heatst as hs
    return getattr(hs, name)


def test_compact_sdc_uneven_lanes_parity(torch):
    """Lanes of different sizes in one plan, each against its own oracle run."""
    ns = [15, 7, 31]
    u0s = [inputs.random_smooth(m, 10 + b) for b, m in enumerate(ns)]
    st, stats, got, refs = _compact_pair(torch, 31, 3, u0s, sweeps=2, lane_n=ns)
    assert st == 0
    for b in range(3):
        ref, s, ost = refs[b]
        assert s == oracle.OK
        assert rel(got[b], ref) <= SDC_TOL, b
        assert stats[b]["total_cycles"] == ost.total_cycles, b


def test_compact_sdc_127_parity(torch):
    """The full 127^3 grid: one step, 3 nodes, one sweep."""
    n = 127
    u0 = inputs.random_smooth(n, 3)
    st, stats, got, refs = _compact_pair(torch, n, 3, [u0], sweeps=1)
    ref, s, ost = refs[0]
    assert st == 0 and s == oracle.OK
    assert rel(got[0], ref) <= SDC_TOL
    assert stats[0]["total_cycles"] == ost.total_cycles


def _scalar_sdc(n, M, nu, dt, c, t0, nsteps, sweeps, amp0):
    """SDC of the compact scheme restricted to the sine mode s(x), on which
    A_h and B_h act as their eigenvalues: the scalar recursion of the
    B-weighted sweep with exact substep solves."""
    h = 1.0 / (n + 1)
    cs = math.cos(math.pi * h)
    lam_a = (4.0 * 3 * cs + 4.0 * 3 * cs * cs - 24.0) / (6.0 * h * h)
    lam_b = 0.5 + 3 * cs / 6.0
    tau, Q = oracle.lobatto_nodes(M), oracle.collocation_matrix(M)
    S = np.diff(Q, axis=0)
    amp = amp0
    for k in range(nsteps):
        tn = t0 + k * dt
        g = np.array([-(math.sin(tn + dt * t) - c * nu * math.pi ** 2 * math.cos(tn + dt * t)) for t in tau])
        U = np.full(M, amp)
        for _ in range(sweeps):
            F = nu * lam_a * U + lam_b * g
            SF = dt * (S @ F)
            new = U.copy()
            for m in range(M - 1):
                dtm = dt * (tau[m + 1] - tau[m])
                rhs = lam_b * new[m] - dtm * nu * lam_a * U[m + 1] + SF[m]
                new[m + 1] = rhs / (lam_b - dtm * nu * lam_a)
            U = new
        amp = U[-1]
    return amp


def test_compact_sdc_sine_mode_at_255(torch):
    """At 255^3 (beyond what the oracle runs in seconds): started on the
    sine mode s(x), the state stays a multiple of s(x) and its amplitude is
    the scalar recursion's, to the solves' tolerance."""
    from paper_1307_7867_amd import heatst as hs
    n, M, nsteps, sweeps = 255, 3, 2, 3
    s = inputs.sine_product(n)
    plan = hs.Plan(hs.Problem(n=n, order=hs.HS_ORDER_COMPACT, nnodes=M, nu=0.1, dt=0.05, nsteps=nsteps,
                              sweeps=sweeps, tol=1e-12))
    print(f"compact sdc sine mode n={n}", flush=True)
    plan.set_state(torch.from_numpy(s.ravel().copy()).cuda())
    plan.solve()
    got = plan.get_state().cpu().numpy().reshape(n, n, n)
    st, _ = plan.stats()
    assert st == 0
    amp = _scalar_sdc(n, M, 0.1, 0.05, 3.0, 0.0, nsteps, sweeps, 1.0)
    assert np.abs(got - amp * s).max() <= 1e-10 * abs(amp)


def test_compact_plan_rejects_order_specific_calls(torch):
    """A compact plan refuses the calls that apply the order-2/4 operators
    and an F_I array from outside (HS_EINVAL), and accepts node values."""
    from paper_1307_7867_amd import heatst as hs
    n, M = 7, 3
    plan = hs.Plan(hs.Problem(n=n, order=hs.HS_ORDER_COMPACT, nnodes=M, sweeps=1))
    u = torch.zeros(n ** 3, dtype=torch.float64, device="cuda")
    U = torch.zeros(M * n ** 3, dtype=torch.float64, device="cuda")
    for call in (lambda: plan.lap_apply(u, 1.0, 0.0), lambda: plan.heat_rhs(u, 0.0),
                 lambda: plan.mg_vcycle(u, u.clone(), 0.01), lambda: plan.set_nodes(0, U, U.clone()),
                 lambda: plan.solve_graph()):
        with pytest.raises(hs.HeatstError) as e:
            call()
        assert e.value.status == hs.HS_EINVAL
    plan.set_nodes(0, U, None)


def test_compact_step_level_calls_match_solve(torch):
    """begin_step, sweeps and end_step through the ABI give the state that
    hs_step gives, bit for bit."""
    from paper_1307_7867_amd import heatst as hs
    n, M, K = 15, 3, 2
    u0 = torch.from_numpy(inputs.random_smooth(n, 9).ravel().copy()).cuda()
    pb = hs.Problem(n=n, order=hs.HS_ORDER_COMPACT, nnodes=M, sweeps=K, nsteps=1, tol=1e-12)
    a = hs.Plan(pb)
    a.set_state(u0)
    a.step()
    b = hs.Plan(pb)
    b.set_state(u0)
    b.begin_step()
    for _ in range(K):
        b.sdc_sweep(0)
    b.end_step()
    assert torch.equal(a.get_state(), b.get_state())


# ----------------------------------------------------------------------------
# two-level MLSDC with the compact fine level (B_h^{-1} in the FAS restriction)
# ----------------------------------------------------------------------------

def _compact_mlsdc_pair(torch, nf, Mf, nc, Mc, u0s, nsteps=2, sweeps=2, sdc_tol=1e-10, max_sweeps=30,
                        fas_interp=1):
    from paper_1307_7867_amd import heatst as hs
    kw = dict(nu=0.1, dt=0.05, nsteps=nsteps, sweeps=sweeps, sdc_tol=sdc_tol, max_sweeps=max_sweeps)
    print(f"compact mlsdc {nf}/{nc} M={Mf}/{Mc} sweeps={sweeps} interp={fas_interp} lanes={len(u0s)}", flush=True)
    plan = hs.Plan(hs.Problem(n=nf, order=hs.HS_ORDER_COMPACT, nnodes=Mf, coarse=(nc, 2, Mc), batch=len(u0s),
                              tol=1e-12, fas_interp=fas_interp, **kw))
    plan.set_state(torch.from_numpy(np.concatenate([u.ravel() for u in u0s])).cuda())
    plan.solve()
    flat = plan.get_state().cpu().numpy()
    st, stats = plan.stats()
    got = [flat[b * nf ** 3:(b + 1) * nf ** 3].reshape(nf, nf, nf) for b in range(len(u0s))]
    refs = [oracle.run(oracle.problem([(nf, oracle.COMPACT, Mf), (nc, 2, Mc)], mg=oracle.mg_params(tol=1e-12),
                                      fas_interp=fas_interp, **kw), u) for u in u0s]
    return st, stats, got, refs


@pytest.mark.parametrize("nf,Mf,nc,Mc", [(15, 5, 7, 3), (31, 5, 15, 3), (63, 3, 31, 2)])
def test_compact_mlsdc_parity(torch, nf, Mf, nc, Mc):
    u0 = inputs.random_smooth(nf, 12)
    st, stats, got, refs = _compact_mlsdc_pair(torch, nf, Mf, nc, Mc, [u0])
    ref, s, ost = refs[0]
    assert st == 0 and s == oracle.OK
    assert rel(got[0], ref) <= SDC_TOL
    assert stats[0]["level_cycles"][0] == ost.total_cycles
    assert stats[0]["total_sweeps"] == ost.total_sweeps


def test_compact_mlsdc_tricubic_two_lanes_parity(torch):
    u0s = [inputs.random_smooth(31, 13 + b) for b in range(2)]
    st, stats, got, refs = _compact_mlsdc_pair(torch, 31, 5, 15, 3, u0s, fas_interp=3)
    assert st == 0
    for b in range(2):
        ref, s, ost = refs[b]
        assert s == oracle.OK
        assert rel(got[b], ref) <= SDC_TOL, b
        assert stats[b]["level_cycles"][0] == ost.total_cycles, b


def test_compact_mlsdc_tolerance_mode_parity(torch):
    """Iterations until the B-weighted fine residual meets sdc_tol: the same
    count as the oracle, then the same state."""
    u0 = inputs.random_smooth(15, 14)
    st, stats, got, refs = _compact_mlsdc_pair(torch, 15, 5, 7, 3, [u0], sweeps=0, sdc_tol=1e-8, max_sweeps=60,
                                               fas_interp=3)
    ref, s, ost = refs[0]
    assert st == 0 and s == oracle.OK
    assert stats[0]["total_sweeps"] == ost.total_sweeps > 2
    assert rel(got[0], ref) <= SDC_TOL
    assert stats[0]["last_sdc_res"] <= 1e-8


def test_compact_mlsdc_127_one_iteration_parity(torch):
    """The full 127^3/63^3 hierarchy: one compact MLSDC iteration (B_h^{-1}
    through the sine basis at 127^3, two row tiles of its transform)."""
    u0 = inputs.random_smooth(127, 15)
    st, stats, got, refs = _compact_mlsdc_pair(torch, 127, 3, 63, 2, [u0], nsteps=1, sweeps=1, fas_interp=3)
    ref, s, ost = refs[0]
    assert np.isfinite(got[0]).all(), int((~np.isfinite(got[0])).sum())
    print(f"rel {rel(got[0], ref):.3e}", flush=True)
    assert st == 0 and s == oracle.OK
    assert rel(got[0], ref) <= SDC_TOL
    assert stats[0]["level_cycles"][0] == ost.total_cycles


def test_compact_mlsdc_step_level_calls_match_solve(torch):
    """begin_step, K hs_mlsdc_iter calls and end_step give the state that
    hs_step gives with K iterations, bit for bit."""
    from paper_1307_7867_amd import heatst as hs
    nf, K = 15, 2
    u0 = torch.from_numpy(inputs.random_smooth(nf, 16).ravel().copy()).cuda()
    pb = hs.Problem(n=nf, order=hs.HS_ORDER_COMPACT, nnodes=5, coarse=(7, 2, 3), sweeps=K, nsteps=1, tol=1e-12)
    a = hs.Plan(pb)
    a.set_state(u0)
    a.step()
    b = hs.Plan(pb)
    b.set_state(u0)
    b.begin_step()
    for _ in range(K):
        b.mlsdc_iter()
    b.end_step()
    assert torch.equal(a.get_state(), b.get_state())
    for call in (lambda: b.fas_restrict(), lambda: b.fas_interp()):
        with pytest.raises(hs.HeatstError) as e:
            call()
        assert e.value.status == hs.HS_EINVAL
