"""Parity at the full benchmark sizes, in the launch configuration the
benchmark times.

* 511^3 (the largest grid): one weighted-Jacobi sweep of the 4th-order
  operator, element by element against the oracle.
* 127^3 fine / 63^3 coarse two-level MLSDC (the headline workload): one
  MLSDC iteration of the first step, every node of both levels against the
  oracle.  The multigrid runs a fixed 2 V(2,1) cycles per solve so the CPU
  oracle finishes in seconds; the kernels, tables and launch shapes are the
  ones of the tolerance-driven benchmark run.
* 255^3, 4th order, 5 nodes, FP64 multigrid, SDC swept to a residual of
  1e-10, 8 random sine modes (the mixed-precision runs of this configuration
  are in test_gpu_configs.py): the CPU oracle is too slow at this size, so
  the end state is compared with the exact collocation solution (per-mode
  solve of eq. (6), which converged SDC reaches).  Bound: the SDC residual
  R <= sdc_tol per step maps to an error
  of at most ||(I - z Q)^{-1}|| * R <= 1.7 R per step over all stiffness
  z = dt nu lambda <= 0 (5 Lobatto nodes; checked by the
  oracle pin test_collocation_inverse_bound), the step map is a contraction, so after
  K steps the error is below 1.7 K sdc_tol per mode; the test allows
  4 K sdc_tol in the max norm.
"""
import numpy as np
import pytest

import oracle
from oracle import collocation
from paper_1307_7867_amd import inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch as t
    if not t.cuda.is_available():
        pytest.skip("no GPU")
    return t


def dev(torch, a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64).ravel()).cuda()


def host(t):
    return t.detach().cpu().numpy()


def rel(a, b):
    return np.abs(np.asarray(a) - np.asarray(b)).max() / max(np.abs(b).max(), 1e-300)


def test_jacobi_511_parity(torch):
    from paper_1307_7867_amd import heatst as hs
    n = 511
    a = 0.1 * 0.05 * 0.17267316464601146
    plan = hs.Plan(hs.Problem(n=n, order=4, nnodes=2, nu=0.1, dt=0.05, sweeps=1, fixed_cycles=1))
    rng = np.random.default_rng(511)
    u = rng.standard_normal(n ** 3)
    b = rng.standard_normal(n ** 3)
    du, db = dev(torch, u), dev(torch, b)
    tmp = torch.empty_like(du)
    plan.smooth(du, db, tmp, a, 1)
    got = host(du).reshape(n, n, n)
    del du, db, tmp
    torch.cuda.empty_cache()
    ref = oracle.jacobi(u.reshape(n, n, n), b.reshape(n, n, n), 4, a)
    assert rel(got, ref) <= 1e-13


def test_mlsdc_127_first_iteration_parity(torch):
    from paper_1307_7867_amd import heatst as hs
    nf, nc, nu, dt = 127, 63, 0.1, 0.05
    pb = hs.Problem(n=nf, order=4, nnodes=5, coarse=(nc, 2, 3), nu=nu, dt=dt, t0=0.0, forcing_c=3.0,
                    nsteps=20, sweeps=3, nu1=2, nu2=1, omega=6.0 / 7.0, n_coarsest=3, fixed_cycles=2)
    plan = hs.Plan(pb)
    u0 = inputs.sine_product(nf)
    plan.set_state(dev(torch, u0))
    plan.begin_step()
    plan.mlsdc_iter()
    gUf, gFf, _, _ = plan.get_nodes(0)
    gUc, _, _, gtau = plan.get_nodes(1)
    torch.cuda.synchronize()

    opb = oracle.problem([(nf, 4, 5), (nc, 2, 3)], nu=nu, dt=dt, nsteps=1, sweeps=1, forcing_c=3.0,
                         mg=oracle.mg_params(fixed_cycles=2))
    Uf, FIf = oracle.spread(opb.lev[0], nu, u0)
    Uc = np.zeros((3, nc, nc, nc))
    FIc, Ut, tau = np.zeros_like(Uc), np.zeros_like(Uc), np.zeros_like(Uc)
    oracle.mlsdc_iter(opb, 0.0, Uf, FIf, Uc, FIc, Ut, tau)
    assert rel(host(gUf).reshape(Uf.shape), Uf) <= 1e-12
    assert rel(host(gFf).reshape(FIf.shape), FIf) <= 1e-11
    assert rel(host(gUc).reshape(Uc.shape), Uc) <= 1e-12
    # tau is a difference of time integrals dt*Q*F, so it carries the tolerance of F
    # (1e-11 relative: the 1/h^2 of the stencil amplifies rounding in U) times dt
    assert np.abs(host(gtau).reshape(tau.shape) - tau).max() <= 1e-11 * dt * np.abs(FIf).max()


def test_fp64_255_vs_collocation(torch):
    from paper_1307_7867_amd import heatst as hs
    n, M, nu, dt, nsteps, sdc_tol = 255, 5, 0.1, 0.02, 2, 1e-10
    precision = "fp64"
    modes = inputs.random_modes(0)
    pb = hs.Problem(n=n, order=4, nnodes=M, nu=nu, dt=dt, nsteps=nsteps, sweeps=0, sdc_tol=sdc_tol,
                    max_sweeps=40, precision=hs.HS_FP64, tol=1e-12, max_cycles=80)
    plan = hs.Plan(pb)
    plan.set_state(dev(torch, inputs.modes_field(n, modes)))
    plan.solve()
    st, stats = plan.stats()
    assert st == 0
    got = host(plan.get_state()).reshape(n, n, n)
    del plan
    torch.cuda.empty_cache()
    ref = collocation.field(n, collocation.coefficients(n, 4, M, nu, 0.0, dt, nsteps, modes))
    err = np.abs(got - ref).max()
    print(f"255^3 {precision}: max |u - u_collocation| = {err:.3e} (bound {4 * nsteps * sdc_tol:.1e})")
    assert err <= 4 * nsteps * sdc_tol
