"""Benchmark workloads besides the headline PFASST run (bench.py).

Each function takes the parsed bench.py arguments and returns one JSON-able
record.  Inputs are synthetic (paper_1307_7867_amd.inputs), generated on the
host and copied to HBM before any timed region.

  sdc15     15^3, 2nd order, 3 nodes, dt 0.125, 8 steps to T = 1, 4 sweeps,
            V(2,1) to 1e-12: per-step latency (launch-bound).
  mlsdc127  two-level MLSDC, fine 127^3 4th order 5 nodes, coarse 63^3 2nd
            order 3 nodes, dt 0.05, 20 steps, 3 iterations: DOF-updates/s and
            the coarse/fine sweep-time ratio alpha of eq. (10).
  eq10      the PFASST speedup model of eq. (10) with GPU-measured inputs:
            alpha, beta, K_S (serial SDC sweeps per step to the 1e-10
            residual) and K_P (PFASST iterations to it, 16 slices, with and
            without the coarse predictor); beside it the measured time of the
            16 batched slices against 16 serial SDC steps.
  sdcnp127  127^3 SDC to the 1e-10 residual with sequential sweeps and with
            node-parallel sweeps (the M-1 solves of a sweep as one batch).
  mixed255  255^3, 4th order, 5 nodes, dt 0.02, 10 steps, 8 random sine
            modes: FP32 V(2,2) inside FP64 refinement to 1e-12 relative
            residual, against FP64 V(2,1) to 1e-12; SDC sweeps until the
            collocation residual is below --sdc-tol (1e-10).
  uneven64  64 independent instances with n drawn from {31, 63, 127}: one
            batched plan against one plan per instance run in turn.
  compact127 127^3, 5 nodes, nu 0.1, dt 0.05, 4 steps from u = s(x), sweeps
            until the collocation residual is <= 1e-10, V(2,1) to 1e-12: the
            compact fourth-order pair against the wide 13-point stencil, time
            per step and the error against the exact solution s(x) cos t;
            and two-level MLSDC with the compact fine level (coarse 63^3,
            2nd order, 3 nodes, tricubic transfer).
  micro511  single-kernel rates on the finest grid of the 511^3 hierarchy
            (FP64 and the FP32 inner cycles of mixed precision) and of a
            batch of two 255^3 grids, from HIP events on each launch.
  serving   Poisson stream of requests (n from {31..255} by default,
            weighted 8:4:2:1, nu, dt, steps random) through the serving core
            (mixed precision) and, replayed with the same arrival times, the
            plain path (one request at a time, FP64 V-cycles); both measured.
"""
from __future__ import annotations

import sys
import time

import numpy as np


def _log(msg):
    print(f"[workload] {msg}", file=sys.stderr, flush=True)


def _sync():
    import torch
    torch.cuda.synchronize()


def _dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64).ravel()).cuda()


def _timed(fn):
    _sync()
    t0 = time.perf_counter()
    fn()
    _sync()
    return time.perf_counter() - t0


# ----------------------------------------------------------------------------
# configuration 1: 15^3 SDC latency
# ----------------------------------------------------------------------------

def sdc15(args):
    from . import heatst as hs
    from . import inputs
    n = 15
    pb = hs.Problem(n=n, order=2, nnodes=3, nu=0.1, dt=0.125, nsteps=8, sweeps=4, tol=1e-12)
    plan = hs.Plan(pb)
    u0 = _dev(inputs.sine_product(n))
    plan.set_state(u0)
    plan.solve()
    per = []
    for _ in range(5):
        plan.set_state(u0)
        per.append(_timed(plan.solve) / 8)
    st, stats = plan.stats()
    return {"workload": "sdc15", "metric": "ms per SDC step", "value": float(np.median(per)) * 1e3,
            "unit": "ms", "steps": 8, "runs": len(per), "min_ms": min(per) * 1e3,
            "vcycles_per_solve": stats[0]["total_cycles"] / stats[0]["total_solves"]}


# ----------------------------------------------------------------------------
# configuration 2: two-level MLSDC at 127^3 / 63^3, alpha
# ----------------------------------------------------------------------------

def _sweep_alpha(hs, nf, nc, dt, reps=3, fas_interp=1):
    """alpha = time of one coarse sweep / time of one fine sweep (one lane);
    beta = time of restriction + interpolation / time of one fine sweep."""
    from . import inputs
    pb = hs.Problem(n=nf, order=4, nnodes=5, coarse=(nc, 2, 3), nu=0.1, dt=dt, nsteps=1, sweeps=1,
                    tol=1e-12, max_cycles=60, fas_interp=fas_interp)
    plan = hs.Plan(pb)
    plan.set_state(_dev(inputs.sine_product(nf)))
    tf, tc, tr = [], [], []
    for _ in range(reps):
        plan.begin_step()
        plan.sdc_sweep(0)
        tr.append(_timed(plan.fas_restrict))
        tf.append(_timed(lambda: plan.sdc_sweep(0)))
        tc.append(_timed(lambda: plan.sdc_sweep(1)))
        tr[-1] += _timed(plan.fas_interp)
    f, c, r = min(tf), min(tc), min(tr)
    return c / f, r / f, {"fine_sweep_ms": f * 1e3, "coarse_sweep_ms": c * 1e3, "transfer_ms": r * 1e3}


def _mlsdc127_run(hs, inputs, nf, nc, K, steps, interp):
    pb = hs.Problem(n=nf, order=4, nnodes=5, coarse=(nc, 2, 3), nu=0.1, dt=0.05, nsteps=steps, sweeps=K,
                    tol=1e-12, max_cycles=60, fas_interp=interp)
    plan = hs.Plan(pb)
    u0 = _dev(inputs.sine_product(nf))
    plan.set_state(u0)
    plan.step()
    plan.set_state(u0)
    el = _timed(plan.solve)
    st, stats = plan.stats()
    hs.check(st, "mlsdc127")
    u = plan.get_state().cpu().numpy().reshape(nf, nf, nf)
    del plan
    return el, stats, u


def mlsdc127(args):
    """Config 2: 20 steps of two-level MLSDC, 3 iterations each, with the
    transfer of the coarse correction chosen by --fas-interp; the other
    transfer's step time beside it."""
    from . import heatst as hs
    from . import inputs
    nf, nc, K, steps = 127, 63, 3, 20
    interp = getattr(args, "fas_interp", 3)
    el, stats, u = _mlsdc127_run(hs, inputs, nf, nc, K, steps, interp)
    other = 1 if interp == 3 else 3
    el_o, stats_o, u_o = _mlsdc127_run(hs, inputs, nf, nc, K, steps, other)
    ex = inputs.sine_product(nf) * np.cos(steps * 0.05)
    alpha, beta, t = _sweep_alpha(hs, nf, nc, 0.05, fas_interp=interp)
    return {"workload": "mlsdc127", "metric": "DOF-updates/s", "value": nf ** 3 * 4 * K * steps / el,
            "unit": "DOF-updates/s", "ms_per_step": el / steps * 1e3, "steps": steps,
            "vcycles": stats[0]["total_cycles"], "solves": stats[0]["total_solves"],
            "error_vs_exact": float(np.abs(u - ex).max() / np.abs(ex).max()),
            "fas_transfer": "tricubic" if interp == 3 else "trilinear",
            "other_transfer": {"fas_transfer": "tricubic" if other == 3 else "trilinear",
                               "ms_per_step": el_o / steps * 1e3, "vcycles": stats_o[0]["total_cycles"],
                               "error_vs_exact": float(np.abs(u_o - ex).max() / np.abs(ex).max())},
            "alpha_coarse_over_fine_sweep": alpha, **t}


# ----------------------------------------------------------------------------
# eq. (10): the PFASST speedup model with GPU-measured inputs
# ----------------------------------------------------------------------------

def eq10(args):
    """s(P) = K_S P / (P alpha + K_P (1 + alpha + beta)) (eq. (10)) for P = 16
    slices of the 127^3/63^3 problem at dt = 0.01 to the residual 1e-10, with
    alpha, beta, K_S and K_P measured here; and the one-GPU time ratio of 16
    serial SDC steps to the 16 batched PFASST slices (each to 1e-10)."""
    from . import heatst as hs
    from . import inputs
    nf, nc, P, dt, tol = 127, 63, 16, 0.01, 1e-10
    u0 = _dev(inputs.sine_product(nf))
    # serial single-level SDC on the fine problem: K_S
    sdc = hs.Plan(hs.Problem(n=nf, order=4, nnodes=5, nu=0.1, dt=dt, nsteps=P, sweeps=0, sdc_tol=tol,
                             max_sweeps=30, tol=1e-12, max_cycles=60))
    sdc.set_state(u0)
    sdc.step()
    sdc.set_state(u0)
    t_sdc = _timed(sdc.solve)
    st, stats = sdc.stats()
    hs.check(st, "eq10 serial SDC")
    K_S = stats[0]["total_sweeps"] / P
    u_sdc = sdc.get_state().cpu().numpy()
    del sdc
    rows = {}
    common = None
    # trilinear transfer of the coarse correction (the default reading), then tricubic
    for interp, name, preds in ((1, "trilinear", (0, 1)), (3, "tricubic", (1,))):
        # serial MLSDC to the same residual (the paper's P_T = 1 point)
        ml = hs.Plan(hs.Problem(n=nf, order=4, nnodes=5, coarse=(nc, 2, 3), nu=0.1, dt=dt, nsteps=P, sweeps=0,
                                sdc_tol=tol, max_sweeps=30, tol=1e-12, max_cycles=60, fas_interp=interp))
        ml.set_state(u0)
        ml.step()
        ml.set_state(u0)
        t_ml = _timed(ml.solve)
        st, mstats = ml.stats()
        hs.check(st, "eq10 serial MLSDC")
        del ml
        alpha, beta, t = _sweep_alpha(hs, nf, nc, dt, fas_interp=interp)
        part = {"alpha": alpha, "beta": beta, "serial_mlsdc_seconds": t_ml,
                "serial_mlsdc_iterations_per_step": mstats[0]["total_sweeps"] / P, **t}
        for pred in preds:
            pf = hs.Plan(hs.Problem(n=nf, order=4, nnodes=5, coarse=(nc, 2, 3), nu=0.1, dt=dt, nsteps=P, sweeps=0,
                                    sdc_tol=tol, max_sweeps=args.pfasst_max_iters, tol=1e-12, max_cycles=60,
                                    batch=P, nslices=P, pfasst_pred_sweeps=pred, fas_interp=interp))
            pf.set_state(u0)
            pf.pfasst_run()
            pf.set_state(u0)
            t_pf = _timed(pf.pfasst_run)
            st, pstats = pf.stats()
            hs.check(st, "eq10 PFASST", allow=(hs.HS_ENOCONV,))
            K_P = pstats[0]["total_sweeps"]
            u_pf = pf.get_state().cpu().numpy()
            del pf
            model = K_S * P / (P * alpha + K_P * (1 + alpha + beta))
            part[f"predictor_{pred}"] = {
                "K_P": K_P, "converged": st == hs.HS_OK, "last_residual": max(x["last_sdc_res"] for x in pstats),
                "model_speedup_P16": model, "pfasst_seconds": t_pf,
                "one_gpu_speedup_vs_serial_sdc": t_sdc / t_pf, "one_gpu_speedup_vs_serial_mlsdc": t_ml / t_pf,
                "rel_diff_vs_serial_sdc": float(np.abs(u_pf - u_sdc).max() / np.abs(u_sdc).max())}
        rows[name] = part
        if common is None:
            common = part
    return {"workload": "eq10", "P": P, "K_S": K_S, "serial_sdc_seconds": t_sdc,
            # the trilinear (default) figures at the top level, both in full below
            "alpha": common["alpha"], "beta": common["beta"],
            "predictor_0": common["predictor_0"], "predictor_1": common["predictor_1"],
            "fas_transfer": rows,
            "note": "model: eq. (10) for P processors, one slice each; one-GPU ratios: the 16 slices run as "
                    "one batch on a single GPU"}


# ----------------------------------------------------------------------------
# three levels against two
# ----------------------------------------------------------------------------

def levels3(args):
    """Two against three MLSDC levels on the 127^3 problem (fine 127^3, 4th
    order, 5 nodes; 63^3, 2nd order, 3 nodes; third level 31^3, 2nd order,
    with 2 or with 3 nodes), tricubic transfer, nu 0.1: serial MLSDC over
    16 steps of dt 0.01 to the 1e-10 residual, 16 PFASST slices in one batch
    with the coarse predictor to the same residual, and the 20-step MLSDC
    run of dt 0.05 with 3 iterations per step."""
    from . import heatst as hs
    from . import inputs
    nf, P, dt, tol = 127, 16, 0.01, 1e-10
    u0 = _dev(inputs.sine_product(nf))
    lv = {"levels_2": (2, dict(coarse=(63, 2, 3))),
          "levels_3_m2": (3, dict(coarse=(63, 2, 3), coarse2=(31, 2, 2))),
          "levels_3_m3": (3, dict(coarse=(63, 2, 3), coarse2=(31, 2, 3)))}
    out = {}
    for key, (L, kw) in lv.items():
        _log(f"levels3: {key}")
        base = dict(n=nf, order=4, nnodes=5, nu=0.1, tol=1e-12, max_cycles=60, fas_interp=3, **kw)
        ml = hs.Plan(hs.Problem(dt=dt, nsteps=P, sweeps=0, sdc_tol=tol, max_sweeps=30, **base))
        ml.set_state(u0)
        ml.step()
        ml.set_state(u0)
        t_ml = _timed(ml.solve)
        st, mstats = ml.stats()
        hs.check(st, f"levels3 serial MLSDC, {L} levels")
        u_ml = ml.get_state().cpu().numpy()
        del ml
        pf = hs.Plan(hs.Problem(dt=dt, nsteps=P, sweeps=0, sdc_tol=tol, max_sweeps=args.pfasst_max_iters,
                                batch=P, nslices=P, pfasst_pred_sweeps=1, **base))
        pf.set_state(u0)
        pf.pfasst_run()
        pf.set_state(u0)
        t_pf = _timed(pf.pfasst_run)
        st, pstats = pf.stats()
        hs.check(st, f"levels3 PFASST, {L} levels", allow=(hs.HS_ENOCONV,))
        u_pf = pf.get_state().cpu().numpy()
        del pf
        c2 = hs.Plan(hs.Problem(dt=0.05, nsteps=20, sweeps=3, **base))
        c2.set_state(u0)
        c2.step()
        c2.set_state(u0)
        t_c2 = _timed(c2.solve)
        st, cstats = c2.stats()
        hs.check(st, f"levels3 MLSDC 20 steps, {L} levels")
        u_c2 = c2.get_state().cpu().numpy().reshape(nf, nf, nf)
        del c2
        ex = inputs.sine_product(nf) * np.cos(20 * 0.05)
        out[key] = {
            "serial_mlsdc": {"seconds": t_ml, "iterations_per_step": mstats[0]["total_sweeps"] / P,
                             "level_cycles": mstats[0]["level_cycles"][:L]},
            "pfasst16": {"seconds": t_pf, "K_P": pstats[0]["total_sweeps"], "converged": st == hs.HS_OK,
                         "last_residual": max(x["last_sdc_res"] for x in pstats),
                         "rel_diff_vs_serial_mlsdc": float(np.abs(u_pf - u_ml).max() / np.abs(u_ml).max()),
                         "speedup_vs_serial_mlsdc": t_ml / t_pf},
            "mlsdc_dt0.05_3it": {"ms_per_step": t_c2 / 20 * 1e3,
                                 "error_vs_exact": float(np.abs(u_c2 - ex).max() / np.abs(ex).max())}}
    return {"workload": "levels3", "P": P, "dt": dt, "sdc_tol": tol, "fas_transfer": "tricubic", **out,
            "note": "PFASST slices run as one batch on one GPU; with three levels the serial pipeline runs on "
                    "the 31^3 grids (levels_3_m2: 2 nodes, levels_3_m3: 3 nodes)"}


# ----------------------------------------------------------------------------
# node-parallel against sequential SDC sweeps
# ----------------------------------------------------------------------------

def sdcnp127(args):
    """127^3, 4th order, 5 nodes, nu 0.1, dt 0.01, 8 steps, sweeps until the
    collocation residual is <= 1e-10, V(2,1) to 1e-12: the sequential IMEX
    sweep (4 solves one after the other) against the node-parallel sweep
    (the 4 solves as one batched solve); both reach the same collocation
    solution."""
    from . import heatst as hs
    from . import inputs
    n, steps = 127, 8
    u0 = _dev(inputs.random_smooth(n, 5))
    res, outs = {}, {}
    for name, npar in (("sequential", 0), ("node_parallel", 1)):
        plan = hs.Plan(hs.Problem(n=n, order=4, nnodes=5, nu=0.1, dt=0.01, nsteps=steps, sweeps=0, sdc_tol=1e-10,
                                  max_sweeps=60, tol=1e-12, max_cycles=60, sdc_node_parallel=npar))
        plan.set_state(u0)
        plan.step()
        plan.set_state(u0)
        el = _timed(plan.solve)
        st, stats = plan.stats()
        hs.check(st, f"sdcnp127 {name}")
        outs[name] = plan.get_state().cpu().numpy()
        res[name] = {"seconds": el, "ms_per_step": el / steps * 1e3, "sweeps_per_step": stats[0]["total_sweeps"] / steps,
                     "vcycles": stats[0]["total_cycles"], "solves": stats[0]["total_solves"]}
        del plan
    diff = float(np.abs(outs["node_parallel"] - outs["sequential"]).max() / np.abs(outs["sequential"]).max())
    return {"workload": "sdcnp127", "metric": "ms per step", "value": res["node_parallel"]["ms_per_step"],
            "unit": "ms", **res, "speedup_node_parallel": res["sequential"]["seconds"] / res["node_parallel"]["seconds"],
            "rel_diff": diff}


# ----------------------------------------------------------------------------
# compact fourth-order pair against the wide fourth-order stencil
# ----------------------------------------------------------------------------

def compact127(args):
    """Both schemes from the sine mode with the forcing that makes s(x) cos t
    the exact solution (c = 3): the compact pair's smaller error constant
    against its cost (one lane, a host check per cycle)."""
    import math
    from . import heatst as hs
    from . import inputs
    n, M, dt, steps = 127, 5, 0.05, 4
    s = inputs.sine_product(n)
    u0 = _dev(s)
    exact = s * math.cos(steps * dt)
    res = {}
    for name, order, coarse in (("compact", hs.HS_ORDER_COMPACT, None), ("wide", 4, None),
                                ("compact_mlsdc", hs.HS_ORDER_COMPACT, (63, 2, 3))):
        _log(f"compact127: {name}")
        plan = hs.Plan(hs.Problem(n=n, order=order, nnodes=M, nu=0.1, dt=dt, nsteps=steps, sweeps=0, sdc_tol=1e-10,
                                  max_sweeps=40, tol=1e-12, max_cycles=60, coarse=coarse, fas_interp=3))
        plan.set_state(u0)
        plan.solve()
        plan.set_state(u0)
        el = _timed(plan.solve)
        st, stats = plan.stats()
        hs.check(st, f"compact127 {name}")
        got = plan.get_state().cpu().numpy().reshape(n, n, n)
        res[name] = {"ms_per_step": el / steps * 1e3, "sweeps_per_step": stats[0]["total_sweeps"] / steps,
                     "vcycles_per_solve": stats[0]["total_cycles"] / stats[0]["total_solves"],
                     "max_error_vs_exact": float(np.abs(got - exact).max())}
        del plan
    return {"workload": "compact127", "metric": "ms per step (compact)", "value": res["compact"]["ms_per_step"],
            "unit": "ms", "n": n, "nodes": M, "dt": dt, "steps": steps, **res,
            "error_ratio_wide_over_compact": res["wide"]["max_error_vs_exact"] / res["compact"]["max_error_vs_exact"]}


# ----------------------------------------------------------------------------
# configuration 3: 255^3 mixed precision
# ----------------------------------------------------------------------------

def mixed255(args):
    from . import heatst as hs
    from . import inputs
    n, M, dt, nsteps = 255, 5, 0.02, 10
    seeds = [int(x) for x in str(args.seeds).split(",")]
    out = {"workload": "mixed255", "metric": "steps/s", "unit": "steps/s", "sdc_tol": args.sdc_tol,
           "seeds": {}}
    for seed in seeds:
        u0 = _dev(inputs.random_smooth(n, seed))
        res, outs = {}, {}
        # refinement to 1e-12 relative: the SDC threshold 1e-10 is then reachable and the
        # mixed result stays within 1e-10 of the FP64 one
        for name, prec in (("mixed", hs.HS_MIXED), ("fp64", hs.HS_FP64)):
            pb = hs.Problem(n=n, order=4, nnodes=M, nu=0.1, dt=dt, nsteps=nsteps, sweeps=0,
                            sdc_tol=args.sdc_tol, max_sweeps=40, precision=prec, tol=1e-12, max_cycles=80,
                            inner_nu1=2, inner_nu2=2)
            plan = hs.Plan(pb)
            plan.set_state(u0)
            plan.step()                      # warm-up step (state reset below)
            plan.set_state(u0)
            el = _timed(plan.solve)
            st, stats = plan.stats()
            s0 = stats[0]
            outs[name] = plan.get_state().cpu().numpy()
            res[name] = {"seconds": el, "ms_per_step": el / nsteps * 1e3, "status": st,
                         "sweeps": s0["total_sweeps"], "solves": s0["total_solves"],
                         "cycles_or_refinements": s0["total_cycles"],
                         "dof_updates_per_s": n ** 3 * (M - 1) * s0["total_sweeps"] / el}
            _log(f"mixed255 seed {seed} {name}: {el:.3f} s, sweeps {s0['total_sweeps']}")
            del plan
        diff = float(np.abs(outs["mixed"] - outs["fp64"]).max() / np.abs(outs["fp64"]).max())
        out["seeds"][str(seed)] = {"mixed": res["mixed"], "fp64": res["fp64"],
                                   "speedup_mixed_vs_fp64": res["fp64"]["seconds"] / res["mixed"]["seconds"],
                                   "rel_diff_mixed_vs_fp64": diff}
    first = out["seeds"][str(seeds[0])]
    out["value"] = nsteps / first["mixed"]["seconds"]
    out["speedup_mixed_vs_fp64"] = first["speedup_mixed_vs_fp64"]
    return out


# ----------------------------------------------------------------------------
# configuration 4 (second part): uneven batch of 64 instances
# ----------------------------------------------------------------------------

def uneven64(args):
    from . import heatst as hs
    from . import inputs
    ns = inputs.uneven_sizes(0, 64)
    dt, nsteps, sweeps = 0.01, 2, 4
    u0s = [inputs.random_smooth(n, 100 + i) for i, n in enumerate(ns)]
    flat = _dev(np.concatenate([u.ravel() for u in u0s]))
    pb = hs.Problem(n=31, order=2, nnodes=5, nu=0.1, dt=dt, nsteps=nsteps, sweeps=sweeps, tol=1e-12,
                    max_cycles=60, batch=len(ns), lane_n=ns)
    plan = hs.Plan(pb)
    plan.set_state(flat)
    plan.step()
    plan.set_state(flat)
    t_b = _timed(plan.solve)
    got = plan.get_state().cpu().numpy()
    del plan
    # one plan per instance, in turn
    plans = {}
    t_s = 0.0
    maxdiff = 0.0
    off = 0
    for i, n in enumerate(ns):
        if n not in plans:
            plans[n] = hs.Plan(hs.Problem(n=n, order=2, nnodes=5, nu=0.1, dt=dt, nsteps=nsteps, sweeps=sweeps,
                                          tol=1e-12, max_cycles=60))
            plans[n].set_state(_dev(u0s[i]))
            plans[n].step()            # warm-up
        p = plans[n]
        p.set_state(_dev(u0s[i]))
        t_s += _timed(p.solve)
        alone = p.get_state().cpu().numpy()
        maxdiff = max(maxdiff, float(np.abs(alone - got[off:off + n ** 3]).max()))
        off += n ** 3
    dof = sum(n ** 3 for n in ns) * 4 * sweeps * nsteps
    return {"workload": "uneven64", "metric": "DOF-updates/s", "value": dof / t_b, "unit": "DOF-updates/s",
            "batched_seconds": t_b, "sequential_seconds": t_s, "speedup_batched_vs_sequential": t_s / t_b,
            "max_abs_diff_batched_vs_alone": maxdiff, "sizes": {str(n): ns.count(n) for n in (31, 63, 127)}}


# ----------------------------------------------------------------------------
# kernel microbenchmark on the 511^3 hierarchy
# ----------------------------------------------------------------------------

# algorithmic bytes per grid point of each timed kernel (each input read once,
# each output written once)
_BYTES = {("pjac", 0): 25.0, ("resid_fw", 0): 17.0, ("sweep1", 0): 24.0, ("sweep2", 0): 24.0,
          ("pjac", 1): 12.5, ("resid_fw", 1): 8.5, ("sweep2", 1): 8.0}


def _kernel_rates(hs, plan, kinds, run, npts, prec, reps=3):
    out = {}
    for name, kind in kinds:
        plan.timer(kind | (hs.HS_TIMER_FP32 if prec else 0), 256)
        for _ in range(reps):
            run()
        launches, ms = plan.timer_read()
        plan.timer(0, 0)
        if launches == 0:
            continue
        us = ms / launches * 1e3
        gbs = _BYTES[(name, prec)] * npts / (us * 1e-6) / 1e9
        out[name] = {"us_per_launch": us, "launches": launches, "GBps_algorithmic": gbs,
                     "frac_of_8TBps": gbs / 8000.0, "bytes_per_point": _BYTES[(name, prec)]}
    return out


def micro511(args):
    """Finest-grid kernels in the solver's own launches: fixed-cycle V(2,1)
    solves (FP64) and refinement iterations with FP32 V(2,2) cycles (mixed),
    4th order, at 511^3 and on a batch of two 255^3 grids; the Jacobi sweep
    and the operator application alone through hs_smooth / hs_lap_apply, and
    the compact pair B_h - a A_h through hs_compact_apply."""
    import torch
    from . import heatst as hs
    from . import inputs
    res = {}
    kinds64 = [("sweep1", hs.HS_TIMER_SWEEP1), ("sweep2", hs.HS_TIMER_SWEEP2), ("resid_fw", hs.HS_TIMER_RESID_FW),
               ("pjac", hs.HS_TIMER_PJAC)]
    kinds32 = [("sweep2", hs.HS_TIMER_SWEEP2), ("resid_fw", hs.HS_TIMER_RESID_FW), ("pjac", hs.HS_TIMER_PJAC)]
    a = 0.1 * 0.05 * 0.17267316464601146
    for n, batch in ((511, 1), (255, 2)):
        N = n ** 3 * batch
        g = torch.Generator(device="cuda").manual_seed(0)
        b = torch.randn(N, dtype=torch.float64, device="cuda", generator=g)
        u = torch.zeros_like(b)
        for prec, kinds in ((0, kinds64), (1, kinds32)):
            plan = hs.Plan(hs.Problem(n=n, order=4, nnodes=2, nu=0.1, dt=0.05, fixed_cycles=2, batch=batch,
                                      precision=hs.HS_MIXED if prec else hs.HS_FP64, inner_nu1=2, inner_nu2=2))
            plan.mg_vcycle(u, b, a)      # tables and warm-up
            rates = _kernel_rates(hs, plan, kinds, lambda: plan.mg_vcycle(u, b, a), N, prec)
            res[f"{n}^3 x{batch} {'fp32' if prec else 'fp64'}"] = rates
            if prec == 0 and batch == 1:
                # the operator alone and plain Jacobi sweeps (one launch each)
                y = torch.empty_like(b)
                tmp = torch.empty_like(b)
                s = torch.cuda.current_stream()
                for name, fn, bpp in (("lap_apply", lambda: plan.lap_apply(u, 1.0, -a, out=y), 16.0),
                                      ("compact_apply", lambda: hs.compact_apply(b, y, n, batch, 1.0, -a), 16.0),
                                      ("jacobi", lambda: plan.smooth(u, b, tmp, a, 2), 24.0)):
                    fn()
                    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                    s.synchronize()
                    e0.record(s)
                    for _ in range(5):
                        fn()
                    e1.record(s)
                    e1.synchronize()
                    per = e0.elapsed_time(e1) / (5 * (2 if name == "jacobi" else 1)) * 1e-3
                    gbs = bpp * N / per / 1e9
                    rates[name] = {"us_per_launch": per * 1e6, "GBps_algorithmic": gbs, "frac_of_8TBps": gbs / 8000.0,
                                   "bytes_per_point": bpp}
                del y, tmp
            del plan
            torch.cuda.empty_cache()
        del b, u
        torch.cuda.empty_cache()
    return {"workload": "micro511", "order": 4, "kernels": res,
            "note": "per-launch times from HIP events that record each kernel's own start and end; "
                    "algorithmic bytes: every input read once, every output written once"}


# ----------------------------------------------------------------------------
# configuration 5: serving
# ----------------------------------------------------------------------------

def _plain_replay(hs, reqs, u0_of, keep):
    """The plain path under the same arrivals: one request at a time, in
    arrival order, FP64 V(2,1) to 1e-12, SDC to 1e-10; latency = completion -
    arrival on one clock."""
    plans = {}
    for r in reqs:
        if r.n not in plans:
            plans[r.n] = hs.Plan(hs.Problem(n=r.n, order=2, nnodes=5, nu=0.1, dt=0.01, nsteps=1, sweeps=0,
                                            sdc_tol=1e-10, max_sweeps=40, tol=1e-12, max_cycles=80))
    inputs_dev = [u0_of(r) for r in reqs]
    _sync()
    t_start = time.perf_counter()
    t_note = t_start
    lat, outs = [], {}
    for r, u0 in zip(reqs, inputs_dev):
        if time.perf_counter() - t_note >= 30.0:
            t_note = time.perf_counter()
            _log(f"plain replay: {len(lat)}/{len(reqs)} done after {t_note - t_start:.0f} s")
        now = time.perf_counter() - t_start
        if now < r.arrival:
            time.sleep(r.arrival - now)
        p = plans[r.n]
        p.set_lane(0, r.nu, r.dt, 0.0, r.nsteps)
        p.set_lane_state(0, u0)
        for _ in range(r.nsteps):
            p.step()
        _sync()
        lat.append(time.perf_counter() - t_start - r.arrival)
        if keep:
            outs[r.rid] = p.get_lane_state(0).cpu().numpy()
    wall = time.perf_counter() - t_start
    return np.array(lat), wall, outs


def serving(args):
    from . import heatst as hs
    from . import inputs
    from . import serving as sv
    sizes = tuple(n for n in (31, 63, 127, 255, 511) if n <= args.max_n)
    weights = (8, 4, 2, 1, 1)[:len(sizes)]
    R = args.requests

    def u0_of(r):
        return _dev(inputs.random_smooth(r.n, r.seed))

    # capacity of the plain path: the stream with every request at t = 0
    if getattr(args, "plain_capacity", 0.0) > 0:
        plain_capacity, lat0, wall0 = args.plain_capacity, None, None
    else:
        burst = inputs.serving_requests(1, R, 1e9, sizes=sizes, weights=weights)
        lat0, wall0, _ = _plain_replay(hs, burst, u0_of, False)
        plain_capacity = R / wall0
    _log(f"plain path: {plain_capacity:.3f} solves/s over {R} requests")
    budget = int(args.budget_gb * 1e9)
    srv = sv.Server.for_budget(budget, sizes, weights, precision=hs.HS_MIXED, tol=1e-12, sdc_tol=1e-10,
                               max_sweeps=40)
    rows = []
    for f in [float(x) for x in args.rates.split(",")]:
        rate = f * plain_capacity
        reqs = inputs.serving_requests(1, R, rate, sizes=sizes, weights=weights)
        res, tickets, infos = sv.replay(srv, reqs, u0_of, keep_results=True, progress=_log)
        served = {r.rid: srv.result(tk).cpu().numpy() for tk, r, _ in tickets}
        for tk, _, _ in tickets:
            srv.release(tk)
        bad = sum(1 for i in infos if i.status != 0)
        plat, pwall, pouts = _plain_replay(hs, reqs, u0_of, True)
        worst = max(float(np.abs(served[k] - pouts[k]).max() / np.abs(pouts[k]).max()) for k in pouts)
        rows.append({"rate_factor": f, "rate_per_s": rate, "solves_per_s": res.solves_per_s,
                     "p50_s": res.p50_s, "p99_s": res.p99_s, "failed": bad,
                     "plain_solves_per_s": R / pwall, "plain_p50_s": float(np.percentile(plat, 50)),
                     "plain_p99_s": float(np.percentile(plat, 99)),
                     "max_rel_diff_served_vs_plain": worst})
        _log(f"rate x{f}: served {res.solves_per_s:.3f} solves/s p50 {res.p50_s:.3f} p99 {res.p99_s:.3f}; "
             f"plain {R / pwall:.3f} solves/s p50 {np.percentile(plat, 50):.3f} p99 {np.percentile(plat, 99):.3f}; "
             f"max diff {worst:.2e}")
    res = None
    if not getattr(args, "no_saturated", False):
        reqs = inputs.serving_requests(1, R, 1e9, sizes=sizes, weights=weights)
        res, _, _ = sv.replay(srv, reqs, u0_of, progress=_log)
    srv.close()
    sat = None if res is None else {"p50_s": res.p50_s, "p99_s": res.p99_s, "wall_s": res.wall_s}
    value = res.solves_per_s if res is not None else max(r["solves_per_s"] for r in rows)
    return {"workload": "serving", "metric": "solves/s", "value": value, "unit": "solves/s",
            "plain_fp64_solves_per_s": plain_capacity, "speedup_vs_plain": value / plain_capacity,
            "saturated": sat,
            "plain_saturated": None if lat0 is None else
            {"p50_s": float(np.percentile(lat0, 50)), "p99_s": float(np.percentile(lat0, 99)), "wall_s": wall0},
            "rates": rows, "requests_per_rate": R, "sizes": list(sizes), "weights": list(weights),
            "budget_bytes": budget, "tolerances": {"sdc_residual": 1e-10, "inner_relative_residual": 1e-12}}
