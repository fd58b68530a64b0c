"""Benchmark workloads besides the headline MLSDC run (bench.py --workload).

Each function takes the parsed bench.py arguments and returns one JSON-able
record.  Inputs are synthetic (paper_1307_7867_amd.inputs), generated on the
host and copied to HBM before any timed region.

  mixed255  255^3, 4th order, 5 nodes, dt 0.02, 10 steps, 8 random sine
            modes: FP32 V(2,2) inside FP64 refinement to 1e-12 relative
            residual, against FP64 V(2,1) to 1e-12; SDC sweeps until the
            collocation residual is below --sdc-tol (1e-10).
  pfasst16  16 PFASST time slices x 5 nodes, 127^3 (4th order) / 63^3 (2nd
            order), dt 0.01, 4 iterations, every phase one batched launch
            sequence over the slices; against 16 serial MLSDC steps; plus the
            coarse-to-fine sweep time ratio alpha of the paper's speedup model.
  uneven64  64 independent instances with n drawn from {31, 63, 127}: one
            batched plan against one plan per instance run in turn.
  serving   Poisson stream of requests (n from {31..511} weighted 8:4:2:1:1,
            nu, dt, steps random) through the serving core (mixed precision)
            against the plain path (one request at a time, FP64 V-cycles).
"""
from __future__ import annotations

import math
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


def mixed255(args):
    from . import heatst as hs
    from . import inputs
    n, M, dt, nsteps = 255, 5, 0.02, 10
    u0 = _dev(inputs.random_smooth(n, args.seed))
    res = {}
    outs = {}
    # refinement to 1e-12 relative: the SDC threshold 1e-10 is then reachable and the
    # mixed result stays within 1e-10 of the FP64 one
    for name, prec, tol, inner in (("mixed", hs.HS_MIXED, 1e-12, (2, 2)), ("fp64", hs.HS_FP64, 1e-12, (2, 2))):
        pb = hs.Problem(n=n, order=4, nnodes=M, nu=0.1, dt=dt, nsteps=nsteps, sweeps=0,
                        sdc_tol=args.sdc_tol, max_sweeps=40, precision=prec, tol=tol, max_cycles=80,
                        inner_nu1=inner[0], inner_nu2=inner[1])
        plan = hs.Plan(pb)
        plan.set_state(u0)
        plan.step()                      # warm-up step (state reset below)
        _sync()
        plan.set_state(u0)
        _sync()
        t0 = time.perf_counter()
        plan.solve()
        _sync()
        el = time.perf_counter() - t0
        st, stats = plan.stats()
        s0 = stats[0]
        outs[name] = plan.get_state().cpu().numpy()
        res[name] = {"seconds": el, "ms_per_step": el / nsteps * 1e3, "status": st,
                     "sweeps": s0["total_sweeps"], "solves": s0["total_solves"],
                     "cycles_or_refinements": s0["total_cycles"],
                     "dof_updates_per_s": n ** 3 * (M - 1) * s0["total_sweeps"] / el,
                     "steps_per_s": nsteps / el}
        _log(f"{name}: {el:.3f} s, sweeps {s0['total_sweeps']}, inner iterations {s0['total_cycles']}")
        del plan
    diff = float(np.abs(outs["mixed"] - outs["fp64"]).max() / np.abs(outs["fp64"]).max())
    return {"workload": "mixed255", "metric": "steps/s", "value": res["mixed"]["steps_per_s"],
            "unit": "steps/s", "seed": args.seed, "sdc_tol": args.sdc_tol, "mixed": res["mixed"],
            "fp64": res["fp64"], "speedup_mixed_vs_fp64": res["fp64"]["seconds"] / res["mixed"]["seconds"],
            "rel_diff_mixed_vs_fp64": diff}


def _sweep_alpha(hs, nf, nc):
    """alpha = time of one coarse sweep / time of one fine sweep (single lane)."""
    pb = hs.Problem(n=nf, order=4, nnodes=5, coarse=(nc, 2, 3), nu=0.1, dt=0.01, nsteps=1, sweeps=1,
                    tol=1e-12, max_cycles=60)
    plan = hs.Plan(pb)
    from . import inputs
    plan.set_state(_dev(inputs.sine_product(nf)))
    times = {}
    for level in (0, 1, 0, 1):
        plan.begin_step()
        plan.sdc_sweep(0)
        plan.fas_restrict()
        _sync()
        t0 = time.perf_counter()
        plan.sdc_sweep(level)
        _sync()
        times[level] = time.perf_counter() - t0
    return times[1] / times[0], times


def pfasst16(args):
    from . import heatst as hs
    from . import inputs
    P, nf, nc, dt, K = 16, 127, 63, 0.01, 4
    u0 = _dev(inputs.sine_product(nf))
    pb = hs.Problem(n=nf, order=4, nnodes=5, coarse=(nc, 2, 3), nu=0.1, dt=dt, nsteps=P, sweeps=K,
                    tol=1e-12, max_cycles=60, batch=P, nslices=P)
    plan = hs.Plan(pb)
    plan.set_state(u0)
    plan.pfasst_run()
    _sync()
    plan.set_state(u0)
    _sync()
    t0 = time.perf_counter()
    plan.pfasst_run()
    _sync()
    t_pf = time.perf_counter() - t0
    upf = plan.get_state().cpu().numpy()
    del plan
    # serial MLSDC over the same 16 steps with the same iteration count
    ser = hs.Plan(hs.Problem(n=nf, order=4, nnodes=5, coarse=(nc, 2, 3), nu=0.1, dt=dt, nsteps=P,
                             sweeps=K, tol=1e-12, max_cycles=60))
    ser.set_state(u0)
    ser.step()
    _sync()
    ser.set_state(u0)
    _sync()
    t0 = time.perf_counter()
    ser.solve()
    _sync()
    t_ser = time.perf_counter() - t0
    user = ser.get_state().cpu().numpy()
    del ser
    alpha, times = _sweep_alpha(hs, nf, nc)
    dof = nf ** 3 * 4 * K * P
    return {"workload": "pfasst16", "metric": "DOF-updates/s", "value": dof / t_pf, "unit": "DOF-updates/s",
            "pfasst_seconds": t_pf, "serial_mlsdc_seconds": t_ser, "speedup_vs_serial": t_ser / t_pf,
            "rel_diff_pfasst_vs_serial": float(np.abs(upf - user).max() / np.abs(user).max()),
            "alpha_coarse_over_fine_sweep": alpha,
            "fine_sweep_ms": times[0] * 1e3, "coarse_sweep_ms": times[1] * 1e3}


def uneven64(args):
    from . import heatst as hs
    from . import inputs
    ns = inputs.uneven_sizes(args.seed, 64)
    dt, nsteps, sweeps = 0.01, 2, 4
    u0s = [inputs.random_smooth(n, 100 + i) for i, n in enumerate(ns)]
    flat = _dev(np.concatenate([u.ravel() for u in u0s]))
    pb = hs.Problem(n=31, order=2, nnodes=5, nu=0.1, dt=dt, nsteps=nsteps, sweeps=sweeps, tol=1e-12,
                    max_cycles=60, batch=len(ns), lane_n=ns)
    plan = hs.Plan(pb)
    plan.set_state(flat)
    plan.step()
    _sync()
    plan.set_state(flat)
    _sync()
    t0 = time.perf_counter()
    plan.solve()
    _sync()
    t_b = time.perf_counter() - t0
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
        u = _dev(u0s[i])
        p.set_state(u)
        _sync()
        t0 = time.perf_counter()
        p.solve()
        _sync()
        t_s += time.perf_counter() - t0
        alone = p.get_state().cpu().numpy()
        maxdiff = max(maxdiff, float(np.abs(alone - got[off:off + n ** 3]).max()))
        off += n ** 3
    dof = sum(n ** 3 for n in ns) * 4 * sweeps * nsteps
    return {"workload": "uneven64", "metric": "DOF-updates/s", "value": dof / t_b, "unit": "DOF-updates/s",
            "batched_seconds": t_b, "sequential_seconds": t_s, "speedup_batched_vs_sequential": t_s / t_b,
            "max_abs_diff_batched_vs_alone": maxdiff, "sizes": {str(n): ns.count(n) for n in (31, 63, 127)}}


def serving(args):
    from . import heatst as hs
    from . import inputs
    from . import serving as sv
    sizes = tuple(n for n in (31, 63, 127, 255, 511) if n <= args.max_n)
    weights = (8, 4, 2, 1, 1)[:len(sizes)]
    R = args.requests

    def u0_of(r):
        return _dev(inputs.random_smooth(r.n, r.seed))

    # plain path: one request at a time, FP64 V(2,1) cycles to 1e-12, SDC to 1e-10
    sample = inputs.serving_requests(args.seed + 1, R, 1.0, sizes=sizes, weights=weights)
    plans = {}
    service = []
    for r in sample:
        if r.n not in plans:
            plans[r.n] = hs.Plan(hs.Problem(n=r.n, order=2, nnodes=5, nu=0.1, dt=0.01, nsteps=1, sweeps=0,
                                            sdc_tol=1e-10, max_sweeps=40, tol=1e-12, max_cycles=80))
        p = plans[r.n]
        p.set_lane(0, r.nu, r.dt, 0.0, r.nsteps)
        p.set_lane_state(0, u0_of(r))
        _sync()
        t0 = time.perf_counter()
        for _ in range(r.nsteps):
            p.step()
        _sync()
        service.append(time.perf_counter() - t0)
        _log(f"plain request {len(service)}/{len(sample)}: n={r.n} steps={r.nsteps} {service[-1]:.3f} s")
    plain_capacity = len(sample) / sum(service)
    del plans
    _log(f"plain path: {plain_capacity:.3f} solves/s over {len(sample)} requests")

    def fifo_latencies(arrivals, svc):
        t, lat = 0.0, []
        for a, s in zip(arrivals, svc):
            t = max(t, a) + s
            lat.append(t - a)
        return np.array(lat)

    budget = int(args.budget_gb * 1e9)
    slots = sv.slots_for_budget(budget, sizes, weights, precision=hs.HS_MIXED, tol=1e-12)
    _log(f"slots {slots}")
    srv = sv.Server(slots, precision=hs.HS_MIXED, tol=1e-12, sdc_tol=1e-10, max_sweeps=40, budget_bytes=budget)
    rows = []
    for f in [float(x) for x in args.rates.split(",")]:
        rate = f * plain_capacity
        reqs = inputs.serving_requests(args.seed + 1, R, rate, sizes=sizes, weights=weights)
        res, tickets, infos = sv.replay(srv, reqs, u0_of)
        bad = sum(1 for i in infos if i.status != 0)
        plain_lat = fifo_latencies([r.arrival for r in reqs], service)
        rows.append({"rate_factor": f, "rate_per_s": rate, "solves_per_s": res.solves_per_s,
                     "p50_s": res.p50_s, "p99_s": res.p99_s, "failed": bad,
                     "plain_p50_s": float(np.percentile(plain_lat, 50)),
                     "plain_p99_s": float(np.percentile(plain_lat, 99)),
                     "plain_solves_per_s": len(reqs) / float(max(r.arrival + l for r, l in zip(reqs, plain_lat)))})
        _log(f"rate x{f}: {res.solves_per_s:.3f} solves/s p50 {res.p50_s:.3f} s p99 {res.p99_s:.3f} s")
    # saturation: every request at t = 0
    reqs = inputs.serving_requests(args.seed + 1, R, 1e9, sizes=sizes, weights=weights)
    res, _, infos = sv.replay(srv, reqs, u0_of)
    srv.close()
    return {"workload": "serving", "metric": "solves/s", "value": res.solves_per_s, "unit": "solves/s",
            "plain_fp64_solves_per_s": plain_capacity,
            "speedup_vs_plain": res.solves_per_s / plain_capacity,
            "saturated": {"p50_s": res.p50_s, "p99_s": res.p99_s, "wall_s": res.wall_s},
            "rates": rows, "slots": {str(k): v for k, v in slots.items()}, "requests_per_rate": R,
            "sizes": list(sizes), "weights": list(weights),
            "tolerances": {"sdc_residual": 1e-10, "inner_relative_residual": 1e-12}}
