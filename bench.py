#!/usr/bin/env python3
"""Benchmark of the space-time heat solver's hot path on one MI355X.

Workload (two-level MLSDC with FAS, FP64): fine level 127^3 with the wide
4th-order stencil and 5 Gauss-Lobatto nodes, coarse level 63^3 with the
7-point stencil and 3 nodes, nu = 0.1, dt = 0.05, 3 MLSDC iterations per
step, every implicit substep solved by V(2,1) multigrid cycles (weighted
Jacobi 6/7, full weighting, trilinear, exact 3^3 solve) to a relative
residual of 1e-12; initial value u0 = sin(pi x) sin(pi y) sin(pi z) and
the consistent manufactured forcing (c = 3).  Inputs are synthetic and
generated on the host, then copied to HBM before timing.

A step is one MLSDC time step.  --steps K time steps are timed (K = 20 is
the run to T = 1); --warmup W steps run first and the state is then reset.

value = space-time DOF-updates/s = 127^3 * (5 - 1) substeps * 3 iterations
        * K / elapsed.

roofline: the dominant kernel, the finest-grid weighted-Jacobi sweep
(k_sweep<double, 4, 0, 1, 0, 0> on 127^3), timed with HIP events on its stream
(one launch per sweep, the solver's launch configuration); algorithmic
bytes 24 per grid point (read u, b; write u').

cpu_baseline: the CPU oracle (plain serial C) on one MLSDC iteration of the
first step of the same workload.
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

PEAK_HBM_GBS = 8000.0
NF, NC, MF, MC, ITERS = 127, 63, 5, 3, 3
KERNEL_SRC = os.path.join(ROOT, "paper_1307_7867_amd", "csrc", "hs_kernels.hip")
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "jacobi_fp64_order4_127.traffic.json")


def problem(hs, fused_sweeps=1, cycle_graphs=0):
    return hs.Problem(n=NF, order=4, nnodes=MF, coarse=(NC, 2, MC), nu=0.1, dt=0.05, t0=0.0,
                      forcing_c=3.0, nsteps=20, sweeps=ITERS, nu1=2, nu2=1, omega=6.0 / 7.0,
                      n_coarsest=3, tol=1e-12, max_cycles=60, fused_sweeps=fused_sweeps,
                      cycle_graphs=cycle_graphs)


def kernel_hash():
    with open(KERNEL_SRC, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def measure_jacobi(torch, hs, plan, n, sweeps_a=10, sweeps_b=60):
    """Average duration of one finest-grid Jacobi launch, from HIP events on
    the stream the launches go to (difference of two launch counts removes
    the fixed cost of the call).  About 2 ms of device work (fills of a
    1 GiB buffer) is queued ahead of the first event, so the host has queued
    every timed launch before the device reaches them: the figure is the
    device's back-to-back time, not the host's launch rate."""
    N = n ** 3
    g = torch.Generator(device="cuda").manual_seed(0)
    u = torch.randn(N, dtype=torch.float64, device="cuda", generator=g)
    b = torch.randn(N, dtype=torch.float64, device="cuda", generator=g)
    tmp = torch.empty_like(u)
    pad = torch.empty(2 ** 27, dtype=torch.float64, device="cuda")
    a = 0.1 * 0.05 * 0.17267316464601146
    s = torch.cuda.current_stream()
    plan.smooth(u, b, tmp, a, 2)   # table upload and warm-up
    times = []
    for k in (sweeps_a, sweeps_b):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        s.synchronize()
        for _ in range(10):
            pad.fill_(1.0)
        e0.record(s)
        plan.smooth(u, b, tmp, a, k)
        e1.record(s)
        e1.synchronize()
        times.append(e0.elapsed_time(e1))
    return (times[1] - times[0]) / (sweeps_b - sweeps_a) * 1e-3   # seconds per launch


def cpu_baseline(sample_iters=1):
    import numpy as np
    import oracle
    from paper_1307_7867_amd import inputs
    pb = oracle.problem([(NF, 4, MF), (NC, 2, MC)], nu=0.1, dt=0.05, nsteps=1, sweeps=1,
                        forcing_c=3.0, mg=oracle.mg_params(tol=1e-12, max_cycles=60))
    u0 = inputs.sine_product(NF)
    Uf, FIf = oracle.spread(pb.lev[0], pb.nu, u0)
    Uc = np.zeros((MC, NC, NC, NC))
    FIc, Ut, tau = np.zeros_like(Uc), np.zeros_like(Uc), np.zeros_like(Uc)
    t0 = time.perf_counter()
    for _ in range(sample_iters):
        oracle.mlsdc_iter(pb, 0.0, Uf, FIf, Uc, FIc, Ut, tau)
    el = time.perf_counter() - t0
    return {"value": NF ** 3 * (MF - 1) * sample_iters / el, "unit": "DOF-updates/s", "cores": 1,
            "kind": "oracle",
            "sample": f"{sample_iters} MLSDC iteration(s) of the first time step of the same workload "
                      f"(fine sweep with 4 multigrid solves to 1e-12, FAS restriction, coarse sweep, "
                      f"interpolation), serial C, {el:.1f} s"}


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-hbm511", action="store_true", help="skip the 511^3 Jacobi measurement")
    ap.add_argument("--workload", default="mlsdc127",
                    choices=["mlsdc127", "mixed255", "pfasst16", "uneven64", "serving"],
                    help="mlsdc127 (default): the headline two-level MLSDC run; the others are the "
                         "mixed-precision, PFASST-slice, uneven-batch and serving workloads")
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--sdc-tol", type=float, default=1e-10)
    ap.add_argument("--requests", type=int, default=64)
    ap.add_argument("--rates", default="0.5,1.0,1.5")
    ap.add_argument("--max-n", type=int, default=511)
    ap.add_argument("--budget-gb", type=float, default=200.0)
    ap.add_argument("--fused-sweeps", type=int, default=1, choices=[1, 2],
                    help="2: run the finest grid's first two pre-smoothing sweeps as one pass")
    ap.add_argument("--cycle-graphs", type=int, default=0, choices=[0, 1],
                    help="1: replay the predicted cycles of each solve from HIP graphs (measured "
                         "slower than launching every kernel from the host)")
    ap.add_argument("--calibration-copy", action="store_true",
                    help="first run a plain 512 MiB device copy (reference for byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: this build runs on one GPU; --gpus {args.gpus} is not supported "
              "(the path shards by lanes or PFASST slices across GPUs only in design).",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    from paper_1307_7867_amd import heatst as hs
    from paper_1307_7867_amd import inputs

    torch.cuda.set_device(0)
    if args.calibration_copy:
        src = torch.ones(64 * 2**20, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    if args.workload != "mlsdc127":
        from paper_1307_7867_amd import workloads
        out = getattr(workloads, args.workload)(args)
        print(json.dumps(out), flush=True)
        return
    pb = problem(hs, args.fused_sweeps, args.cycle_graphs)
    plan = hs.Plan(pb)
    u0 = torch.from_numpy(inputs.sine_product(NF).ravel()).cuda()

    plan.set_state(u0)
    for _ in range(args.warmup):
        plan.step()
    torch.cuda.synchronize()
    plan.set_state(u0)            # timed run starts at t = 0
    torch.cuda.synchronize()
    print(f"[bench] timing {args.steps} MLSDC steps of {NF}^3/{NC}^3", file=sys.stderr, flush=True)
    t0 = time.perf_counter()
    for _ in range(args.steps):
        plan.step()
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    st, stats = plan.stats()
    hs.check(st, "bench solve")
    u = plan.get_state().cpu().numpy().reshape(NF, NF, NF)
    T = args.steps * pb.dt
    ex = inputs.sine_product(NF) * math.cos(T)
    err = float(np.abs(u - ex).max() / np.abs(ex).max())
    dof_updates = NF ** 3 * (MF - 1) * ITERS * args.steps
    value = dof_updates / elapsed
    s0 = stats[0]
    print(f"[bench] {elapsed:.3f} s, {value:.3e} DOF-updates/s, V-cycles {s0['total_cycles']} over "
          f"{s0['total_solves']} solves", file=sys.stderr, flush=True)

    # dominant kernel: finest-grid Jacobi sweep
    jac_s = measure_jacobi(torch, hs, plan, NF)
    jac_bytes = 24 * NF ** 3
    achieved = jac_bytes / jac_s / 1e9
    traffic = None
    if os.path.exists(TRAFFIC_FILE):
        rec = json.load(open(TRAFFIC_FILE))
        if rec.get("kernel_src_sha") == kernel_hash():
            traffic = rec.get("bytes_per_launch")
    extra = {}
    if not args.no_hbm511:
        big = hs.Plan(hs.Problem(n=511, order=4, nnodes=2, nu=0.1, dt=0.05, sweeps=1, fixed_cycles=1))
        js = measure_jacobi(torch, hs, big, 511, 4, 24)
        extra["jacobi_511_fp64_order4"] = {"us_per_launch": js * 1e6,
                                           "GBps_algorithmic": 24 * 511 ** 3 / js / 1e9,
                                           "frac_of_8TBps": 24 * 511 ** 3 / js / 1e9 / PEAK_HBM_GBS}
        del big
        torch.cuda.empty_cache()

    out = {
        "metric": "DOF-updates/s",
        "value": value,
        "unit": "DOF-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": elapsed / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "two-level MLSDC + FAS, FP64: fine 127^3 4th-order 5 Lobatto nodes, "
                               "coarse 63^3 2nd-order 3 nodes, nu=0.1, dt=0.05, 3 iterations/step, "
                               "V(2,1) Jacobi 6/7 to 3^3, rel. residual 1e-12",
                   "fine_n": NF, "coarse_n": NC, "dt": pb.dt, "iterations_per_step": ITERS,
                   "mg_tol": pb.tol, "fused_sweeps": pb.fused_sweeps, "cycle_graphs": pb.cycle_graphs},
        "roofline": {"bound": "hbm", "kernel": "k_sweep<double, 4, 0, 1, 0, 0> (finest-grid weighted Jacobi) on 127^3",
                     "achieved": achieved, "peak": PEAK_HBM_GBS, "unit": "GB/s",
                     "frac": achieved / PEAK_HBM_GBS, "traffic": traffic,
                     "us_per_launch": jac_s * 1e6, "algorithmic_bytes_per_launch": jac_bytes},
        "error_vs_exact": err,
        "vcycles": s0["total_cycles"],
        "solves": s0["total_solves"],
        "extra": extra,
    }
    if not args.no_cpu_baseline:
        print("[bench] CPU oracle baseline", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
