#!/usr/bin/env python3
"""Benchmark of the space-time heat solver's hot path on one MI355X.

Headline workload (the largest FP64 configuration that runs on one GPU):
PFASST with 16 concurrent time slices on one GPU, two-level MLSDC per
slice -- fine level 127^3 with the wide 4th-order stencil and 5
Gauss-Lobatto nodes, coarse level 63^3 with the 7-point stencil and 3
nodes -- nu = 0.1, dt = 0.01, a serial coarse predictor (one coarse sweep
per slice) and then 4 PFASST iterations per block of 16 steps, every
implicit substep solved by V(2,1) multigrid cycles (weighted Jacobi
6/7, full weighting, trilinear, exact 3^3 solve) to a relative residual of
1e-12; initial value u0 = sin(pi x) sin(pi y) sin(pi z) and the consistent
manufactured forcing (c = 3).  Inputs are synthetic, generated on the host
and copied to HBM before timing.  The coarse corrections go back to the
fine level by tricubic interpolation (--fas-interp 1: trilinear; both are
pinned readings of a transfer the paper leaves to its references).  The
slices run in 4 groups of 4: the fine
sweeps of one group (one batched launch per kernel over its 4 slices)
overlap the coarse pipeline of the group before it, which a second host
thread issues on a second stream (--groups; the results are bit for bit
those of the one-batch order).

A step is one PFASST block (16 time slices, 4 iterations).  --steps K
blocks are timed back to back (16 K time steps); --warmup W blocks run first
and the state is then reset.

value = space-time DOF-updates/s = 127^3 * (5 - 1) substeps * 4 iterations
        * 16 slices * K / elapsed.

roofline: the dominant kernel of the batched fine sweeps, k_pjac<double, 4>
(prolongation + first post-smoothing sweep) on one group's 127^3 finest grids,
timed live inside the timed run with HIP events that record each launch's
own start and end on the stream it runs on (hs_plan_timer); algorithmic
bytes 25 per grid point of every lane the launch updates (read u, b and the
coarse correction at 1/8 density, write u'), summed from the lanes' own
fine-level cycle counts.

cpu_baseline: the CPU oracle (plain serial C, one core) on one MLSDC
iteration of the first slice of the same workload.

serial_mlsdc_equal_work: the same 16 K steps by one-lane MLSDC with 4
iterations per step, the speedup of the PFASST run over it.

one_batch: the same run without slice groups (all 16 slices' fine sweeps in
one batch, then the coarse pipeline), with k_pjac timed on 16 x 127^3 finest
grids, a working set far beyond the Infinity Cache.

extra: the other configurations as records of their own -- 15^3 SDC
latency, the 127^3/63^3 MLSDC run with the coarse/fine sweep-time ratio,
the eq. (10) PFASST model, node-parallel against sequential SDC sweeps,
the 255^3 mixed-precision run, the uneven batch of 64 instances, the 511^3
kernel microbenchmark and a short serving stream -- unless --no-extras.
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
NF, NC, MF, MC, ITERS, SLICES, DT = 127, 63, 5, 3, 4, 16, 0.01
PJAC_BYTES = 25          # per fine grid point: read u, b (16), coarse e at 1/8 density (1), write u' (8)
# the kernels and the structures they read (the traffic record is void once either changes)
KERNEL_SRC = [os.path.join(ROOT, "paper_1307_7867_amd", "csrc", f) for f in ("hs_kernels.hip", "hs_internal.h")]
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "pjac_fp64_order4_pfasst16.traffic.json")


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


PRED = 1                 # coarse sweeps per slice of the serial coarse predictor
GROUPS = 4               # slice groups: a group's fine sweeps overlap the previous group's coarse pipeline
FAS_INTERP = 3           # spatial transfer of the coarse correction (1 trilinear, 3 tricubic)


def problem(hs, nblocks, groups=GROUPS, fas_interp=FAS_INTERP, **kw):
    return hs.Problem(n=NF, order=4, nnodes=MF, coarse=(NC, 2, MC), nu=0.1, dt=DT, t0=0.0, forcing_c=3.0,
                      nsteps=SLICES * nblocks, sweeps=ITERS, nu1=2, nu2=1, omega=6.0 / 7.0, n_coarsest=3,
                      tol=1e-12, max_cycles=60, batch=SLICES, nslices=SLICES, pfasst_pred_sweeps=PRED,
                      pfasst_groups=groups, fas_interp=fas_interp, **kw)


def kernel_hash():
    h = hashlib.sha256()
    for path in KERNEL_SRC:
        with open(path, "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def cpu_baseline():
    """One MLSDC iteration of slice 0 of the first block, as the GPU runs it
    (fine sweep of 4 multigrid solves to 1e-12 from the spread initial value,
    restriction + tau, coarse sweep, interpolation), by the serial C oracle."""
    import numpy as np
    import oracle
    from paper_1307_7867_amd import inputs
    pb = oracle.problem([(NF, 4, MF), (NC, 2, MC)], nu=0.1, dt=DT, nsteps=1, sweeps=1, forcing_c=3.0,
                        mg=oracle.mg_params(tol=1e-12, max_cycles=60))
    u0 = inputs.sine_product(NF)
    Uf, FIf = oracle.spread(pb.lev[0], pb.nu, u0)
    Uc = np.zeros((MC, NC, NC, NC))
    FIc, Ut, tau = np.zeros_like(Uc), np.zeros_like(Uc), np.zeros_like(Uc)
    t0 = time.perf_counter()
    s, st = oracle.mlsdc_iter(pb, 0.0, Uf, FIf, Uc, FIc, Ut, tau)
    el = time.perf_counter() - t0
    cps = st.total_cycles / max(1, st.total_solves)
    return {"value": NF ** 3 * (MF - 1) / el, "unit": "DOF-updates/s", "cores": 1, "kind": "oracle",
            "sample": f"1 MLSDC iteration of slice 0 of the first block of the same workload (fine sweep of "
                      f"{st.total_solves} multigrid solves to 1e-12 from the spread initial value, "
                      f"{cps:.1f} V-cycles per solve; FAS restriction, coarse sweep, interpolation), "
                      f"serial C, {el:.1f} s",
            "vcycles_per_solve": cps, "seconds": el}


def headline(args, torch, hs, inputs):
    u0 = torch.from_numpy(inputs.sine_product(NF).ravel()).cuda()
    warm = hs.Plan(problem(hs, 1, args.groups, args.fas_interp))
    for _ in range(args.warmup):
        warm.set_state(u0)
        warm.pfasst_run()
    torch.cuda.synchronize()
    del warm
    plan = hs.Plan(problem(hs, args.steps, args.groups, args.fas_interp))
    plan.set_state(u0)
    plan.timer(hs.HS_TIMER_PJAC, 8192)
    torch.cuda.synchronize()
    log(f"timing {args.steps} PFASST block(s) of {SLICES} slices x {ITERS} iterations, {NF}^3/{NC}^3")
    t0 = time.perf_counter()
    plan.pfasst_run()
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    launches, kms = plan.timer_read()
    st, stats = plan.stats()
    hs.check(st, "bench PFASST run")
    u = plan.get_state().cpu().numpy().reshape(NF, NF, NF)
    T = args.steps * SLICES * DT
    import numpy as np
    ex = inputs.sine_product(NF) * math.cos(T)
    err = float(np.abs(u - ex).max() / np.abs(ex).max())
    fine_lane_cycles = sum(s["level_cycles"][0] for s in stats)
    fine_solves = SLICES * args.steps * ITERS * (MF - 1)
    dof_updates = NF ** 3 * (MF - 1) * ITERS * SLICES * args.steps
    value = dof_updates / elapsed
    pjac_bytes = PJAC_BYTES * NF ** 3 * fine_lane_cycles
    achieved = pjac_bytes / (kms * 1e-3) / 1e9
    traffic = None
    if os.path.exists(TRAFFIC_FILE):
        rec = json.load(open(TRAFFIC_FILE))
        if rec.get("kernel_src_sha") == kernel_hash():
            traffic = rec.get("bytes_per_launch")
    log(f"{elapsed:.3f} s, {value:.3e} DOF-updates/s, k_pjac {launches} launches {kms / launches * 1e3:.1f} us, "
        f"{achieved:.0f} GB/s")
    del plan
    gb = SLICES // args.groups if args.groups >= 2 else SLICES   # lanes per fine launch
    shapes = {f"{n}^3 order {o} x{b}": list(hs.tune_lookup(n, o, 0, b))
              for n, o, b in ((127, 4, gb), (63, 4, gb), (31, 4, gb), (63, 2, 1), (31, 2, 1))}
    builtin_s = None
    if not args.no_builtin_compare:
        builtin_s = builtin_shapes_run(args, torch, hs, u0)
    out = _headline_record(args, elapsed, value, achieved, traffic, launches, kms, pjac_bytes, fine_lane_cycles,
                           fine_solves, err, stats, shapes, builtin_s)
    if not args.no_serial_compare:
        out["serial_mlsdc_equal_work"] = serial_mlsdc_run(args, torch, hs, inputs, u0, elapsed)
    if args.groups >= 2 and not args.no_one_batch:
        out["one_batch"] = one_batch_run(args, torch, hs, u0, elapsed)
    return out


def one_batch_run(args, torch, hs, u0, grouped_s):
    """The same blocks with all 16 slices' fine sweeps in one batch (no slice
    groups): its k_pjac launches cover 16 x 127^3 finest grids, a working set
    (16 lanes x u, t, b = 786 MB) far beyond the Infinity Cache."""
    plan = hs.Plan(problem(hs, args.steps, 0, args.fas_interp))
    plan.set_state(u0)
    plan.timer(hs.HS_TIMER_PJAC, 8192)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    plan.pfasst_run()
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    launches, kms = plan.timer_read()
    st, stats = plan.stats()
    hs.check(st, "bench one-batch PFASST run")
    del plan
    byts = PJAC_BYTES * NF ** 3 * sum(x["level_cycles"][0] for x in stats)
    gbs = byts / (kms * 1e-3) / 1e9
    log(f"one batch: {el:.3f} s; k_pjac {launches} launches {kms / launches * 1e3:.1f} us, {gbs:.0f} GB/s")
    return {"seconds": el, "groups_speedup": el / grouped_s, "pjac_launches": launches,
            "pjac_us_per_launch": kms / launches * 1e3, "pjac_achieved_GBps": gbs, "pjac_frac": gbs / PEAK_HBM_GBS}


def serial_mlsdc_run(args, torch, hs, inputs, u0, pfasst_s):
    """The same 16 K time steps by one-lane MLSDC, step after step, with the
    PFASST run's 4 iterations per step (equal fine work, no predictor)."""
    import numpy as np
    pb = hs.Problem(n=NF, order=4, nnodes=MF, coarse=(NC, 2, MC), nu=0.1, dt=DT, t0=0.0, forcing_c=3.0,
                    nsteps=SLICES * args.steps, sweeps=ITERS, nu1=2, nu2=1, omega=6.0 / 7.0, n_coarsest=3,
                    tol=1e-12, max_cycles=60, fas_interp=args.fas_interp)
    plan = hs.Plan(pb)
    plan.set_state(u0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    plan.solve()
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    st, _ = plan.stats()
    hs.check(st, "bench serial MLSDC")
    u = plan.get_state().cpu().numpy().reshape(NF, NF, NF)
    ex = inputs.sine_product(NF) * math.cos(args.steps * SLICES * DT)
    del plan
    log(f"serial MLSDC, same steps and iterations: {el:.3f} s (PFASST {pfasst_s / el:.3f} of it)")
    return {"seconds": el, "steps": SLICES * args.steps, "iterations_per_step": ITERS,
            "pfasst_speedup": el / pfasst_s, "error_vs_exact": float(np.abs(u - ex).max() / np.abs(ex).max())}


def builtin_shapes_run(args, torch, hs, u0):
    """The same run with the built-in launch shapes: what the autotuner's table gains."""
    hs.tune_clear()
    base = hs.Plan(problem(hs, args.steps, args.groups, args.fas_interp))
    base.set_state(u0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    base.pfasst_run()
    torch.cuda.synchronize()
    builtin_s = time.perf_counter() - t0
    del base
    if os.path.exists(hs.TUNE_CACHE):
        hs.tune_load(hs.TUNE_CACHE)
    log(f"built-in launch shapes: {builtin_s:.3f} s")
    return builtin_s


def _headline_record(args, elapsed, value, achieved, traffic, launches, kms, pjac_bytes, fine_lane_cycles,
                     fine_solves, err, stats, shapes, builtin_s):
    return {
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
        "config": {"workload": "PFASST, 16 time slices batched on one GPU x 5 Lobatto nodes, two-level MLSDC + "
                               "FAS per slice, FP64: fine 127^3 4th-order, coarse 63^3 2nd-order 3 nodes, nu=0.1, "
                               "dt=0.01, coarse predictor + 4 PFASST iterations per block of 16 steps, V(2,1) "
                               "Jacobi 6/7 to 3^3, rel. residual 1e-12; slices in groups whose batched fine "
                               "sweeps overlap the coarse pipeline; tricubic transfer of the coarse correction",
                   "fine_n": NF, "coarse_n": NC, "slices": SLICES, "dt": DT, "iterations": ITERS,
                   "blocks": args.steps, "mg_tol": 1e-12, "predictor_coarse_sweeps": PRED,
                   "slice_groups": args.groups,
                   "fas_transfer": "tricubic" if args.fas_interp == 3 else "trilinear"},
        "roofline": {"bound": "hbm",
                     "kernel": f"k_pjac<double, 4> on the finest 127^3 grids of one slice group "
                               f"({SLICES // max(1, args.groups)} lanes per launch)",
                     "achieved": achieved, "peak": PEAK_HBM_GBS, "unit": "GB/s", "frac": achieved / PEAK_HBM_GBS,
                     "traffic": traffic, "launches": launches, "us_per_launch": kms / launches * 1e3,
                     "algorithmic_bytes_per_launch": pjac_bytes / launches,
                     "algorithmic_bytes_per_point": PJAC_BYTES, "lane_cycles": fine_lane_cycles},
        "error_vs_exact": err,
        "tuning": {"shapes_zb_zb_rfw": shapes, "seconds_builtin_shapes": builtin_s,
                   "gain_over_builtin": builtin_s / elapsed if builtin_s else None},
        "fine_vcycles_per_solve": fine_lane_cycles / fine_solves,
        "coarse_vcycles": sum(s["level_cycles"][1] for s in stats),
    }


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=4, help="PFASST blocks (16 time steps each) timed")
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true", help="only the headline PFASST measurement")
    ap.add_argument("--groups", type=int, default=GROUPS,
                    help="PFASST slice groups whose fine sweeps overlap the coarse pipeline (0: one batch)")
    ap.add_argument("--fas-interp", type=int, default=FAS_INTERP, choices=(1, 3),
                    help="spatial transfer of the coarse correction: 1 trilinear, 3 tricubic")
    ap.add_argument("--no-serial-compare", action="store_true",
                    help="skip the serial MLSDC run of the same steps")
    ap.add_argument("--no-one-batch", action="store_true",
                    help="skip the run without slice groups (k_pjac on 16 x 127^3)")
    ap.add_argument("--no-builtin-compare", action="store_true",
                    help="skip the second headline run with the built-in launch shapes")
    ap.add_argument("--plain-capacity", type=float, default=0.0,
                    help="serving: the plain path's solves/s (skips measuring it)")
    ap.add_argument("--no-saturated", action="store_true",
                    help="serving: skip the closing all-at-once stream")
    ap.add_argument("--workload", default="pfasst16",
                    choices=["pfasst16", "sdc15", "mlsdc127", "mixed255", "uneven64", "serving", "micro511",
                             "eq10", "levels3", "sdcnp127", "compact127"],
                    help="pfasst16 (default): the headline line with every other workload as an extra; "
                         "any other name runs that workload alone")
    ap.add_argument("--seeds", default="0", help="mixed255: comma-separated seeds")
    ap.add_argument("--sdc-tol", type=float, default=1e-10)
    ap.add_argument("--pfasst-max-iters", type=int, default=40,
                    help="eq10: cap on PFASST iterations to the 1e-10 residual")
    ap.add_argument("--requests", type=int, default=16)
    ap.add_argument("--rates", default="1.0")
    ap.add_argument("--max-n", type=int, default=255)
    ap.add_argument("--budget-gb", type=float, default=200.0)
    ap.add_argument("--calibration-copy", action="store_true",
                    help="first run a plain 512 MiB device copy (reference for byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: this build runs on one GPU; --gpus {args.gpus} is not supported "
              "(the path shards by lanes or PFASST slices across GPUs only in design).",
              file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1307_7867_amd import heatst as hs
    from paper_1307_7867_amd import inputs
    from paper_1307_7867_amd import workloads

    torch.cuda.set_device(0)
    if args.calibration_copy:
        src = torch.ones(64 * 2**20, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    if args.workload != "pfasst16":
        out = getattr(workloads, args.workload)(args)
        print(json.dumps(out), flush=True)
        return
    out = headline(args, torch, hs, inputs)
    if not args.no_extras:
        extra = {}
        for name in ("sdc15", "mlsdc127", "eq10", "levels3", "sdcnp127", "compact127", "mixed255", "uneven64",
                     "micro511", "serving"):
            log(f"extra: {name}")
            t0 = time.perf_counter()
            extra[name] = getattr(workloads, name)(args)
            extra[name]["wall_s"] = time.perf_counter() - t0
            log(f"extra {name}: {extra[name]['wall_s']:.1f} s")
            torch.cuda.empty_cache()
        out["extra"] = extra
    if not args.no_cpu_baseline:
        log("CPU oracle baseline")
        out["cpu_baseline"] = cpu_baseline()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
