"""Autotuner of the plane-marching launch shapes (run on the GPU).

For every (grid size n, Laplacian order, precision, batch) of interest it
times fixed-cycle multigrid solves on a plan whose finest grids are `batch`
grids of n^3, over candidate z-chunk lengths of the sweep / prolongation
kernels (zb) and of the residual + restriction kernel (zb_rfw), and keeps
the fastest.  Sizes run from small to large, so a hierarchy's coarser grids
already use their tuned shapes when its finest grid is tuned.  The result
is a JSON file that hs_tune_load reads (the binding loads
paper_1307_7867_amd/tune_cache.json when it exists):

    {"device": ..., "entries": [{"n", "order", "precision", "batch", "zb", "zb_rfw",
                                 "us_per_cycle", "us_per_cycle_builtin"}, ...]}

Shapes only move work between blocks; every shape gives bitwise the same
results (tests/test_gpu_tuning.py).

    python -m paper_1307_7867_amd.tune [--out FILE] [--quick] [--missing]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
DEFAULT_OUT = os.path.join(HERE, "tune_cache.json")

# (n, order, precision, batch): the launch shapes of the benchmark's workloads
# (PFASST 16 x 127^3/63^3 in one batch or in slice groups of 8, 4 or 2, the MLSDC
# and SDC runs, the mixed-precision 255^3 run, the uneven batch and the
# serving classes)
SHAPES = [
    (31, 4, 0, 1), (63, 4, 0, 1), (127, 4, 0, 1),
    (31, 4, 0, 16), (63, 4, 0, 16), (127, 4, 0, 16),
    (31, 4, 0, 8), (63, 4, 0, 8), (127, 4, 0, 8),
    (31, 4, 0, 4), (63, 4, 0, 4), (127, 4, 0, 4),
    (31, 4, 0, 2), (63, 4, 0, 2), (127, 4, 0, 2),
    (31, 2, 0, 1), (63, 2, 0, 1), (31, 2, 0, 16), (63, 2, 0, 16),
    (31, 2, 0, 19), (63, 2, 0, 22), (127, 2, 0, 23),
    (255, 4, 0, 1), (63, 4, 1, 1), (127, 4, 1, 1), (255, 4, 1, 1),
]
ZB = (1, 2, 4, 8, 16, 32)
ZB_RFW = (2, 4, 8, 16, 32)


def _time_cycles(hs, torch, n, order, prec, batch, cycles=3, reps=3):
    """Seconds per V-cycle of a fixed-cycle solve (FP64: V(2,1); mixed: one
    refinement iteration around an FP32 V(2,2) cycle)."""
    pb = hs.Problem(n=n, order=order, nnodes=2, nu=0.1, dt=0.05, fixed_cycles=cycles, batch=batch,
                    precision=hs.HS_MIXED if prec else hs.HS_FP64, inner_nu1=2, inner_nu2=2)
    plan = hs.Plan(pb)
    N = n ** 3 * batch
    g = torch.Generator(device="cuda").manual_seed(n)
    b = torch.randn(N, dtype=torch.float64, device="cuda", generator=g)
    u = torch.zeros_like(b)
    a = 0.1 * 0.01 * 0.17267316464601146
    plan.mg_vcycle(u, b, a)
    best = float("inf")
    for _ in range(reps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        plan.mg_vcycle(u, b, a)
        torch.cuda.synchronize()
        best = min(best, (time.perf_counter() - t0) / cycles)
    del plan, b, u
    return best


def tune(shapes=SHAPES, quick=False, log=print, keep=()):
    """Tune `shapes`; entries in `keep` (earlier results) are loaded first and
    not tuned again."""
    import torch
    from . import heatst as hs
    hs.tune_clear()
    for e in keep:
        hs.tune_set(e["n"], e["order"], e["precision"], e["batch"], e["zb"], e["zb_rfw"])
    done = {(e["n"], e["order"], e["precision"], e["batch"]) for e in keep}
    shapes = [sh for sh in shapes if tuple(sh) not in done]
    entries = list(keep)
    for n, order, prec, batch in sorted(shapes, key=lambda s: (s[0], s[3])):
        builtin = hs.tune_lookup(n, order, prec, batch)
        t_builtin = _time_cycles(hs, torch, n, order, prec, batch)
        zbs = [z for z in ZB if z <= max(1, (n + 1) // 2)]
        rfws = [z for z in ZB_RFW if z <= max(2, (n + 1) // 2)]
        if quick:
            zbs = [z for z in zbs if z in (2, 8, 16)] or zbs[:1]
            rfws = [z for z in rfws if z in (2, 8, 16)] or rfws[:1]
        best = (t_builtin, builtin[0], builtin[1])
        for zb in zbs:                                # z chunk of the sweeps, rfw at its current best
            hs.tune_set(n, order, prec, batch, zb, best[2])
            t = _time_cycles(hs, torch, n, order, prec, batch)
            if t < best[0]:
                best = (t, zb, best[2])
        for zr in rfws:                               # then the residual-restriction chunk
            hs.tune_set(n, order, prec, batch, best[1], zr)
            t = _time_cycles(hs, torch, n, order, prec, batch)
            if t < best[0]:
                best = (t, best[1], zr)
        hs.tune_set(n, order, prec, batch, best[1], best[2])
        entries.append({"n": n, "order": order, "precision": prec, "batch": batch, "zb": best[1],
                        "zb_rfw": best[2], "us_per_cycle": best[0] * 1e6,
                        "us_per_cycle_builtin": t_builtin * 1e6, "builtin": list(builtin)})
        log(f"[tune] n={n} order={order} prec={prec} batch={batch}: zb={best[1]} zb_rfw={best[2]} "
            f"{best[0] * 1e6:.1f} us/cycle (built-in {builtin}: {t_builtin * 1e6:.1f})")
        torch.cuda.empty_cache()
    return entries


def main():
    ap = argparse.ArgumentParser(description="tune the plane-marching launch shapes on this GPU")
    ap.add_argument("--out", default=DEFAULT_OUT)
    ap.add_argument("--quick", action="store_true", help="fewer candidates")
    ap.add_argument("--missing", action="store_true",
                    help="keep the entries already in --out and tune only the shapes it lacks")
    args = ap.parse_args()
    import torch
    torch.cuda.set_device(0)
    name = torch.cuda.get_device_properties(0).name
    keep = []
    if args.missing and os.path.exists(args.out):
        keep = json.load(open(args.out)).get("entries", [])
    entries = tune(quick=args.quick, log=lambda m: print(m, file=sys.stderr, flush=True), keep=keep)
    with open(args.out, "w") as f:
        json.dump({"device": name, "arch": "gfx950", "entries": entries}, f, indent=1)
    print(json.dumps({"entries": len(entries), "out": args.out}))


if __name__ == "__main__":
    main()
