"""Summaries of rocprofv3 output for the measurement records under profiles/.

    python -m paper_1307_7867_amd.prof_summary stats <kernel_trace.csv> [--top K]
            [--split REGEX:BLOCKS:PERIOD]
        per-kernel totals over the whole trace and, per launch size (blocks),
        the calls / mean / median duration of each kernel (markdown).
    python -m paper_1307_7867_amd.prof_summary traffic <fetch_counter.csv> <write_counter.csv>
            --kernel REGEX --blocks N [--period P --phase Q] --bytes-per-launch B --src FILE [FILE ...] --out JSON
        FETCH_SIZE / WRITE_SIZE per dispatch (KiB, mean over the kernel's
        launches of N blocks), scaled by what the same counters read for the device copies of
        bench.py --calibration-copy (512 MiB each), as bytes per launch.

Launches of one kernel with the same block count on two grid levels (a
V-cycle launches the kernel on each level in turn) are told apart by their
order: --split / --period take them in dispatch order and number them
0..PERIOD-1 cyclically; --phase keeps one of those phases.
"""
from __future__ import annotations

import argparse
import csv
import hashlib
import json
import re
import statistics
import sys
from collections import defaultdict


def short(name: str) -> str:
    name = name.replace("(anonymous namespace)::", "").replace("void ", "")
    depth, out = 0, []
    for ch in name:                      # drop the argument list, keep template arguments
        if ch == "(" and depth == 0:
            break
        depth += ch == "<"
        depth -= ch == ">"
        out.append(ch)
    return "".join(out).strip()


def blocks(row) -> int:
    g = int(row.get("Grid_Size_X") or row.get("Grid_Size") or 0)
    w = int(row.get("Workgroup_Size_X") or row.get("Workgroup_Size") or 1)
    return g // max(1, w)


def stats(trace, top=30, split=None):
    rows = sorted(csv.DictReader(open(trace)), key=lambda r: int(r["Dispatch_Id"]))
    tot = defaultdict(lambda: [0, 0.0])
    per = defaultdict(list)
    sp_re, sp_blk, sp_per = None, 0, 1
    if split:
        sp_re, b, pr = split.rsplit(":", 2)
        sp_blk, sp_per = int(b), int(pr)
    seen = 0
    for r in rows:
        d = (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3
        k = short(r["Kernel_Name"])
        tot[k][0] += 1
        tot[k][1] += d
        b = blocks(r)
        if sp_re and b == sp_blk and re.search(sp_re, r["Kernel_Name"]):
            k = f"{k} [phase {seen % sp_per}]"
            seen += 1
        per[(k, b)].append(d)
    all_us = sum(v[1] for v in tot.values())
    out = ["| kernel | calls | avg us | total ms | share |", "|---|---:|---:|---:|---:|"]
    for k, (c, t) in sorted(tot.items(), key=lambda kv: -kv[1][1])[:top]:
        out.append(f"| `{k}` | {c} | {t / c:.2f} | {t / 1e3:.2f} | {100 * t / all_us:.1f}% |")
    out += ["", "| kernel | blocks | calls | mean us | median us | total ms |", "|---|---:|---:|---:|---:|---:|"]
    for (k, b), ds in sorted(per.items(), key=lambda kv: -sum(kv[1]))[:top]:
        out.append(f"| `{k}` | {b} | {len(ds)} | {statistics.mean(ds):.2f} | {statistics.median(ds):.2f} | "
                   f"{sum(ds) / 1e3:.2f} |")
    return "\n".join(out)


def _counter_rows(path):
    rows = list(csv.DictReader(open(path)))
    out = []
    for r in rows:
        out.append((int(r.get("Dispatch_Id", 0)), r["Kernel_Name"], blocks(r), r["Counter_Name"],
                    float(r["Counter_Value"])))
    return out


def _per_dispatch(rows, regex, nblk=None, period=1, phase=0):
    acc = defaultdict(float)
    for disp, name, b, cname, val in rows:
        if re.search(regex, name) and (nblk is None or b == nblk):
            acc[disp] += val
    vals = [acc[k] for k in sorted(acc)]
    return vals[phase::period]


def traffic(fetch_csv, write_csv, kernel, nblk, bytes_per_launch, src, out, period=1, phase=0):
    copy_bytes = 512 * 1024 * 1024
    f_rows, w_rows = _counter_rows(fetch_csv), _counter_rows(write_csv)
    f_cal = _per_dispatch(f_rows, "copyBuffer|copy")
    w_cal = _per_dispatch(w_rows, "copyBuffer|copy")
    f_cal = [v for v in f_cal if v > 0.25 * copy_bytes / 1024][:3]
    w_cal = [v for v in w_cal if v > 0.25 * copy_bytes / 1024][:3]
    f_fac = copy_bytes / 1024 / statistics.median(f_cal)
    w_fac = copy_bytes / 1024 / statistics.median(w_cal)
    # mean over every dispatch: launches differ in how many lanes are still active
    fd, wd = _per_dispatch(f_rows, kernel, nblk, period, phase), _per_dispatch(w_rows, kernel, nblk, period, phase)
    fk, wk = statistics.mean(fd), statistics.mean(wd)
    # the other phases' means, to show the levels apart
    others = {q: statistics.mean(_per_dispatch(f_rows, kernel, nblk, period, q)) for q in range(period) if q != phase}
    h = hashlib.sha256()
    for path in src:            # the hash bench.py compares: the sources in this order
        h.update(open(path, "rb").read())
    sha = h.hexdigest()[:16]
    rec = {"kernel": kernel, "blocks": nblk, "period": period, "phase": phase,
           "fetch_kib_other_phases": others, "kernel_src_sha": sha, "dispatches": [len(fd), len(wd)],
           "fetch_kib": fk, "write_kib": wk,
           "fetch_factor": f_fac, "write_factor": w_fac, "calibration_fetch_kib": f_cal,
           "calibration_write_kib": w_cal,
           "bytes_per_launch": fk * 1024 * f_fac + wk * 1024 * w_fac,
           "algorithmic_bytes_per_launch": bytes_per_launch}
    rec["ratio_to_algorithmic"] = rec["bytes_per_launch"] / bytes_per_launch
    with open(out, "w") as f:
        json.dump(rec, f, indent=1)
    return rec


def main():
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    s = sub.add_parser("stats")
    s.add_argument("trace")
    s.add_argument("--top", type=int, default=30)
    s.add_argument("--split", default=None)
    t = sub.add_parser("traffic")
    t.add_argument("fetch")
    t.add_argument("write")
    t.add_argument("--kernel", required=True)
    t.add_argument("--blocks", type=int, required=True)
    t.add_argument("--bytes-per-launch", type=float, required=True)
    t.add_argument("--period", type=int, default=1)
    t.add_argument("--phase", type=int, default=0)
    t.add_argument("--src", required=True, nargs="+")
    t.add_argument("--out", required=True)
    a = ap.parse_args()
    if a.cmd == "stats":
        print(stats(a.trace, a.top, a.split))
    else:
        print(json.dumps(traffic(a.fetch, a.write, a.kernel, a.blocks, a.bytes_per_launch, a.src, a.out,
                                 a.period, a.phase), indent=1))


if __name__ == "__main__":
    sys.exit(main())
