"""Summarise rocprofv3 output as short markdown tables.

usage:
  python -m paper_2403_15051_amd.prof_summary trace <results.db> [title] [--last N]
      per kernel and workgroup size (the stage kernel has one launch per velocity-set group):
      calls, total and average duration, share of GPU time, grid/workgroup sizes and the
      register/LDS footprint recorded by the profiler;
  python -m paper_2403_15051_amd.prof_summary pmc <counter_collection.csv> <kernel substring> [--last N]
      per-dispatch average of each counter over the matching dispatches, and the per-stage
      total (sum over the workgroup-size groups of one stage).
  --last N keeps only the last N dispatches of every kernel (by name), e.g. the 3 K launches of
  the node and projection kernels in bench.py's final timed pass of K steps (earlier dispatches
  include the tile autotuner's trial launches);
  --match S --last-total N (trace) keeps only kernels whose name contains S and, of those, the last
  N dispatches in all: the stage kernel has several template instances (by tiles per wave), so the
  3 K G stage launches of the final pass over G launch groups span several names;
  --last-total N --per M (pmc) keeps the last N matching dispatches in all and adds each counter's
  sum over them divided by M (e.g. M = 3 K stages).
"""
from __future__ import annotations

import collections
import csv
import sqlite3
import sys


def summarise_trace(db_path: str, title: str = "", last: int = 0, match: str = "", last_total: int = 0) -> str:
    db = sqlite3.connect(db_path)
    cur = db.cursor()
    recs = list(cur.execute(
        "select name, workgroup_x, start, duration, grid_x, grid_y, lds_size, vgpr_count, accum_vgpr_count, "
        "sgpr_count, scratch_size from kernels order by start"))
    if match:
        recs = [r for r in recs if match in r[0]]
    if last_total:
        recs = recs[-last_total:]
    if last:
        by_name = collections.defaultdict(list)
        for r in recs:
            by_name[r[0]].append(r)
        recs = sorted((r for rs in by_name.values() for r in rs[-last:]), key=lambda r: r[2])
    groups = collections.defaultdict(list)
    for r in recs:
        groups[(r[0], r[1])].append(r)
    rows = []
    for (name, wg), rs in groups.items():
        durs = [r[3] for r in rs]
        rows.append((name, wg, len(rs), sum(durs), sum(durs) / len(rs), max(r[4] for r in rs), max(r[5] for r in rs),
                     max(r[6] for r in rs), max(r[7] for r in rs), max(r[8] for r in rs), max(r[9] for r in rs),
                     max(r[10] for r in rs)))
    rows.sort(key=lambda r: -r[3])
    total = sum(r[3] for r in rows) or 1
    out = []
    if title:
        out.append(f"### {title}\n")
    out.append("| kernel | wg | calls | total (ms) | avg (ms) | % GPU time | grid (x*y threads) | LDS B | VGPR | AGPR | "
               "SGPR | scratch |")
    out.append("|---|---|---|---|---|---|---|---|---|---|---|---|")
    for name, wg, calls, tot, avg, gx, gy, lds, vg, ag, sg, sc in rows:
        short = name.replace("(anonymous namespace)::", "").replace("void ", "").split("(")[0]
        out.append(f"| {short} | {wg} | {calls} | {tot / 1e6:.2f} | {avg / 1e6:.3f} | {100 * tot / total:.1f} | "
                   f"{gx}*{gy} | {lds} | {vg} | {ag} | {sg} | {sc} |")
    return "\n".join(out)


def summarise_pmc(csv_path: str, kernel: str, last: int = 0, last_total: int = 0, divide: int = 0) -> str:
    rows = [r for r in csv.DictReader(open(csv_path)) if kernel in r["Kernel_Name"]]
    rows.sort(key=lambda r: int(r.get("Dispatch_Id", 0)))
    if last_total:
        keep = set(sorted({int(r.get("Dispatch_Id", 0)) for r in rows})[-last_total:])
        rows = [r for r in rows if int(r.get("Dispatch_Id", 0)) in keep]
    if last:
        by = collections.defaultdict(list)
        for r in rows:
            by[(r["Kernel_Name"], r["Counter_Name"])].append(r)
        rows = [r for rs in by.values() for r in rs[-last:]]
    per = collections.defaultdict(list)
    for r in rows:
        wg = r.get("Workgroup_Size", r.get("Workgroup_Size_X", ""))
        per[(r["Counter_Name"], wg)].append(float(r["Counter_Value"]))
    out = ["| counter | wg | dispatches | average per dispatch |", "|---|---|---|---|"]
    totals = collections.defaultdict(float)
    for (cname, wg), v in sorted(per.items()):
        avg = sum(v) / len(v)
        totals[cname] += avg
        out.append(f"| {cname} | {wg} | {len(v)} | {avg:.6g} |")
    for cname, tot in sorted(totals.items()):
        out.append(f"| {cname} | all groups | | {tot:.6g} |")
    if divide:
        sums = collections.defaultdict(float)
        for r in rows:
            sums[r["Counter_Name"]] += float(r["Counter_Value"])
        for cname, tot in sorted(sums.items()):
            out.append(f"| {cname} | sum / {divide} | | {tot / divide:.6g} |")
    return "\n".join(out)


if __name__ == "__main__":
    args = sys.argv[1:]

    def option(flag: str, conv=int, default=0):
        global args
        if flag not in args:
            return default
        i = args.index(flag)
        v = conv(args[i + 1])
        args = args[:i] + args[i + 2:]
        return v

    last = option("--last")
    last_total = option("--last-total")
    per = option("--per")
    match = option("--match", str, "")
    if len(args) < 2 or args[0] not in ("trace", "pmc"):
        raise SystemExit(__doc__)
    if args[0] == "trace":
        print(summarise_trace(args[1], args[2] if len(args) > 2 else "", last, match, last_total))
    else:
        print(summarise_pmc(args[1], args[2], last, last_total, per))
