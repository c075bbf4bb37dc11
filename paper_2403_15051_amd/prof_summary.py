"""Summarise rocprofv3 output as short markdown tables.

usage:
  python -m paper_2403_15051_amd.prof_summary trace <results.db> [title]
      per kernel and workgroup size (the stage kernel has one launch per velocity-set group):
      calls, total and average duration, share of GPU time, grid/workgroup sizes and the
      register/LDS footprint recorded by the profiler;
  python -m paper_2403_15051_amd.prof_summary pmc <counter_collection.csv> <kernel substring>
      per-dispatch average of each counter over the matching dispatches, and the per-stage
      total (sum over the workgroup-size groups of one stage).
"""
from __future__ import annotations

import collections
import csv
import sqlite3
import sys


def summarise_trace(db_path: str, title: str = "") -> str:
    db = sqlite3.connect(db_path)
    cur = db.cursor()
    total = list(cur.execute("select sum(duration) from kernels"))[0][0] or 1
    rows = list(cur.execute(
        "select name, workgroup_x, count(*), sum(duration), avg(duration), max(grid_x), max(grid_y), "
        "max(lds_size), max(vgpr_count), max(accum_vgpr_count), max(sgpr_count), max(scratch_size) "
        "from kernels group by name, workgroup_x order by sum(duration) desc"))
    out = []
    if title:
        out.append(f"### {title}\n")
    out.append("| kernel | wg | calls | total (ms) | avg (ms) | % GPU time | grid (x*y threads) | LDS B | VGPR | AGPR | "
               "SGPR | scratch |")
    out.append("|---|---|---|---|---|---|---|---|---|---|---|---|")
    for name, wg, calls, tot, avg, gx, gy, lds, vg, ag, sg, sc in rows:
        short = name.split("(")[0].replace("void ", "")
        out.append(f"| {short} | {wg} | {calls} | {tot / 1e6:.2f} | {avg / 1e6:.3f} | {100 * tot / total:.1f} | "
                   f"{gx}*{gy} | {lds} | {vg} | {ag} | {sg} | {sc} |")
    return "\n".join(out)


def summarise_pmc(csv_path: str, kernel: str) -> str:
    rows = list(csv.DictReader(open(csv_path)))
    per = collections.defaultdict(list)
    for r in rows:
        if kernel in r["Kernel_Name"]:
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
    return "\n".join(out)


if __name__ == "__main__":
    if len(sys.argv) < 3 or sys.argv[1] not in ("trace", "pmc"):
        raise SystemExit(__doc__)
    if sys.argv[1] == "trace":
        print(summarise_trace(sys.argv[2], sys.argv[3] if len(sys.argv) > 3 else ""))
    else:
        print(summarise_pmc(sys.argv[2], sys.argv[3]))
