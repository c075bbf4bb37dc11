"""Summarise a rocprofv3 kernel-trace database (rocpd SQLite) as a short markdown table.

usage: python -m paper_2403_15051_amd.prof_summary <results.db> [title]
Prints, per kernel: calls, total and average duration, share of GPU time, grid/workgroup
sizes and the register/LDS footprint recorded by the profiler.
"""
from __future__ import annotations

import sqlite3
import sys


def summarise(db_path: str, title: str = "") -> str:
    db = sqlite3.connect(db_path)
    cur = db.cursor()
    rows = list(cur.execute("select name, total_calls, total_duration, average, percentage from top_kernels"))
    info = {}
    for r in cur.execute("select name, grid_x, grid_y, workgroup_x, lds_size, vgpr_count, accum_vgpr_count, "
                         "sgpr_count, scratch_size from kernels group by name"):
        info[r[0]] = r[1:]
    out = []
    if title:
        out.append(f"### {title}\n")
    out.append("| kernel | calls | total (ms) | avg (ms) | % GPU time | grid (x*y threads) | wg | LDS B | VGPR | AGPR | "
               "SGPR | scratch |")
    out.append("|---|---|---|---|---|---|---|---|---|---|---|---|")
    for name, calls, tot, avg, pct in rows:
        g = info.get(name, (None,) * 8)
        short = name.split("(")[0]
        out.append(f"| {short} | {calls} | {tot / 1e3:.1f} | {avg / 1e3:.2f} | {pct:.1f} | {g[0]}*{g[1]} | {g[2]} | "
                   f"{g[3]} | {g[4]} | {g[5]} | {g[6]} | {g[7]} |")
    return "\n".join(out)


if __name__ == "__main__":
    print(summarise(sys.argv[1], sys.argv[2] if len(sys.argv) > 2 else ""))
