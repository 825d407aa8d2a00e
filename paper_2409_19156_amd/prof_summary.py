"""Summarise a rocprofv3 kernel trace as a text table.

    python -m paper_2409_19156_amd.prof_summary <run_results.db | run_kernel_stats.csv>

Accepts the rocpd SQLite database or the ``--stats --output-format csv``
kernel statistics file.  Prints per-kernel call count, total, average, min and
max duration (us) and share of GPU time, most expensive first.
"""
from __future__ import annotations

import csv
import sqlite3
import sys


def _rows_db(path):
    con = sqlite3.connect(path)
    return con.execute(
        "select name, count(*), sum(duration), avg(duration), min(duration), max(duration) "
        "from kernels group by name order by sum(duration) desc").fetchall()


def _rows_csv(path):
    rows = []
    with open(path, newline="") as fh:
        for r in csv.DictReader(fh):
            rows.append((r["Name"], int(r["Calls"]), float(r["TotalDurationNs"]), float(r["AverageNs"]),
                         float(r["MinNs"]), float(r["MaxNs"])))
    rows.sort(key=lambda x: -x[2])
    return rows


def summarise(path: str, limit: int = 30) -> str:
    rows = _rows_csv(path) if path.endswith(".csv") else _rows_db(path)
    total = sum(r[2] for r in rows) or 1
    out = ["| kernel | calls | total us | avg us | min us | max us | % |", "|---|---|---|---|---|---|---|"]
    for name, n, tot, avg, mn, mx in rows[:limit]:
        short = name if len(name) < 110 else name[:107] + "..."
        out.append(f"| `{short}` | {n} | {tot / 1e3:.1f} | {avg / 1e3:.2f} | {mn / 1e3:.2f} | {mx / 1e3:.2f} | "
                   f"{100.0 * tot / total:.1f} |")
    return "\n".join(out)


if __name__ == "__main__":
    print(summarise(sys.argv[1]))
