"""Summarise a rocprofv3 kernel-trace database (rocpd SQLite) as a text table.

    python -m paper_2409_19156_amd.prof_summary <run_results.db> [command ...]

Prints per-kernel call count, total, average, min and max duration (us) and
share of GPU time, most expensive first.
"""
from __future__ import annotations

import sqlite3
import sys


def summarise(db_path: str, limit: int = 30) -> str:
    con = sqlite3.connect(db_path)
    rows = con.execute(
        "select name, count(*), sum(duration), avg(duration), min(duration), max(duration) "
        "from kernels group by name order by sum(duration) desc").fetchall()
    total = sum(r[2] for r in rows) or 1
    out = ["| kernel | calls | total us | avg us | min us | max us | % |", "|---|---|---|---|---|---|---|"]
    for name, n, tot, avg, mn, mx in rows[:limit]:
        short = name if len(name) < 110 else name[:107] + "..."
        out.append(f"| `{short}` | {n} | {tot / 1e3:.1f} | {avg / 1e3:.2f} | {mn / 1e3:.2f} | {mx / 1e3:.2f} | "
                   f"{100.0 * tot / total:.1f} |")
    return "\n".join(out)


if __name__ == "__main__":
    print(summarise(sys.argv[1]))
