"""Summarise rocprofv3 output as text tables.

    python -m paper_2409_19156_amd.prof_summary <run_results.db | run_kernel_stats.csv>
    python -m paper_2409_19156_amd.prof_summary <run_counter_collection.csv> [kernel-name filter]

Kernel traces (the rocpd SQLite database or the ``--stats --output-format csv``
kernel statistics file): per-kernel call count, total, average, min and max
duration (us) and share of GPU time, most expensive first.

Counter collections (``--pmc ... --output-format csv``): per kernel, each
counter summed over its instances within a dispatch and averaged over the
dispatches, plus the ratios the SQ counters give when present: MFMA-busy
cycles per GPU-active cycle, LDS bank-conflict cycles per LDS-active cycle,
and LDS-wait cycles per wave cycle.
"""
from __future__ import annotations

import collections
import csv
import re
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


def _short(name: str) -> str:
    m = re.search(r"([A-Za-z_][A-Za-z0-9_]*(<[^()]*>)?)\(", name)
    return m.group(1) if m else name[:60]


def summarise_counters(path: str, name_filter: str = "") -> str:
    sums = collections.defaultdict(lambda: collections.defaultdict(float))  # (kernel, dispatch) -> counter -> sum
    with open(path, newline="") as fh:
        for r in csv.DictReader(fh):
            if name_filter and name_filter not in r["Kernel_Name"]:
                continue
            sums[(_short(r["Kernel_Name"]), r["Dispatch_Id"])][r["Counter_Name"]] += float(r["Counter_Value"])
    per = collections.defaultdict(list)
    for (k, _), c in sums.items():
        per[k].append(c)
    names = sorted({n for c in sums.values() for n in c})
    out = ["| kernel | dispatches | " + " | ".join(names) + " | MFMA busy / GUI active | LDS conflict / LDS active "
           "| LDS wait / wave cycles |", "|---" * (len(names) + 5) + "|"]

    def ratio(avg, a, b):
        return f"{avg[a] / avg[b]:.3f}" if a in avg and avg.get(b) else "-"

    for k in sorted(per):
        ds = per[k]
        avg = {n: sum(d.get(n, 0.0) for d in ds) / len(ds) for n in names}
        cells = " | ".join(f"{avg[n]:.4g}" for n in names)
        out.append(f"| `{k}` | {len(ds)} | {cells} | {ratio(avg, 'SQ_VALU_MFMA_BUSY_CYCLES', 'GRBM_GUI_ACTIVE')} | "
                   f"{ratio(avg, 'SQ_LDS_BANK_CONFLICT', 'SQ_LDS_IDX_ACTIVE')} | "
                   f"{ratio(avg, 'SQ_WAIT_INST_LDS', 'SQ_WAVE_CYCLES')} |")
    return "\n".join(out)


if __name__ == "__main__":
    if "counter_collection" in sys.argv[1]:
        print(summarise_counters(sys.argv[1], sys.argv[2] if len(sys.argv) > 2 else ""))
    else:
        print(summarise(sys.argv[1]))
