"""Summarise rocprofv3 SQLite outputs as short text.

  python -m paper_2110_06322_amd.profile_summary stats <results.db>
      per-kernel calls, total and average duration (the --stats view)
  python -m paper_2110_06322_amd.profile_summary counter <results.db> <kernel-substring>
      per-dispatch value of the collected counter for matching kernels and for
      the device-to-device copy kernel used for calibration
"""
from __future__ import annotations

import sqlite3
import statistics
import sys


def stats(db):
    """Per-kernel totals (rocprofv3's top_kernels view reports microseconds)."""
    con = sqlite3.connect(db)
    rows = con.execute("select name, total_calls, total_duration, average, percentage from top_kernels").fetchall()
    print(f"{'calls':>7} {'total_ms':>12} {'avg_us':>10} {'pct':>6}  kernel")
    for name, calls, tot, avg, pct in rows:
        print(f"{calls:7d} {tot / 1e3:12.3f} {avg:10.3f} {pct:6.2f}  {name}")


def counter(db, pattern):
    con = sqlite3.connect(db)
    rows = con.execute("select kernel_name, counter_name, value, grid_size from counters_collection").fetchall()
    groups = {}
    for name, cname, val, grid in rows:
        if pattern in name:
            key = ("kernel", name)
        elif "copyBuffer" in name and grid > 4096:
            key = ("copy", name)
        else:
            continue
        groups.setdefault((key, cname, grid), []).append(val)
    for ((kind, name), cname, grid), vals in sorted(groups.items()):
        print(f"{kind:6s} {cname:11s} dispatches={len(vals):3d} median_KiB={statistics.median(vals):12.1f} "
              f"grid={grid} {name}")


if __name__ == "__main__":
    if sys.argv[1] == "stats":
        stats(sys.argv[2])
    else:
        counter(sys.argv[2], sys.argv[3])
