"""Summarise rocprofv3 SQLite outputs as short text.

  python -m paper_2110_06322_amd.profile_summary stats <results.db>
      per-kernel calls, total and average duration (the --stats view)
  python -m paper_2110_06322_amd.profile_summary counter <results.db> <kernel-substring>
      per-dispatch value of the collected counter for matching kernels and for
      the device-to-device copy kernel used for calibration
  python -m paper_2110_06322_amd.profile_summary bursts <results.db> <kernel-substring> [min_run]
      launches of matching kernels that come in runs of at least min_run (default
      50) back-to-back dispatches with no other kernel between them (the
      bench's apply bursts), with their average duration
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


def bursts(db, pattern, min_run=50):
    """Average duration of matching launches inside runs of >= min_run consecutive
    matching dispatches (start-time order over all kernels)."""
    con = sqlite3.connect(db)
    rows = con.execute("select name, duration from kernels order by start").fetchall()
    runs, cur = [], []
    for name, dur in rows:
        if pattern in name:
            cur.append(dur)
        elif cur:
            runs.append(cur)
            cur = []
    if cur:
        runs.append(cur)
    sel = [r for r in runs if len(r) >= min_run]
    durs = [d for r in sel for d in r]
    total = sum(len(r) for r in runs)
    if not durs:
        print(f"no runs of {min_run} or more launches of '{pattern}' ({total} launches in all)")
        return
    print(f"runs={len(sel)} launches={len(durs)} of {total} avg_us={sum(durs) / len(durs) / 1e3:.3f} "
          f"median_us={statistics.median(durs) / 1e3:.3f} kernel~'{pattern}'")


if __name__ == "__main__":
    if sys.argv[1] == "stats":
        stats(sys.argv[2])
    elif sys.argv[1] == "bursts":
        bursts(sys.argv[2], sys.argv[3], int(sys.argv[4]) if len(sys.argv) > 4 else 50)
    else:
        counter(sys.argv[2], sys.argv[3])
