"""Summarises a rocprofv3 output database (kernel trace and, when present,
PMC counters) as short text for profiles/.

Usage: python profile_summary.py <results.db> [--min-us 20] [--match square]

Per kernel it prints the dispatch count and mean duration over all
dispatches, and over the dispatches longer than --min-us (kernels of steps
queued after the stop return at once; they are excluded from the second
mean). With counters, it prints the per-dispatch mean of each counter over
the same long dispatches.
"""
from __future__ import annotations

import argparse
import sqlite3
import statistics
import sys


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("db")
    ap.add_argument("--min-us", type=float, default=20.0)
    ap.add_argument("--match", default="")
    args = ap.parse_args()
    con = sqlite3.connect(args.db)
    cur = con.cursor()
    rows = cur.execute("select id, name, duration from kernels").fetchall()
    by = {}
    for kid, name, dur in rows:
        if args.match and args.match not in name:
            continue
        by.setdefault(name, []).append((kid, dur / 1e3))
    print(f"# rocprofv3 summary of {args.db}")
    print(f"# long dispatches: duration > {args.min_us} us")
    print("kernel | calls | mean_us(all) | long_calls | mean_us(long) | median_us(long) | min_us | max_us")
    long_ids = {}
    for name, lst in sorted(by.items(), key=lambda kv: -sum(d for _, d in kv[1])):
        ds = [d for _, d in lst]
        lg = [(k, d) for k, d in lst if d > args.min_us]
        lds = [d for _, d in lg]
        long_ids[name] = {k for k, _ in lg}
        short = name if len(name) < 110 else name[:107] + "..."
        print(f"{short} | {len(ds)} | {statistics.mean(ds):.1f} | {len(lds)} | "
              f"{(statistics.mean(lds) if lds else 0):.1f} | "
              f"{(statistics.median(lds) if lds else 0):.1f} | {min(ds):.1f} | {max(ds):.1f}")
    try:
        pmc = cur.execute(
            "select kernel_name, dispatch_id, counter_name, value, duration "
            "from counters_collection").fetchall()
    except sqlite3.Error:
        pmc = []
    if pmc:
        print("\nkernel | counter | long dispatches | mean value per dispatch")
        vals = {}
        for kname, _did, cname, v, dur in pmc:
            if args.match and args.match not in kname and "copyBuffer" not in kname:
                continue
            if dur is not None and dur / 1e3 <= args.min_us and "copyBuffer" not in kname:
                continue
            vals.setdefault((kname, cname), []).append(v)
        for (kname, cname), vs in sorted(vals.items()):
            short = kname if len(kname) < 110 else kname[:107] + "..."
            print(f"{short} | {cname} | {len(vs)} | {statistics.mean(vs):.6g}")
    return 0


if __name__ == "__main__":
    sys.exit(main())
