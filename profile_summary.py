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
            "select p.event_id, i.name, p.value from rocpd_pmc_event p "
            "join rocpd_info_pmc i on p.pmc_id = i.id").fetchall()
    except sqlite3.Error:
        pmc = []
    if pmc:
        # map event ids to kernel dispatch ids
        try:
            ev2k = dict(cur.execute(
                "select event_id, id from rocpd_kernel_dispatch").fetchall())
        except sqlite3.Error:
            ev2k = {}
        print("\nkernel | counter | dispatches | mean per dispatch")
        for name, ids in long_ids.items():
            vals = {}
            for ev, cname, v in pmc:
                if ev2k.get(ev, ev) in ids:
                    vals.setdefault(cname, []).append(v)
            short = name if len(name) < 110 else name[:107] + "..."
            for cname, vs in sorted(vals.items()):
                print(f"{short} | {cname} | {len(vs)} | {statistics.mean(vs):.1f}")
    return 0


if __name__ == "__main__":
    sys.exit(main())
