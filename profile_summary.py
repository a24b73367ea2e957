"""Summarises a rocprofv3 output database (kernel trace and, when present,
PMC counters) as short text for profiles/.

Usage: python profile_summary.py <results.db> [--min-us 20] [--match square]
       python profile_summary.py <fetch.db> --write-db <write.db> --match square
              --copy-bytes 1073741824 --source <kernel source> --config <name>

Per kernel it prints the dispatch count and mean duration over all
dispatches, and over the dispatches longer than --min-us (kernels of steps
queued after the stop return at once; they are excluded from the second
mean). With counters, it prints the per-dispatch mean of each counter over
the same long dispatches.

Traffic mode (--write-db): the first database holds a FETCH_SIZE pass and the
second a WRITE_SIZE pass of the same command, which ends with plain device
copies of --copy-bytes bytes. Each counter is scaled by the copy's known bytes
over what the counter reads for the copy; the scaled fetch and write bytes of
the matching kernels (main and tail kernel of one step) are summed per step
and printed as one TRAFFIC line with the SHA-256 of the kernel sources
(--source, repeatable; hashed in the given order), so a reader can tell
whether the figure still describes the current kernels. By default a step's
bytes are the per-kernel means over the long dispatches; with --per-step N
they are each kernel's total over all its dispatches divided by N (for a step
made of several kernels that also run, returning at once, after the stop).

--match takes alternatives separated by '|' (plain substrings).
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
    ap.add_argument("--write-db", default=None)
    ap.add_argument("--copy-bytes", type=float, default=float(1 << 30))
    ap.add_argument("--source", action="append", default=None)
    ap.add_argument("--config", default=None)
    ap.add_argument("--per-step", type=int, default=0)
    args = ap.parse_args()
    if args.write_db:
        return traffic(args)
    con = sqlite3.connect(args.db)
    cur = con.cursor()
    rows = cur.execute("select id, name, duration from kernels").fetchall()
    by = {}
    for kid, name, dur in rows:
        if not _matches(name, args.match):
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
            if not _matches(kname, args.match) and "copyBuffer" not in kname:
                continue
            if dur is not None and dur / 1e3 <= args.min_us and "copyBuffer" not in kname:
                continue
            vals.setdefault((kname, cname), []).append(v)
        for (kname, cname), vs in sorted(vals.items()):
            short = kname if len(kname) < 110 else kname[:107] + "..."
            print(f"{short} | {cname} | {len(vs)} | {statistics.mean(vs):.6g}")
    return 0


def _matches(name, match):
    return not match or any(m in name for m in match.split("|"))


def _counter_means(db, counter, match, min_us, copy_bytes, per_step=0):
    """Mean KiB per long dispatch of each matching kernel (with per_step: the
    total over all dispatches / per_step), and the counter's KiB for the
    calibration copies (dispatches of the copy kernel reading at least a
    quarter of copy_bytes)."""
    cur = sqlite3.connect(db).cursor()
    rows = cur.execute("select kernel_name, value, duration from counters_collection "
                       "where counter_name = ?", (counter,)).fetchall()
    per, copies = {}, []
    for kname, v, dur in rows:
        if "copyBuffer" in kname:
            if v * 1024.0 >= 0.25 * copy_bytes:
                copies.append(v)
            continue
        if not _matches(kname, match):
            continue
        if not per_step and dur is not None and dur / 1e3 <= min_us:
            continue
        per.setdefault(kname, []).append(v)
    if per_step:
        return {k: sum(v) / per_step for k, v in per.items()}, per, copies
    return {k: statistics.mean(v) for k, v in per.items()}, per, copies


def traffic(args) -> int:
    import hashlib
    import json
    fetch, fper, fcopy = _counter_means(args.db, "FETCH_SIZE", args.match,
                                        args.min_us, args.copy_bytes, args.per_step)
    write, wper, wcopy = _counter_means(args.write_db, "WRITE_SIZE", args.match,
                                        args.min_us, args.copy_bytes, args.per_step)
    if not fcopy or not wcopy:
        print("no calibration copy found in the databases", file=sys.stderr)
        return 1
    ff = args.copy_bytes / (statistics.mean(fcopy) * 1024.0)
    wf = args.copy_bytes / (statistics.mean(wcopy) * 1024.0)
    print(f"# traffic from {args.db} (FETCH_SIZE) and {args.write_db} (WRITE_SIZE)")
    print(f"# calibration: copies of {args.copy_bytes:.0f} B read as FETCH_SIZE "
          f"{statistics.mean(fcopy):.1f} KiB (x{ff:.3f}) and WRITE_SIZE "
          f"{statistics.mean(wcopy):.1f} KiB (x{wf:.3f}), {len(fcopy)}/{len(wcopy)} copies")
    print("kernel | long dispatches (fetch/write) | FETCH_SIZE KiB | WRITE_SIZE KiB | "
          "scaled read GB | scaled write GB")
    tot_r = tot_w = 0.0
    names = sorted(set(fetch) | set(write))
    for k in names:
        r = fetch.get(k, 0.0) * 1024.0 * ff
        w = write.get(k, 0.0) * 1024.0 * wf
        tot_r += r
        tot_w += w
        short = k if len(k) < 110 else k[:107] + "..."
        print(f"{short} | {len(fper.get(k, []))}/{len(wper.get(k, []))} | "
              f"{fetch.get(k, 0.0):.1f} | {write.get(k, 0.0):.1f} | "
              f"{r / 1e9:.4f} | {w / 1e9:.4f}")
    rec = {"config": args.config, "kernels": names, "read_bytes": round(tot_r),
           "write_bytes": round(tot_w), "bytes_per_step": round(tot_r + tot_w),
           "fetch_factor": round(ff, 4), "write_factor": round(wf, 4)}
    if args.per_step:
        rec["per_step"] = args.per_step
    if args.source:
        h = hashlib.sha256()
        for path in args.source:
            with open(path, "rb") as fh:
                h.update(fh.read())
        rec["sources"] = args.source
        rec["source_sha256"] = h.hexdigest()
    print("TRAFFIC " + json.dumps(rec))
    return 0


if __name__ == "__main__":
    sys.exit(main())
