"""Autotuner of the square-kernel configuration per precision and size.

For each precision and each dimension in a list, every compiled kernel
configuration of that precision runs a few SP2 steps on a seeded dense
input (two-band spectrum) with the library's kernel timing; the fastest
median square time wins. Consecutive sizes with the same winner are merged
into entries (precision, n_max, configuration) and written as JSON, which
Context.load_kernel_table installs into the library. Configurations are
recorded by shape (tile, waves, K slice), not by id, so a table survives a
rebuild that renumbers them.

Run on the GPU: python -m paper_1507_02087_amd.autotune [--out FILE]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

SIZES = [64, 96, 128, 192, 256, 384, 512, 640, 768, 1024, 1536, 2048, 3072, 4096, 8192]


def _input(n: int):
    import numpy as np
    import torch
    rng = np.random.default_rng(n)
    lam = np.sort(np.concatenate([rng.uniform(-1, -0.05, n // 2),
                                  rng.uniform(0.05, 1, n - n // 2)]))
    G = rng.standard_normal((n, n))
    Q, _ = np.linalg.qr(G)
    F = (Q * lam) @ Q.T
    F = 0.5 * (F + F.T)
    return torch.from_numpy(F).cuda(), n // 2


def time_config(ctx, F, n_occ, precision, cfg_id, steps=4, reps=2):
    import numpy as np
    best = None
    for _ in range(reps):
        ctx.init_dense(F, -1.0, 1.0, n_occ, precision=precision, max_iter=steps,
                       kernel_config=cfg_id, kernel_timing=True)
        ctx.run()
        t = float(np.median(ctx.get_kernel_times()))
        best = t if best is None else min(best, t)
    return best


def autotune(sizes=SIZES, precisions=("fp64", "fp32", "bf16x3"), log=print):
    import paper_1507_02087_amd as sp2
    cfgs = sp2.kernel_configs()
    ctx = sp2.Context(0)
    results = []
    for n in sizes:
        F, n_occ = _input(n)
        for prec in precisions:
            row = {}
            for c in cfgs:
                if c["precision"] != prec:
                    continue
                row[c["id"]] = time_config(ctx, F, n_occ, prec, c["id"])
            win = min(row, key=row.get)
            results.append(dict(n=n, precision=prec, best=win,
                                ms={str(k): round(v, 5) for k, v in row.items()}))
            log(f"n={n} {prec}: best id {win} {row[win]:.4f} ms")
    ctx.close()
    by_id = {c["id"]: c for c in cfgs}
    entries = []
    for prec in precisions:
        rs = [r for r in results if r["precision"] == prec]
        for i, r in enumerate(rs):
            nxt = rs[i + 1] if i + 1 < len(rs) else None
            if nxt is not None and nxt["best"] == r["best"]:
                continue
            c = by_id[r["best"]]
            n_max = (r["n"] + nxt["n"]) // 2 if nxt is not None else 65536
            entries.append(dict(precision=prec, n_max=n_max, tile=c["tile"],
                                waves_m=c["waves_m"], waves_n=c["waves_n"],
                                k_slice=c["k_slice"]))
    return dict(entries=entries, measurements=results,
                note="median square-kernel time over 4 SP2 steps, best of 2 runs")


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default=None)
    ap.add_argument("--sizes", default=None)
    args = ap.parse_args()
    import paper_1507_02087_amd as sp2
    sizes = [int(x) for x in args.sizes.split(",")] if args.sizes else SIZES
    t0 = time.time()
    table = autotune(sizes)
    table["seconds"] = round(time.time() - t0, 1)
    out = args.out or sp2.TABLE_PATH
    with open(out, "w") as fh:
        json.dump(table, fh, indent=1)
    print(f"wrote {out}")
    return 0


if __name__ == "__main__":
    sys.exit(main())
