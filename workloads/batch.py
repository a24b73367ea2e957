"""Many independent dense instances of uneven size (batched purification).

Each instance follows the dense recipe with bands [-1,-g/2] and [g/2,1],
n_occ = floor(N/2) and exact bounds -1 and 1; N and the gap g are drawn per
instance.
"""
from __future__ import annotations

import numpy as np

from .dense import dense_instance


def batch_instances(count: int = 512, n_lo: int = 64, n_hi: int = 1024,
                    gap_lo: float = 0.02, gap_hi: float = 0.2,
                    seed: int = 4001):
    rng = np.random.default_rng(seed)
    sizes = rng.integers(n_lo, n_hi + 1, size=count)
    gaps = rng.uniform(gap_lo, gap_hi, size=count)
    seeds = rng.integers(0, 2**31 - 1, size=count)
    out = []
    for n, g, s in zip(sizes, gaps, seeds):
        n = int(n)
        out.append(dense_instance(n, n // 2, -1.0, 1.0, float(g), int(s),
                                  label=f"batch N={n} gap={g:.3f}"))
    return out
