"""Writes tests/golden/band_n32768.json: the FP64 CSR oracle's run of the
block-sparse workload at full size (N = 32768, banded F with entries
exp(-|i-j|/8) z, alternating diagonal shift for a gap of 0.1 at
n_occ = 16384, truncation 1e-6 after every step; seed 5001).

Stored: the input's parameters (so that a test can tell that it regenerated
the same input), the oracle's outcome (n, status, the error history v, the
traces and the polynomial sequence), the invariants of its D (trace,
||D - D^2||_F, ||F D - D F||_F), the Frobenius norm of every 32-row block
row of D, D at 4096 seeded positions inside the band, and a sketch of D:
the 64 numbers u_m^T D w_m for seeded standard-normal vectors u_m, w_m
(E (u^T A w)^2 = ||A||_F^2, so a test estimates ||D_test - D||_F from the
same vectors without the whole D being stored). Calls only
oracle/ (and the input generator); takes a few minutes on 8 cores.

    python tests/golden/make_band_golden.py
"""
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle.sp2_sparse import fro_csr, sp2_csr  # noqa: E402
from workloads.decay_band import decay_band_instance  # noqa: E402

N, SEED, TAU = 32768, 5001, 1e-6
SKETCH_SEED, SKETCH_M = 20151507, 64


def sketch_vectors(n, seed=SKETCH_SEED, m=SKETCH_M):
    """The seeded pairs (u_m, w_m) of the sketch, generated one at a time."""
    rng = np.random.default_rng(seed)
    for _ in range(m):
        yield rng.standard_normal(n), rng.standard_normal(n)


def main():
    t0 = time.time()
    inst = decay_band_instance(n=N, seed=SEED)
    print(f"input ready in {time.time() - t0:.1f} s: delta {inst.delta}, "
          f"gap {inst.gap:.7f}", flush=True)
    t0 = time.time()
    ref = sp2_csr(inst.F, inst.lambda_min, inst.lambda_max, inst.n_occ, tau=TAU)
    print(f"oracle: {ref.status.name} n = {ref.n} in {time.time() - t0:.1f} s",
          flush=True)
    D = ref.X.tocsr()
    D2 = D @ D
    FD = inst.F @ D
    rng = np.random.default_rng(32768)
    i = rng.integers(0, N, 4096)
    j = np.clip(i + rng.integers(-256, 257, 4096), 0, N - 1)
    i[:64] = j[:64] = np.arange(0, N, N // 64)          # some diagonal entries
    vals = np.asarray(D[i, j]).ravel()
    rows = D.power(2).sum(axis=1).A.ravel()
    blk = np.sqrt(rows.reshape(-1, 32).sum(axis=1))
    sketch = [float(u @ (D @ w)) for u, w in sketch_vectors(N)]
    out = dict(
        n=N, seed=SEED, tau=TAU, n_occ=inst.n_occ, delta=inst.delta,
        homo=inst.homo, lumo=inst.lumo, lambda_min=inst.lambda_min,
        lambda_max=inst.lambda_max, nnz_F=int(inst.F.nnz),
        oracle=dict(status=ref.status.name, n_iter=ref.n, v=ref.v, p=ref.p,
                    t1=ref.t1, t2=ref.t2, nnz_D=int(D.nnz)),
        trace=float(D.diagonal().sum()),
        idempotency_fro=fro_csr(D - D2),
        commutator_fro=fro_csr(FD - FD.T),
        F_fro=fro_csr(inst.F),
        block_row_fro=blk.tolist(),
        samples=[[int(a), int(b), float(c)] for a, b, c in zip(i, j, vals)],
        sketch_seed=SKETCH_SEED, sketch=sketch,
    )
    path = os.path.join(HERE, "band_n32768.json")
    with open(path, "w") as fh:
        json.dump(out, fh, indent=0)
    print(f"wrote {path}", flush=True)


if __name__ == "__main__":
    main()
