"""Writes mid_n4096_histories.json: the FP64 oracle's run of Alg. 2 (branch
from the traces, Frobenius-norm error, parameterless stop) on the N = 4096
inputs of the three-gap workload (eigenvalues in [-1, -gap/2] and
[gap/2, 1], n_occ = 2048, gaps 0.1, 1e-2 and 1e-3, seeds 2001-2003): per
iteration the branch p_i, the error v_k = ||X~_k - X~_k^2||_F and the
traces, the stop index n, and the distance of X~_n from the exact D.

Calls only the oracle and the seeded input generator. Run from the
repository root (about a minute per gap on 8 cores):

    python tests/golden/make_mid_histories.py
"""
import json
import math
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import oracle  # noqa: E402
from workloads import config_mid  # noqa: E402

GAPS = [(0.1, 2001), (1e-2, 2002), (1e-3, 2003)]


def main() -> int:
    out = []
    for gap, seed in GAPS:
        t0 = time.time()
        inst = config_mid(gap=gap, seed=seed)
        ref = oracle.sp2(inst.F, inst.lambda_min, inst.lambda_max, inst.n_occ)
        D = oracle.density_from_eigenvectors(inst.Q, inst.n_occ)
        err = float(np.linalg.norm(ref.X - D))
        out.append(dict(gap=gap, seed=seed, n=int(inst.F.shape[0]), n_occ=int(inst.n_occ),
                        lambda_min=inst.lambda_min, lambda_max=inst.lambda_max,
                        status=ref.status.name, n_iter=int(ref.n), p=[int(x) for x in ref.p],
                        v=[float(x) for x in ref.v], t1=[float(x) for x in ref.t1],
                        t2=[float(x) for x in ref.t2],
                        err_fro_vs_exact_D=err, err_per_sqrt_nocc=err / math.sqrt(inst.n_occ)))
        print(f"gap {gap:g}: n = {ref.n}, {ref.status.name}, error {err:.3e}, "
              f"{time.time() - t0:.0f} s", flush=True)
    doc = {"_source": "written by tests/golden/make_mid_histories.py from the FP64 oracle",
           "workload": "dense N=4096, n_occ=2048, bands [-1,-gap/2] and [gap/2,1], bounds +-1",
           "runs": out}
    with open(os.path.join(HERE, "mid_n4096_histories.json"), "w") as fh:
        json.dump(doc, fh, indent=1)
    return 0


if __name__ == "__main__":
    sys.exit(main())
