"""GPU parity of batched SP2: many instances of uneven size in one launch
sequence, each with its own polynomial choices and its own stop."""
import math

import numpy as np
import pytest

import oracle
from oracle import Status
from workloads import dense_instance, batch_instances
from tests.gpu_helpers import print_case

pytestmark = pytest.mark.gpu

D_TOL = {"fp64": 1e-11, "fp32": 2e-5, "bf16x3": 2e-4}


def _mixed_instances():
    specs = [(40, 20, -1.0, 1.0, 0.2), (64, 30, -1.2, 0.8, 0.1),
             (100, 50, -1.0, 1.0, 0.01), (130, 64, -2.0, 1.5, 0.05),
             (257, 128, -1.0, 1.0, 0.15), (300, 151, -0.7, 1.3, 0.03),
             (77, 0, -1.0, 1.0, 0.1), (90, 90, -1.0, 1.0, 0.1)]
    return [dense_instance(n, no, lo, hi, g, seed=500 + i)
            for i, (n, no, lo, hi, g) in enumerate(specs)]


def _to_gpu(insts):
    import torch
    return [torch.from_numpy(i.F).cuda() for i in insts]


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16x3"])
def test_batch_matches_oracle_per_instance(prec):
    import paper_1507_02087_amd as sp2
    insts = _mixed_instances()
    print_case(f"batch of {len(insts)} prec={prec}")
    res, ms = sp2.run_batch(_to_gpu(insts), [i.lambda_min for i in insts],
                            [i.lambda_max for i in insts], [i.n_occ for i in insts],
                            precision=prec)
    for i, (inst, r) in enumerate(zip(insts, res)):
        ref = oracle.sp2(inst.F, inst.lambda_min, inst.lambda_max, inst.n_occ)
        assert ref.status == Status.OK
        assert r.status == sp2.OK, (i, r.status_name)
        D = r.D.cpu().numpy()
        err = np.linalg.norm(D - ref.X) / math.sqrt(max(1, inst.n_occ))
        assert err < D_TOL[prec], (i, err)
        if inst.n_occ in (0, inst.n):
            assert r.n == 0 and r.n_squares == 0
        else:
            assert r.p[r.n] != r.p[r.n - 1] and r.r[r.n] < 1.8
            if prec == "fp64":
                assert abs(r.n - ref.n) <= 6


@pytest.mark.parametrize("prec", ["fp64", "bf16x3"])
def test_batch_equals_single_runs_bitwise(prec):
    """Driven by a launch sequence per step without tail splits, a batch
    instance runs exactly the arithmetic of a single run of the same
    configuration: results and histories are equal bit for bit, and every
    instance stops on its own step. (The persistent driver runs a batch with
    one configuration; its equality with this driver is in
    test_gpu_persistent.py.)"""
    import torch
    import paper_1507_02087_amd as sp2
    insts = _mixed_instances()
    Fs = _to_gpu(insts)
    res, _ = sp2.run_batch(Fs, [i.lambda_min for i in insts],
                           [i.lambda_max for i in insts], [i.n_occ for i in insts],
                           precision=prec, tail_split=1, launch="sequence")
    stops = set()
    for inst, F, r in zip(insts, Fs, res):
        one = sp2.run_dense(F, inst.lambda_min, inst.lambda_max, inst.n_occ,
                            precision=prec, tail_split=1)
        assert (r.status, r.n, r.n_squares) == (one.status, one.n, one.n_squares)
        assert r.v == one.v and r.p == one.p
        assert torch.equal(r.D, one.D)
        stops.add(r.n)
    assert len(stops) >= 3   # instances stop at different steps


def test_batch_with_diverging_instance():
    import paper_1507_02087_amd as sp2
    good = dense_instance(120, 60, -1.0, 1.0, 0.1, seed=1)
    bad = dense_instance(64, 32, -1.0, 1.0, 0.2, seed=2)
    res, _ = sp2.run_batch(_to_gpu([good, bad]), [-1.0, -1.0], [1.0, -0.99], [60, 32])
    assert res[0].status == sp2.OK and res[1].status == sp2.DIVERGED
    ref = oracle.sp2(bad.F, -1.0, -0.99, 32)
    assert res[1].n == ref.n


def test_batch_uneven_sizes_sample():
    """A sample of the 512-instance workload (N uniform in [64, 1024], gap
    uniform in [0.02, 0.2]) in FP32 against the FP64 oracle."""
    import paper_1507_02087_amd as sp2
    insts = batch_instances(count=24, n_lo=64, n_hi=600, seed=4001)
    res, ms = sp2.run_batch(_to_gpu(insts), [i.lambda_min for i in insts],
                            [i.lambda_max for i in insts], [i.n_occ for i in insts],
                            precision="fp32")
    print_case(f"24-instance fp32 batch: {ms:.2f} ms")
    for inst, r in zip(insts, res):
        assert r.status == sp2.OK
        D_exact = oracle.density_from_eigenvectors(inst.Q, inst.n_occ)
        err = np.linalg.norm(r.D.cpu().numpy() - D_exact) / math.sqrt(inst.n_occ)
        assert err < D_TOL["fp32"], err
