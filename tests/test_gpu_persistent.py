"""The persistent batch driver (one graph-captured launch per run; each
instance advances and stops on its own): its results equal, bit for bit,
those of the launch-sequence driver with the same square-kernel
configuration and no tail split, because both compute every tile with the
same kernel code and take every scalar decision with the same code from
partial sums added in the same order. Covered: uneven sizes with ragged
tiles, the trivial occupations, a diverging instance, FP64/FP32/BF16x3,
SP2-ACC, graph reuse across runs and re-capture after an init, the full
512-instance batch, the error path when a queue wait exceeds its limit
(forced from the host with a zero limit; every kernel still returns) and the
argument checks. Every run also goes through the replay of its scalar
decisions (tests/conftest.py)."""
import math
import os

import numpy as np
import pytest

import oracle
from workloads import batch_instances, dense_instance
from tests.gpu_helpers import print_case

pytestmark = pytest.mark.gpu

D_TOL = {"fp64": 1e-11, "fp32": 2e-5, "bf16x3": 2e-4}


def _batch():
    sizes = ((64, 0.2), (200, 0.05), (333, 0.1), (96, 0.02), (150, 0.1), (700, 0.08),
             (129, 0.15), (512, 0.05))
    return [dense_instance(n, n // 2, -1.0, 1.0, g, seed=800 + n) for n, g in sizes]


def _to_gpu(insts):
    import torch
    return [torch.from_numpy(i.F).to("cuda:0") for i in insts]


def _pcfg(prec, nmax):
    """The configuration the persistent driver picks (1-based id)."""
    import paper_1507_02087_amd as sp2
    ctx = sp2.BatchContext(0)
    try:
        import torch
        F = torch.eye(nmax, dtype=torch.float64, device="cuda")
        ctx.batch_init([F, F], [-1.0, -1.0], [1.0, 1.0], [nmax // 2, nmax // 2],
                       precision=prec, launch="persistent")
        return ctx.get_config(0)[0]
    finally:
        ctx.close()


def _both(Fs, lo, hi, no, prec, **kw):
    import paper_1507_02087_amd as sp2
    cfg = _pcfg(prec, max(F.shape[0] for F in Fs))
    per, ms_p = sp2.run_batch(Fs, lo, hi, no, precision=prec, launch="persistent", **kw)
    seq, ms_s = sp2.run_batch(Fs, lo, hi, no, precision=prec, launch="sequence",
                              kernel_config=cfg, tail_split=1, **kw)
    return per, seq, ms_p, ms_s


def _eq(x, y):
    """Equal lists of floats, NaN where both have NaN."""
    return np.array_equal(np.asarray(x, float), np.asarray(y, float), equal_nan=True)


def _same(per, seq):
    import torch
    for b, (p, s) in enumerate(zip(per, seq)):
        assert (p.status, p.n, p.n_squares) == (s.status, s.n, s.n_squares), b
        assert _eq(p.v, s.v) and p.p == s.p and _eq(p.t1, s.t1) and _eq(p.t2, s.t2), b
        assert torch.equal(p.D, s.D), b


@pytest.mark.parametrize("prec", ["fp32", "fp64", "bf16x3"])
def test_persistent_equals_sequence(prec):
    import paper_1507_02087_amd as sp2
    insts = _batch()
    Fs = _to_gpu(insts)
    lo = [i.lambda_min for i in insts]
    hi = [i.lambda_max for i in insts]
    no = [i.n_occ for i in insts]
    # trivial occupations and an instance whose bounds miss the spectrum
    Fs += [Fs[0], Fs[1], Fs[2]]
    lo += [-1.0, -1.0, -1.0]
    hi += [1.0, 1.0, -0.99]
    no += [0, insts[1].n, insts[2].n_occ]
    print_case(f"persistent vs sequence, {len(Fs)} instances, {prec}")
    per, seq, ms_p, ms_s = _both(Fs, lo, hi, no, prec)
    _same(per, seq)
    assert per[-3].status == sp2.OK and per[-3].n == 0
    assert per[-2].status == sp2.OK and per[-2].n == 0
    assert per[-1].status == sp2.DIVERGED
    for inst, r in zip(insts, per):
        assert r.status == sp2.OK
        De = oracle.density_from_eigenvectors(inst.Q, inst.n_occ)
        err = float(np.linalg.norm(r.D.cpu().numpy() - De)) / math.sqrt(inst.n_occ)
        assert err < D_TOL[prec], (inst.n, err)
    print(f"  persistent {ms_p:.2f} ms, sequence {ms_s:.2f} ms", flush=True)


def test_persistent_acc_equals_sequence():
    insts = _batch()[:6]
    Fs = _to_gpu(insts)
    lo = [i.lambda_min for i in insts]
    hi = [i.lambda_max for i in insts]
    no = [i.n_occ for i in insts]
    b = [(float(i.lam[i.n_occ - 1]),) * 2 + (float(i.lam[i.n_occ]),) * 2 for i in insts]
    cols = [list(c) for c in zip(*b)]
    print_case("persistent vs sequence, SP2-ACC, fp32")
    per, seq, _, _ = _both(Fs, lo, hi, no, "fp32", homo_lumo=cols)
    _same(per, seq)


def test_persistent_graph_reuse_and_recapture():
    import torch
    import paper_1507_02087_amd as sp2
    insts = _batch()
    Fs = _to_gpu(insts)
    lo = [i.lambda_min for i in insts]
    hi = [i.lambda_max for i in insts]
    no = [i.n_occ for i in insts]
    ctx = sp2.BatchContext(0)
    try:
        ctx.batch_init(Fs, lo, hi, no, precision="fp32", launch="persistent")
        ctx.batch_run()
        first = [ctx.batch_get(b)[0].clone() for b in range(len(Fs))]
        ctx.batch_run()                       # the captured graph again
        for b in range(len(Fs)):
            assert torch.equal(first[b], ctx.batch_get(b)[0])
        # a new init with other instances captures a new run
        ctx.batch_init(Fs[:3], lo[:3], hi[:3], no[:3], precision="fp32",
                       launch="persistent")
        ctx.batch_run()
        for b in range(3):
            D, st, n, _ = ctx.batch_get(b)
            assert st == sp2.OK
            De = oracle.density_from_eigenvectors(insts[b].Q, insts[b].n_occ)
            assert np.linalg.norm(D.cpu().numpy() - De) / math.sqrt(insts[b].n_occ) < 2e-5
    finally:
        ctx.close()


def test_persistent_single_instance():
    import torch
    import paper_1507_02087_amd as sp2
    inst = dense_instance(777, 300, -1.0, 1.2, 0.1, seed=777)
    F = torch.from_numpy(inst.F).cuda()
    cfg = _pcfg("fp32", 777)
    a = sp2.run_dense(F, inst.lambda_min, inst.lambda_max, inst.n_occ, precision="fp32",
                      launch="persistent")
    b = sp2.run_dense(F, inst.lambda_min, inst.lambda_max, inst.n_occ, precision="fp32",
                      launch="sequence", kernel_config=cfg, tail_split=1)
    assert a.status == sp2.OK and a.n == b.n and a.v == b.v and torch.equal(a.D, b.D)


def test_persistent_full_batch_equals_sequence():
    """The 512-instance FP32 batch (N uniform in [64, 1024], seed 4001) as
    the benchmark runs it: every instance stops by the test of Alg. 2, and
    the persistent run equals the launch sequence with its configuration."""
    import paper_1507_02087_amd as sp2
    insts = batch_instances(count=512, seed=4001)
    Fs = _to_gpu(insts)
    lo = [i.lambda_min for i in insts]
    hi = [i.lambda_max for i in insts]
    no = [i.n_occ for i in insts]
    print_case("512-instance fp32 batch, persistent vs sequence")
    per, seq, ms_p, ms_s = _both(Fs, lo, hi, no, "fp32")
    _same(per, seq)
    worst = 0.0
    for b, (inst, r) in enumerate(zip(insts, per)):
        assert r.status == sp2.OK, b
        if b % 32 == 0:
            De = oracle.density_from_eigenvectors(inst.Q, inst.n_occ)
            err = float(np.linalg.norm(r.D.cpu().numpy() - De)) / math.sqrt(inst.n_occ)
            worst = max(worst, err)
            assert err <= 2e-5, (b, err)
    print(f"  persistent {ms_p:.2f} ms, sequence {ms_s:.2f} ms, worst sampled error "
          f"{worst:.2e}", flush=True)


def test_persistent_wait_limit_reports_error(monkeypatch):
    """With a zero wait limit (forced from the host) a workgroup that finds
    no published item gives up at once: every kernel returns, and the run
    reports the error instead of an outcome."""
    import paper_1507_02087_amd as sp2
    insts = _batch()[:3]
    Fs = _to_gpu(insts)
    monkeypatch.setenv("SP2_PERSIST_WAIT_MS", "0")
    ctx = sp2.BatchContext(0)
    monkeypatch.delenv("SP2_PERSIST_WAIT_MS")
    try:
        ctx.batch_init(Fs, [i.lambda_min for i in insts], [i.lambda_max for i in insts],
                       [i.n_occ for i in insts], precision="fp32", launch="persistent")
        with pytest.raises(sp2.SP2Error) as e:
            ctx.batch_run()
        assert e.value.status == sp2.HIP_ERROR
        assert "limit" in str(e.value)
    finally:
        ctx.close()
    # a context made afterwards (default limit) runs normally
    out, _ = sp2.run_batch(Fs, [i.lambda_min for i in insts], [i.lambda_max for i in insts],
                           [i.n_occ for i in insts], precision="fp32", launch="persistent")
    assert all(r.status == sp2.OK for r in out)


def test_persistent_argument_errors():
    import torch
    import paper_1507_02087_amd as sp2
    F = torch.eye(64, dtype=torch.float64, device="cuda")
    ctx = sp2.BatchContext(0)
    try:
        with pytest.raises(sp2.SP2Error) as e:   # Frobenius norm only
            ctx.batch_init([F, F], [-1.0, -1.0], [1.0, 1.0], [32, 32], precision="fp32",
                           norm="mixed", launch="persistent")
        assert e.value.status == sp2.INVALID_ARG
        big = next(c["id"] for c in sp2.kernel_configs() if c["name"] == "F32_256_2x4")
        with pytest.raises(sp2.SP2Error) as e:   # a configuration not compiled for it
            ctx.batch_init([F, F], [-1.0, -1.0], [1.0, 1.0], [32, 32], precision="fp32",
                           kernel_config=big, launch="persistent")
        assert e.value.status == sp2.INVALID_ARG
        ctx.batch_init([F, F], [-1.0, -1.0], [1.0, 1.0], [32, 32], precision="fp32",
                       launch="persistent")
        with pytest.raises(sp2.SP2Error) as e:   # McWeeny runs step by step
            ctx.set_mcweeny([0.0, 0.0])
        assert e.value.status == sp2.INVALID_ARG
    finally:
        ctx.close()
