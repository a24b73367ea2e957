"""The N = 8192 BF16x3 workload at full size, in the launch configuration
the benchmark times (the library's own choice of square kernel, the padded
row stride, the split of tail tiles): one fused square on sampled elements,
each computed one by one from the oracle's start X~_0 and its bf16 split;
a whole run against the exact D built from the eigenvectors; and its error
history against the eigenvalue-domain recursion while far above rounding
(Remark after Theorem 1: for a spectrally known input every iterate is the
scalar polynomial image of the eigenvalues)."""
import functools
import math

import numpy as np
import pytest

import oracle
from oracle.sp2 import _round_bf16, _store
from workloads import config_metric
from tests.gpu_helpers import print_case, square_bound

pytestmark = pytest.mark.gpu


@functools.lru_cache(maxsize=1)
def _inst():
    return config_metric()


def _run(inst, **kw):
    import torch

    import paper_1507_02087_amd as sp2
    F = torch.from_numpy(inst.F).to("cuda:0")
    res = sp2.run_dense(F, inst.lambda_min, inst.lambda_max, inst.n_occ,
                        precision="bf16x3", **kw)
    torch.cuda.synchronize()
    return res


def test_one_square_all_elements():
    """Every one of the N^2 entries of X~_1 after one fused square at full
    size, against S = H H + H L + L H formed on the host in FP64 from the
    oracle's X~_0 and its bf16 split H = bf16(x), L = bf16(x - H): the
    products of two bf16 values are exact in FP64 and the FP64 sums are
    far below the bound, so the host S is exact to ~1e-12."""
    inst = _inst()
    n = inst.F.shape[0]
    print_case(f"N={n} bf16x3 one square, all elements")
    res = _run(inst, max_iter=1)
    assert res.status_name == "NOT_CONVERGED" and res.n == 1
    X0 = _store(oracle.f0(inst.F, inst.lambda_min, inst.lambda_max), "bf16x3")
    t1, t2 = float(np.trace(X0)), float(np.sum(X0 * X0))
    p1 = oracle.choose_polynomial(t1, t2, inst.n_occ)
    assert res.p[1] == p1
    X32 = X0.astype(np.float32)
    H32 = _round_bf16(X32)
    L = _round_bf16(X32 - H32).astype(np.float64)
    HL = H32.astype(np.float64) + L          # exact: H and L share no bits
    del X32, H32
    S = HL @ HL
    S -= L @ L                               # H H + H L + L H
    del HL, L
    ref = S if p1 == 1 else 2.0 * X0 - S
    D = res.D.cpu().numpy()
    tol = square_bound(n, "bf16x3") + 2.0 ** -22
    diff = np.abs(D - ref)
    worst = float(diff.max())
    where = np.unravel_index(int(diff.argmax()), diff.shape)
    print(f"  worst |dx| over all {n * n} entries: {worst:.3e} at {where} "
          f"(bound {tol:.3e}); mean {float(diff.mean()):.3e}", flush=True)
    assert worst <= tol, (worst, where, tol)
    assert np.array_equal(D, D.T)


def _eigen_images(inst, p, steps):
    """v_k = ||x_k - x_k^2|| over the eigenvalue images of the run's own
    polynomial sequence (Remark after Theorem 1), k = 0 .. steps - 1."""
    lam = np.sort(np.asarray(inst.lam, dtype=np.float64))
    x = (inst.lambda_max - lam) / (inst.lambda_max - inst.lambda_min)
    out = []
    for k in range(steps):
        out.append(math.sqrt(float(np.sum((x - x * x) ** 2))))
        x = x * x if p[k + 1] == 1 else 2 * x - x * x
    return out


def test_full_run_against_exact_density():
    """The whole BF16x3 run at full size: the automatic stop, D against the
    exact D, and the error history against the eigenvalue images of its own
    polynomial sequence at every step down to the rounding floor. Floor: the
    run perturbs its iterate by Delta_k, and |v(X + Delta) - v(X)| <=
    ||Delta - X Delta - Delta X - Delta^2||_F <= 3 ||Delta||_F for
    ||X||_2 <= 1. Delta_k is rounding accumulated through steps whose
    polynomials have |p'| <= 2 on [0, 1], and at the end it is the distance
    of X~_n from D; the history is checked against 3 * 4 ||X~_n - D||_F
    (a factor 4 for Delta_k's growth over the two steps of an
    alternation) plus 1e-3 relative."""
    inst = _inst()
    n = inst.F.shape[0]
    print_case(f"N={n} bf16x3 full run")
    res = _run(inst)
    assert res.status_name == "OK", res.status_name
    D = res.D.cpu().numpy()
    De = oracle.density_from_eigenvectors(inst.Q, inst.n_occ)
    dist = float(np.linalg.norm(D - De))
    err = dist / math.sqrt(inst.n_occ)
    print(f"  n = {res.n}, {res.n_squares} squares, error {err:.3e}", flush=True)
    assert err <= 2e-4, err
    assert abs(float(np.trace(D)) - inst.n_occ) <= 1e-2
    exact = _eigen_images(inst, res.p, len(res.v))
    floor = 3.0 * 4.0 * dist
    worst = 0.0
    for k, (got, want) in enumerate(zip(res.v, exact)):
        dev = abs(got - want)
        worst = max(worst, dev / (floor + 1e-3 * want))
        print(f"  k={k:2d} v={got:.6e} eigen-image={want:.6e} |dv|={dev:.2e}", flush=True)
        assert dev <= floor + 1e-3 * want, (k, got, want, floor)
    print(f"  worst |dv| / (floor + 1e-3 v) = {worst:.3f}, floor {floor:.2e}", flush=True)


def test_full_run_fp64_against_exact_density():
    """The FP64 comparison run of the benchmark at full size: the automatic
    stop, D within 1e-11 sqrt(n_occ) of the exact D, the trace, and the
    error history against the eigenvalue images of its polynomial sequence
    (FP64 rounding moves each v_k by far less than 1e-6 relative while v_k
    is above 1e-6)."""
    inst = _inst()
    n = inst.F.shape[0]
    print_case(f"N={n} fp64 full run")
    import torch

    import paper_1507_02087_amd as sp2
    F = torch.from_numpy(inst.F).to("cuda:0")
    res = sp2.run_dense(F, inst.lambda_min, inst.lambda_max, inst.n_occ,
                        precision="fp64")
    torch.cuda.synchronize()
    assert res.status_name == "OK", res.status_name
    D = res.D.cpu().numpy()
    De = oracle.density_from_eigenvectors(inst.Q, inst.n_occ)
    err = float(np.linalg.norm(D - De)) / math.sqrt(inst.n_occ)
    print(f"  n = {res.n}, {res.n_squares} squares, error {err:.3e}, "
          f"{res.run_ms:.1f} ms", flush=True)
    assert err <= 1e-11, err
    assert abs(float(np.trace(D)) - inst.n_occ) <= 1e-8
    exact = _eigen_images(inst, res.p, len(res.v))
    for k, (got, want) in enumerate(zip(res.v, exact)):
        if want > 1e-6:
            assert got == pytest.approx(want, rel=1e-6), (k, got, want)


def test_batch_full_size():
    """The 512-instance FP32 batch (N uniform in [64, 1024], seed 4001) as the
    benchmark runs it: every instance stops by the test of Alg. 2 (the
    branch alternates, r < 1.8), and every 16th instance's D is the exact
    one within the FP32 tolerance."""
    import torch

    import paper_1507_02087_amd as sp2
    from workloads import batch_instances
    insts = batch_instances(count=512, seed=4001)
    print_case("512-instance fp32 batch, full size")
    Fs = [torch.from_numpy(i.F).to("cuda:0") for i in insts]
    res, ms = sp2.run_batch(Fs, [i.lambda_min for i in insts], [i.lambda_max for i in insts],
                            [i.n_occ for i in insts], precision="fp32")
    worst = 0.0
    for b, (inst, r) in enumerate(zip(insts, res)):
        assert r.status == sp2.OK, (b, r.status)
        assert r.p[r.n] != r.p[r.n - 1] and r.r[r.n] < 1.8, b
        if b % 16 == 0:
            De = oracle.density_from_eigenvectors(inst.Q, inst.n_occ)
            err = float(np.linalg.norm(r.D.cpu().numpy() - De)) / math.sqrt(inst.n_occ)
            worst = max(worst, err)
            assert err <= 2e-5, (b, err)
    print(f"  {ms:.2f} ms, worst sampled error {worst:.3e}", flush=True)


def test_bsr_full_size():
    """The block-sparse workload (banded N = 32768, 48 Givens layers, BSR
    32 x 32 FP32, truncation 1e-6, seed 5001) as the benchmark runs it: the
    stop of Alg. 2, the trace, and the distance from the exactly known D,
    block row by block row."""
    import torch

    import paper_1507_02087_amd as sp2
    from workloads.banded import banded_instance, to_bsr_blocks
    n = 32768
    inst = banded_instance(n=n, layers=48, seed=5001)
    print_case(f"bsr n={n} full size")
    rp, ci, bl = to_bsr_blocks(inst.F, 32)
    ctx = sp2.BsrContext(0)
    try:
        ctx.init_bsr(n, torch.from_numpy(rp).cuda(), torch.from_numpy(ci).cuda(),
                     torch.from_numpy(np.ascontiguousarray(bl)).cuda(),
                     inst.lambda_min, inst.lambda_max, inst.n_occ, trunc_tau=1e-6)
        st = ctx.run()
        n_it, n_sq, ms = ctx.get_info()
        hist = ctx.get_history()
        rpo, cio, blo = (t.cpu().numpy() for t in ctx.get_bsr(as_fp64=True))
    finally:
        ctx.close()
    assert st == sp2.OK
    assert hist["p"][n_it] != hist["p"][n_it - 1] and hist["r"][n_it] < 1.8
    De = inst.density_exact().tocsr()
    err2, tr = 0.0, 0.0
    for r in range(n // 32):
        rows = De[32 * r:32 * r + 32].toarray()
        got = np.zeros_like(rows)
        for q in range(rpo[r], rpo[r + 1]):
            c = cio[q]
            assert q == rpo[r] or c > cio[q - 1]     # sorted block columns
            got[:, 32 * c:32 * c + 32] = blo[q]
            if c == r:
                tr += float(np.trace(blo[q]))
        err2 += float(np.sum((got - rows) ** 2))
    err = math.sqrt(err2) / math.sqrt(inst.n_occ)
    print(f"  n = {n_it}, {ms:.2f} ms, error {err:.3e}", flush=True)
    assert err <= 1e-4, err
    assert abs(tr - inst.n_occ) <= 1e-3 * math.sqrt(n)
