"""GPU parity of the spectral-norm stop (Alg. 2's e_k = ||X~_k - X~_k^2||_2)
against the FP64 oracle: the Lanczos estimate of the first error on inputs
whose extreme eigenvalue of E is isolated (every precision, ragged sizes,
a negative extreme), full runs, a batch whose instances finish their Lanczos
processes at different steps, SP2-ACC and McW-ACC with the spectral norm,
determinism, and the error paths, through the C ABI."""
import math

import numpy as np
import pytest

import oracle
from oracle import Status
from oracle.mcweeny import mcweeny
from workloads import config_small, dense_instance
from workloads.dense import assemble, random_orthogonal
from workloads.banded import banded_instance, to_bsr_blocks
from tests.gpu_helpers import print_case

pytestmark = pytest.mark.gpu

D_TOL = {"fp64": 1e-11, "fp32": 2e-5, "bf16x3": 2e-4}
U_EFF = {"fp64": 2.0 ** -53, "fp32": 2.0 ** -24, "bf16x3": 2.0 ** -16}
# Where the top eigenvalues of E cluster (the first steps, spectrum of X~
# spread over [0, 1]), 64 Lanczos steps leave the Ritz value below the norm
# by up to ~3e-4 relative (measured with the same process in FP64 on the CPU)
CLUSTER_REL = 2e-3


def _exact_spectral(X):
    """||X - X^2||_2 of a stored iterate, in FP64."""
    return float(np.max(np.abs(np.linalg.eigvalsh(X - X @ X))))


def _isolated_instance(n, seed, outlier=None):
    """Dense F with random eigenvectors whose X_0 = (1 I - F)/2 has one
    eigenvalue near 1/2 (lambda = -0.03) and the rest at distance >= 1/4
    from it, so E_0's top eigenvalue is isolated; `outlier` puts one
    eigenvalue outside the bounds [-1, 1], which makes E_0's bottom
    eigenvalue the largest in magnitude."""
    rng = np.random.default_rng(seed)
    n_occ = max(1, n // 2)
    occ = rng.uniform(-1.0, -0.5, n_occ)
    occ[-1] = -0.03
    virt = rng.uniform(0.5, 1.0, n - n_occ)
    if outlier is not None:
        virt[-1] = outlier
    lam = np.sort(np.concatenate([occ, virt]))
    Q = random_orthogonal(n, rng)
    return assemble(Q, lam), n_occ


def _stored_x0(F, prec):
    X = (1.0 * np.eye(F.shape[0]) - F) / 2.0
    return X if prec == "fp64" else X.astype(np.float32).astype(np.float64)


def _run(F, lmin, lmax, n_occ, **kw):
    import torch
    import paper_1507_02087_amd as sp2
    Ft = torch.from_numpy(np.ascontiguousarray(F)).to("cuda:0")
    res = sp2.run_dense(Ft, lmin, lmax, n_occ, norm="spectral", **kw)
    torch.cuda.synchronize()
    return res


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16x3"])
@pytest.mark.parametrize("n", [2, 31, 33, 300, 1000])
def test_first_spectral_norm_isolated(prec, n):
    """e_0 = ||X~_0 - X~_0^2||_2 of the stored X~_0, isolated top: the
    Lanczos estimate converges to the exact value (partial chunks of 2, 31,
    1 and 8 rows; one to 32 chunks)."""
    F, n_occ = _isolated_instance(n, seed=50 + n)
    print_case(f"spectral e0 n={n} prec={prec}")
    res = _run(F, -1.0, 1.0, n_occ, precision=prec, max_iter=1)
    assert res.status_name == "NOT_CONVERGED" and len(res.m) == 1
    ref = _exact_spectral(_stored_x0(F, prec))
    assert res.m[0] == pytest.approx(ref, rel=1e-10), (res.m[0], ref)
    # spectral <= Frobenius (the latter from the working-precision square)
    assert res.m[0] <= res.v[0] * (1 + 1e-12) + 8 * n * U_EFF[prec]


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_negative_extreme(prec):
    """An eigenvalue of F above lambda_max maps to x < 0, where x - x^2 is
    negative and larger in magnitude than any positive eigenvalue of E: the
    estimate is the magnitude of the bottom Ritz value."""
    F, n_occ = _isolated_instance(200, seed=9, outlier=1.5)
    print_case(f"spectral negative extreme prec={prec}")
    res = _run(F, -1.0, 1.0, n_occ, precision=prec, max_iter=1)
    X = _stored_x0(F, prec)
    ev = np.linalg.eigvalsh(X - X @ X)
    assert -ev[0] > ev[-1] > 0.2
    assert res.m[0] == pytest.approx(-ev[0], rel=1e-10)


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16x3"])
def test_spectral_full_run(prec):
    """N = 512: the stop driven by the spectral norm fires on an alternation
    with r < 1.8 computed from e; the e history follows the oracle's (which
    takes the exact eigenvalues of X~ - S); D matches the oracle and the
    exact D."""
    inst = config_small()
    print_case(f"spectral full run N=512 prec={prec}")
    res = _run(inst.F, inst.lambda_min, inst.lambda_max, inst.n_occ, precision=prec)
    ref = oracle.sp2(inst.F, inst.lambda_min, inst.lambda_max, inst.n_occ,
                     norm="spectral", working=prec)
    assert res.status_name == "OK" and ref.status == Status.OK
    D = res.D.cpu().numpy()
    assert np.linalg.norm(D - ref.X) / math.sqrt(inst.n_occ) < D_TOL[prec]
    D_exact = oracle.density_from_eigenvectors(inst.Q, inst.n_occ)
    assert np.linalg.norm(D - D_exact) / math.sqrt(inst.n_occ) < D_TOL[prec]
    k = res.n
    print_case(f"  n_gpu={k} n_oracle={ref.n}")
    assert res.p[k] != res.p[k - 1] and 0 < res.m[k - 2] < 1.0
    r = math.log(res.m[k] / oracle.C_SP2) / math.log(res.m[k - 2])
    assert r < oracle.Q_TILDE and res.r[k] == pytest.approx(r, rel=1e-12)
    u = U_EFF[prec]
    for j, (x, y) in enumerate(zip(res.m, ref.v)):
        if y > 1e-3 and res.p[:j + 1] == ref.p[:j + 1]:
            assert abs(x - y) <= (CLUSTER_REL + 100 * (j + 1) * u) * y, (j, x, y)
    if prec == "fp64":
        assert abs(res.n - ref.n) <= 6
        # in the quadratic phase (isolated top) the estimate is converged
        for j, (x, y) in enumerate(zip(res.m, ref.v)):
            if 1e-9 < y < 0.2 and res.p[:j + 1] == ref.p[:j + 1]:
                assert x == pytest.approx(y, rel=1e-6), (j, x, y)


def test_spectral_batch():
    """Batch of uneven sizes (and one trivial instance) in FP64: the
    instances' Lanczos processes run in one launch per step and finish at
    different Lanczos steps; each one's e history and D against the
    oracle."""
    import torch
    import paper_1507_02087_amd as sp2
    insts = [dense_instance(n, n // 2, -1.0, 1.0, g, seed=600 + n)
             for n, g in ((64, 0.2), (200, 0.05), (333, 0.1), (97, 0.3))]
    Fs = [torch.from_numpy(i.F).cuda() for i in insts] + [torch.from_numpy(insts[0].F).cuda()]
    lo = [i.lambda_min for i in insts] + [-1.0]
    hi = [i.lambda_max for i in insts] + [1.0]
    no = [i.n_occ for i in insts] + [0]
    out, _ = sp2.run_batch(Fs, lo, hi, no, precision="fp64", norm="spectral")
    for inst, r in zip(insts, out):
        print_case(f"spectral batch member n={inst.n}")
        ref = oracle.sp2(inst.F, inst.lambda_min, inst.lambda_max, inst.n_occ,
                         norm="spectral")
        assert r.status == sp2.OK and ref.status == Status.OK
        for j, (x, y) in enumerate(zip(r.m, ref.v)):
            if y > 1e-9 and r.p[:j + 1] == ref.p[:j + 1]:
                assert abs(x - y) <= CLUSTER_REL * y + 1e-14, (j, x, y)
        assert np.linalg.norm(r.D.cpu().numpy() - ref.X) < 1e-11 * math.sqrt(inst.n_occ)
    assert out[-1].status == sp2.OK and out[-1].n == 0 and out[-1].m == []


def test_spectral_deterministic():
    """Two runs give the same e history bit for bit (every sum over chunks is
    taken in a fixed order)."""
    inst = dense_instance(700, 350, -1.0, 1.0, 0.05, seed=77)
    a = _run(inst.F, -1.0, 1.0, 350, precision="fp32")
    b = _run(inst.F, -1.0, 1.0, 350, precision="fp32")
    assert a.m == b.m and a.n == b.n


def test_spectral_acc():
    """SP2-ACC (Alg. 3/4) with the spectral norm, the error the paper's
    Alg. 4 reads: the schedule is followed and the stop fires at or after
    n_min as in the oracle."""
    inst = config_small()
    h, l = float(inst.lam[inst.n_occ - 1]), float(inst.lam[inst.n_occ])
    sched = oracle.acc_schedule(inst.lambda_min, inst.lambda_max, h, h, l, l)
    print_case("spectral SP2-ACC N=512 fp64")
    res = _run(inst.F, inst.lambda_min, inst.lambda_max, inst.n_occ,
               homo_lumo=(h, h, l, l))
    ref = oracle.sp2_acc(inst.F, inst.lambda_min, inst.lambda_max, sched, norm="spectral")
    assert res.status_name == "OK" and ref.status == Status.OK
    assert res.p[1:res.n + 1] == sched.p[1:res.n + 1]
    assert abs(res.n - ref.n) <= 2
    assert np.linalg.norm(res.D.cpu().numpy() - ref.X) < 1e-11 * math.sqrt(inst.n_occ)


@pytest.mark.parametrize("acc", [False, True])
def test_spectral_mcweeny(acc):
    """McWeeny / McW-ACC with the spectral norm (C = 4, the stop tested from
    step 1 and the stretch kept on): step count and D against the oracle."""
    inst = config_small()
    h, l = float(inst.lam[inst.n_occ - 1]), float(inst.lam[inst.n_occ])
    mu, xi = 0.5 * (h + l), (l - h if acc else None)
    print_case(f"spectral McWeeny acc={acc}")
    res = _run(inst.F, inst.lambda_min, inst.lambda_max, inst.n_occ, mcweeny=(mu, xi))
    ref = mcweeny(inst.F, inst.lambda_min, inst.lambda_max, mu, xi=xi, norm="spectral")
    assert res.status_name == "OK" and ref.status == Status.OK
    assert abs(res.n - ref.n) <= 1
    for j, (x, y) in enumerate(zip(res.m, ref.v)):
        if y > 1e-9:
            assert abs(x - y) <= CLUSTER_REL * y + 1e-14, (j, x, y)
    assert np.linalg.norm(res.D.cpu().numpy() - ref.X) < 1e-11 * math.sqrt(inst.n_occ)


def test_spectral_argument_errors():
    import torch
    import paper_1507_02087_amd as sp2
    inst = dense_instance(64, 32, -1.0, 1.0, 0.2, seed=2)
    F = torch.from_numpy(inst.F).cuda()
    ctx = sp2.Context(0)
    ctx.init_dense(F, -1.0, 1.0, 32)
    assert ctx.run() == sp2.OK
    with pytest.raises(sp2.SP2Error) as e:      # Frobenius run: no norm history
        ctx.get_norm_history()
    assert e.value.status == sp2.BAD_STATE
    ctx.init_dense(F, -1.0, 1.0, 32, norm="spectral")
    assert ctx.run() == sp2.OK
    assert len(ctx.get_norm_history()) == ctx.get_info()[1]
    with pytest.raises(sp2.SP2Error) as e:      # not a mixed-norm run
        ctx.get_mixed_history()
    assert e.value.status == sp2.BAD_STATE
    ctx.close()
    b = banded_instance(n=256, layers=4, seed=3)
    rp, ci, bl = to_bsr_blocks(b.F, 32)
    bctx = sp2.BsrContext(0)
    # block-sparse runs take the spectral norm too, and report its history
    bctx.init_bsr(256, torch.from_numpy(rp).cuda(), torch.from_numpy(ci).cuda(),
                  torch.from_numpy(np.ascontiguousarray(bl)).cuda(), b.lambda_min,
                  b.lambda_max, b.n_occ, norm="spectral")
    assert bctx.run() == sp2.OK
    assert len(bctx.get_norm_history()) == bctx.get_info()[1]
    with pytest.raises(sp2.SP2Error) as e:      # not a mixed-norm run
        bctx.get_mixed_history()
    assert e.value.status == sp2.BAD_STATE
    bctx.close()


@pytest.mark.parametrize("n,layers,tau", [(1024, 12, 1e-6), (1000, 20, 1e-5)])
def test_spectral_block_sparse(n, layers, tau):
    """The spectral-norm stop on the block-sparse path (the Lanczos products
    walk the flagged blocks of each block row of the stored iterate) against
    the FP64 oracle run on the dense form with the same truncation and norm:
    D, the e history (within the Lanczos cluster tolerance while the
    trajectories agree) and the stop index (against the oracle with FP32
    storage, whose rounding level sets where the error stagnates)."""
    import torch
    import paper_1507_02087_amd as sp2
    b = banded_instance(n=n, layers=layers, seed=17 + n)
    rp, ci, bl = to_bsr_blocks(b.F, 32)
    print_case(f"spectral block-sparse n={n} layers={layers} tau={tau}")
    ctx = sp2.BsrContext(0)
    try:
        ctx.init_bsr(n, torch.from_numpy(rp).cuda(), torch.from_numpy(ci).cuda(),
                     torch.from_numpy(np.ascontiguousarray(bl)).cuda(), b.lambda_min,
                     b.lambda_max, b.n_occ, trunc_tau=tau, norm="spectral")
        st = ctx.run()
        D = ctx.get_density(as_fp64=True).cpu().numpy()
        n_it, _, _ = ctx.get_info()
        hist = ctx.get_history()
        m = ctx.get_norm_history()
    finally:
        ctx.close()
    Fd = b.F.toarray()
    ref = oracle.sp2(Fd, b.lambda_min, b.lambda_max, b.n_occ, tau=tau, norm="spectral")
    ref32 = oracle.sp2(Fd, b.lambda_min, b.lambda_max, b.n_occ, tau=tau, norm="spectral",
                       working="fp32")
    assert st == sp2.OK and ref.status == Status.OK
    err = np.linalg.norm(D - ref.X) / math.sqrt(b.n_occ)
    print(f"  n_gpu={n_it} n_oracle={ref.n} (fp32 storage {ref32.n}) err={err:.2e}",
          flush=True)
    assert err < 1e-4
    assert abs(n_it - ref32.n) <= 2
    assert len(m) == n_it + 1
    u = U_EFF["fp32"]
    for j, (x, y) in enumerate(zip(m, ref.v)):
        if y > 1e-3 and hist["p"][:j + 1] == ref.p[:j + 1]:
            assert abs(x - y) <= (CLUSTER_REL + 100 * (j + 1) * u) * y, (j, x, y)


def test_spectral_krylov_and_timing():
    """The Lanczos steps behind each estimate (1..64) and the per-step
    duration of the spectral launch (HIP events) are reported."""
    import torch
    import paper_1507_02087_amd as sp2
    inst = dense_instance(300, 150, -1.0, 1.0, 0.1, seed=31)
    F = torch.from_numpy(inst.F).cuda()
    ctx = sp2.Context(0)
    ctx.init_dense(F, -1.0, 1.0, 150, precision="fp32", norm="spectral",
                   kernel_timing=True)
    assert ctx.run() == sp2.OK
    e, ks = ctx.get_norm_history(krylov=True)
    sq = ctx.get_info()[1]
    assert len(e) == len(ks) == sq
    assert all(1 <= k <= 64 for k in ks)
    nt = ctx.get_norm_times()
    assert len(nt) == sq and all(t > 0 for t in nt)
    ctx.init_dense(F, -1.0, 1.0, 150, precision="fp32", norm="mixed", kernel_timing=True)
    assert ctx.run() == sp2.OK
    with pytest.raises(sp2.SP2Error) as err:   # no spectral launches timed
        ctx.get_norm_times()
    assert err.value.status == sp2.BAD_STATE
    _, ks = ctx.get_norm_history(krylov=True)
    assert all(1 <= k <= 64 for k in ks)
    ctx.close()


def test_spectral_with_presplit_config():
    """The pre-split BF16x3 family normally leaves the FP32 iterate's lower
    triangle unwritten (only its bf16 split is read by the next square);
    with the spectral norm, whose products read whole rows of the iterate,
    the mirror is written: the errors of the first steps match the FP32
    oracle's, and D (rebuilt from the upper triangle otherwise) matches."""
    import paper_1507_02087_amd as sp2
    cfg = [c["id"] for c in sp2.kernel_configs() if c["name"] == "B3P_256_2x4_32"][0]
    F, n_occ = _isolated_instance(300, seed=77)
    print_case(f"spectral with presplit config {cfg}")
    res = _run(F, -1.0, 1.0, n_occ, precision="bf16x3", max_iter=3, kernel_config=cfg)
    ref = oracle.sp2(F, -1.0, 1.0, n_occ, norm="spectral", working="bf16x3", max_iter=3)
    assert len(res.m) == 3
    for j, (x, y) in enumerate(zip(res.m, ref.v)):
        assert x == pytest.approx(y, rel=1e-3), (j, x, y)
    D = res.D.cpu().numpy()
    assert np.array_equal(D, D.T)
    assert np.max(np.abs(D - ref.X)) < 1e-3
