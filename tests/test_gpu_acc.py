"""GPU parity of SP2-ACC (Alg. 3 schedule + Alg. 4 scale-and-fold) against the
FP64 oracle, for the dense, batched and block-sparse paths, through the C ABI.

The schedule is fixed before the run, so the GPU and the oracle apply the
same polynomial with the same stretch at every step; their iterates differ
only by rounding (the GPU expands each polynomial in the one square it
computes, the oracle squares (1 - a) I + a X as written)."""
import math

import numpy as np
import pytest

import oracle
from oracle import Status
from workloads import config_small, dense_instance, diagonal_instance
from workloads.banded import banded_instance, to_bsr_blocks
from tests.gpu_helpers import print_case, square_bound

pytestmark = pytest.mark.gpu

PRECS = ("fp64", "fp32", "bf16x3")
D_TOL = {"fp64": 1e-11, "fp32": 2e-5, "bf16x3": 2e-4}
U_STORE = {"fp64": 2.0 ** -53, "fp32": 2.0 ** -24, "bf16x3": 2.0 ** -24}


def _exact_bounds(inst):
    """homo_out = homo_in = highest occupied, lumo_in = lumo_out = lowest
    unoccupied eigenvalue of the construction."""
    h, l = float(inst.lam[inst.n_occ - 1]), float(inst.lam[inst.n_occ])
    return h, h, l, l


def _configs():
    try:
        import paper_1507_02087_amd as sp2
        return [(c["precision"], c["id"]) for c in sp2.kernel_configs()]
    except Exception:
        return [(p, 0) for p in PRECS]


CONFIGS = _configs()


def _run(inst, bounds, accelerate=True, **kw):
    import torch
    import paper_1507_02087_amd as sp2
    F = torch.from_numpy(np.ascontiguousarray(inst.F)).to("cuda:0")
    res = sp2.run_dense(F, inst.lambda_min, inst.lambda_max, inst.n_occ,
                        homo_lumo=bounds, accelerate=accelerate, **kw)
    torch.cuda.synchronize()
    return res


@pytest.mark.parametrize("prec,cfg", CONFIGS)
@pytest.mark.parametrize("n", [31, 300])
@pytest.mark.parametrize("split", [0, 1])
def test_acc_first_step_elementwise(prec, cfg, n, split):
    """X~_1 = ((1 - a) I + a X~_0)^2 with a stretch a > 1.3, element by
    element against the FP64 oracle, for every kernel configuration: the
    stretched matrix Y = a X~_0 + (1 - a) I that the affine start stores is
    right in every tile, on the diagonal and off it, and in the ragged tail,
    and the step squares it."""
    inst = dense_instance(n, n // 2, -1.0, 1.3, 0.1, seed=2000 + n)
    b = _exact_bounds(inst)
    sched = oracle.acc_schedule(inst.lambda_min, inst.lambda_max, *b)
    assert sched.p[1] == 1 and sched.alpha[1] > 1.3
    print_case(f"acc first step n={n} prec={prec} cfg={cfg} split={split}")
    res = _run(inst, b, precision=prec, max_iter=1, kernel_config=cfg, tail_split=split)
    ref = oracle.sp2_acc(inst.F, inst.lambda_min, inst.lambda_max, sched, max_iter=1)
    assert res.status_name == "NOT_CONVERGED" and res.n == 1
    assert ref.status == Status.NOT_CONVERGED and ref.n == 1
    assert res.p[1] == 1
    D = res.D.cpu().numpy()
    a = sched.alpha[1]
    # Y = a X~_0 + (1 - a) I carries the storage rounding of X~_0 (scaled by
    # a) and its own; rows of Y have norm <= 1, so that rounding moves an
    # entry of Y^2 by at most 2 sqrt(n) (a + 1) u; the square itself is
    # within the square bound, and X~_1 is rounded once more
    u = U_STORE[prec]
    tol = square_bound(n, prec) + 2 * math.sqrt(n) * (a + 1) * u + 2 * u
    err = float(np.max(np.abs(D - ref.X)))
    assert err <= tol, (err, tol)
    assert np.array_equal(D, D.T)
    assert abs(res.t1[1] - ref.t1[1]) <= n * tol + 1e-12


@pytest.mark.parametrize("prec", PRECS)
def test_acc_full_run(prec):
    """Dense N = 512: the GPU follows the schedule, stops on an alternation
    at or after n_min (or at n_max), matches the oracle's D, and needs fewer
    squares than Alg. 2 on the same input."""
    import paper_1507_02087_amd as sp2
    inst = config_small()
    b = _exact_bounds(inst)
    sched = oracle.acc_schedule(inst.lambda_min, inst.lambda_max, *b)
    print_case(f"acc full run N=512 prec={prec}")
    res = _run(inst, b, precision=prec)
    ref = oracle.sp2_acc(inst.F, inst.lambda_min, inst.lambda_max, sched)
    assert res.status_name == "OK" and ref.status == Status.OK
    D = res.D.cpu().numpy()
    err = np.linalg.norm(D - ref.X) / math.sqrt(inst.n_occ)
    print_case(f"  n_gpu={res.n} n_oracle={ref.n} n_min={sched.n_min} "
               f"n_max={sched.n_max} err={err:.3e}")
    assert err < D_TOL[prec]
    D_exact = oracle.density_from_eigenvectors(inst.Q, inst.n_occ)
    assert np.linalg.norm(D - D_exact) / math.sqrt(inst.n_occ) < D_TOL[prec]
    assert res.p[1:res.n + 1] == sched.p[1:res.n + 1]
    assert res.n <= sched.n_max
    if res.n < sched.n_max:
        assert res.n >= sched.n_min and res.p[res.n] != res.p[res.n - 1]
        assert res.r[res.n] < 1.8
    if prec == "fp64":
        assert abs(res.n - ref.n) <= 2
    # History against the oracle while the error is well above rounding: the
    # GPU squares the stretched matrix like the oracle, so the relative
    # deviation stays within 100 (k + 1) u_eff (u_eff the working
    # precision's unit roundoff; bf16x3 carries 16 significant bits), capped
    # at 1e-2.
    u_eff = {"fp64": 2.0 ** -53, "fp32": 2.0 ** -24, "bf16x3": 2.0 ** -16}[prec]
    worst = 0.0
    for k, (x, y) in enumerate(zip(res.v, ref.v)):
        if y > 1e-3:
            bound = min(100 * (k + 1) * u_eff, 1e-2)
            worst = max(worst, abs(x - y) / y)
            assert abs(x - y) <= bound * y + 1e-13, (k, x, y, bound)
    print_case(f"  worst relative history deviation {worst:.2e}")
    plain = sp2.run_dense(res.D.new_tensor(inst.F), inst.lambda_min, inst.lambda_max,
                          inst.n_occ, precision=prec)
    assert res.n_squares < plain.n_squares


@pytest.mark.parametrize("prec", ["fp64", "bf16x3"])
def test_acc_ragged_and_padding(prec):
    """N = 333 (padded to the tile edge): the identity term of the fold must
    not reach the zero padding, or the traces and the error would include it."""
    inst = dense_instance(333, 170, -1.3, 0.9, 0.12, seed=333)
    b = _exact_bounds(inst)
    res = _run(inst, b, precision=prec)
    assert res.status_name == "OK"
    D = res.D.cpu().numpy()
    D_exact = oracle.density_from_eigenvectors(inst.Q, inst.n_occ)
    assert np.linalg.norm(D - D_exact) / math.sqrt(inst.n_occ) < D_TOL[prec]
    # traces reported by the device are those of the matrix proper
    assert abs(res.t1[res.n] - np.trace(D)) < 1e-6 * inst.n_occ
    assert abs(res.t1[res.n] - inst.n_occ) < 1e-3


def test_acc_loose_bounds_and_no_acceleration():
    """Looser outer bounds and the unaccelerated schedule (Theorem 2's
    setting) both reach D; without acceleration every stretch is 1."""
    inst = config_small()
    h, _, l, _ = _exact_bounds(inst)
    D_exact = oracle.density_from_eigenvectors(inst.Q, inst.n_occ)
    for bounds, acc in (((h - 0.3, h, l, l + 0.3), True), ((h, h, l, l), False)):
        sched = oracle.acc_schedule(inst.lambda_min, inst.lambda_max, *bounds, accelerate=acc)
        res = _run(inst, bounds, accelerate=acc)
        ref = oracle.sp2_acc(inst.F, inst.lambda_min, inst.lambda_max, sched)
        assert res.status_name == "OK"
        assert res.p[1:res.n + 1] == sched.p[1:res.n + 1]
        assert np.linalg.norm(res.D.cpu().numpy() - ref.X) < 1e-11 * math.sqrt(inst.n_occ)
        assert np.linalg.norm(res.D.cpu().numpy() - D_exact) < 1e-11 * math.sqrt(inst.n_occ)


def test_acc_diagonal_bitwise_pattern():
    """Diagonal F: every iterate stays diagonal (no fill from the identity
    term or the fold) and reaches the exact 0/1 projector."""
    rng = np.random.default_rng(3)
    d = np.concatenate([rng.uniform(-1.0, -0.05, 40), rng.uniform(0.05, 1.0, 24)])
    d[0], d[1] = -0.05, 0.05
    inst = diagonal_instance(d, 40, -1.0, 1.0, perm_seed=1)
    res = _run(inst, (-0.05, -0.05, 0.05, 0.05))
    D = res.D.cpu().numpy()
    assert res.status_name == "OK"
    assert np.max(np.abs(D - np.diag(np.diag(D)))) == 0.0
    occ = np.diag(inst.F) < 0
    assert np.max(np.abs(np.diag(D) - occ)) < 1e-14


def test_acc_reinit_returns_to_alg2():
    """A later init drops the schedule: the run equals a fresh Alg. 2 run."""
    import torch
    import paper_1507_02087_amd as sp2
    inst = dense_instance(256, 128, -1.0, 1.0, 0.1, seed=41)
    F = torch.from_numpy(inst.F).cuda()
    ctx = sp2.Context(0)
    ctx.init_dense(F, -1.0, 1.0, 128)
    ctx.set_homo_lumo(*_exact_bounds(inst))
    assert ctx.run() == sp2.OK
    acc_n = ctx.get_info()[0]
    ctx.init_dense(F, -1.0, 1.0, 128)
    assert ctx.run() == sp2.OK
    h = ctx.get_history()
    D = ctx.get_density()
    ctx.close()
    plain = sp2.run_dense(F, -1.0, 1.0, 128)
    assert h["p"] == plain.p and torch.equal(D, plain.D)
    assert acc_n < plain.n


def test_acc_argument_errors():
    import torch
    import paper_1507_02087_amd as sp2
    inst = dense_instance(64, 32, -1.0, 1.0, 0.2, seed=2)
    F = torch.from_numpy(inst.F).cuda()
    ctx = sp2.Context(0)
    with pytest.raises(sp2.SP2Error) as e:
        ctx.set_homo_lumo(-0.1, -0.1, 0.1, 0.1)
    assert e.value.status == sp2.BAD_STATE
    ctx.init_dense(F, -1.0, 1.0, 32)
    for b in ((-0.1, 0.1, 0.0, 0.2), (-1.0, -1.0, 0.1, 0.1), (-0.2, -0.1, 0.1, 1.5)):
        with pytest.raises(sp2.SP2Error) as e:
            ctx.set_homo_lumo(*b)
        assert e.value.status == sp2.INVALID_ARG
    with pytest.raises(sp2.SP2Error) as e:
        ctx.set_homo_lumo([-0.1, -0.1], [-0.1, -0.1], [0.1, 0.1], [0.1, 0.1])
    assert e.value.status == sp2.INVALID_ARG
    # the context still runs Alg. 2 after the rejected calls
    assert ctx.run() == sp2.OK
    ctx.close()


def test_acc_batch_matches_oracle_and_single_runs():
    """A batch of uneven sizes (one with n_occ = 0) under SP2-ACC: each
    instance matches the oracle, and the batch equals single runs bitwise."""
    import torch
    import paper_1507_02087_amd as sp2
    insts = [dense_instance(n, n // 2, -1.0, 1.0, g, seed=500 + n)
             for n, g in ((64, 0.2), (200, 0.05), (333, 0.1), (96, 0.02), (150, 0.1))]
    Fs = [torch.from_numpy(i.F).cuda() for i in insts]
    n_occ = [i.n_occ for i in insts] + [0]
    Fs.append(Fs[0])
    lo = [i.lambda_min for i in insts] + [-1.0]
    hi = [i.lambda_max for i in insts] + [1.0]
    bounds = [_exact_bounds(i) for i in insts] + [(-0.5, -0.5, 0.5, 0.5)]
    cols = [list(c) for c in zip(*bounds)]
    out, ms = sp2.run_batch(Fs, lo, hi, n_occ, homo_lumo=cols, precision="fp32",
                            tail_split=1)
    for b, inst in enumerate(insts):
        sched = oracle.acc_schedule(inst.lambda_min, inst.lambda_max, *bounds[b])
        ref = oracle.sp2_acc(inst.F, inst.lambda_min, inst.lambda_max, sched)
        r = out[b]
        assert r.status == sp2.OK and ref.status == Status.OK
        err = np.linalg.norm(r.D.cpu().numpy() - ref.X) / math.sqrt(inst.n_occ)
        assert err < D_TOL["fp32"], (b, err)
        assert r.p[1:r.n + 1] == sched.p[1:r.n + 1]
        single = sp2.run_dense(Fs[b], inst.lambda_min, inst.lambda_max, inst.n_occ,
                               precision="fp32", tail_split=1, homo_lumo=bounds[b])
        assert single.n == r.n and torch.equal(single.D, r.D)
    assert out[-1].status == sp2.OK and out[-1].n == 0
    assert float(out[-1].D.abs().max()) == 0.0


def test_acc_block_sparse_matches_truncated_oracle():
    """Banded N = 1024 (BSR FP32, tau = 1e-6) under SP2-ACC against the FP64
    oracle with the same truncation on the dense form."""
    import torch
    import paper_1507_02087_amd as sp2
    inst = banded_instance(n=1024, layers=12, seed=7 + 1024)
    tau = 1e-6
    b = (float(inst.lam[inst.n_occ - 1]),) * 2 + (float(inst.lam[inst.n_occ]),) * 2
    rp, ci, bl = to_bsr_blocks(inst.F, 32)
    ctx = sp2.BsrContext(0)
    ctx.init_bsr(1024, torch.from_numpy(rp).cuda(), torch.from_numpy(ci).cuda(),
                 torch.from_numpy(np.ascontiguousarray(bl)).cuda(), inst.lambda_min,
                 inst.lambda_max, inst.n_occ, trunc_tau=tau)
    ctx.set_homo_lumo(*b)
    st = ctx.run()
    D = ctx.get_density(as_fp64=True).cpu().numpy()
    n_it, n_sq, _ = ctx.get_info()
    h = ctx.get_history()
    ctx.close()
    sched = oracle.acc_schedule(inst.lambda_min, inst.lambda_max, *b)
    ref = oracle.sp2_acc(inst.F.toarray(), inst.lambda_min, inst.lambda_max, sched, tau=tau)
    assert st == sp2.OK and ref.status == Status.OK
    assert h["p"][1:n_it + 1] == sched.p[1:n_it + 1]
    err = np.linalg.norm(D - ref.X) / math.sqrt(inst.n_occ)
    err_exact = np.linalg.norm(D - inst.density_exact().toarray()) / math.sqrt(inst.n_occ)
    print_case(f"  bsr acc n_gpu={n_it} n_oracle={ref.n} err={err:.2e} exact={err_exact:.2e}")
    assert err < 1e-4 and err_exact < 1e-3
    plain = oracle.sp2(inst.F.toarray(), inst.lambda_min, inst.lambda_max, inst.n_occ, tau=tau)
    assert n_sq < plain.n_squares


def test_acc_block_sparse_empty_diagonal_block():
    """A stretched step of Alg. 4 squares a X~ + (1 - a) I: where a whole
    diagonal block of X~ is zero, the stored operand there is still
    (1 - a) I and must take part in the products. Block-diagonal F
    (N = 256, eight 32 x 32 blocks) whose last block is lambda_max I, so X~_0
    and X~_1 are zero there and step 2 (p = 1, a = 1.69) is stretched. GPU
    (BSR FP32, tau = 1e-5) against the FP64 oracle with the same truncation:
    D, the polynomials, and the error history while it is well above the
    FP32 level."""
    import scipy.sparse as sps
    import torch
    import paper_1507_02087_amd as sp2
    rng = np.random.default_rng(91)
    n, bs, tau = 256, 32, 1e-5
    F = np.zeros((n, n))
    for b in range(8):
        sl = slice(b * bs, (b + 1) * bs)
        if b == 7:
            F[sl, sl] = np.eye(bs)
        else:
            ev = np.concatenate([rng.uniform(-1.0, -0.1, 16), rng.uniform(0.1, 1.0, 16)])
            Q, _ = np.linalg.qr(rng.standard_normal((bs, bs)))
            F[sl, sl] = (Q * ev) @ Q.T
    F = (F + F.T) / 2
    lam = np.linalg.eigvalsh(F)
    n_occ = 7 * 16
    b = (float(lam[n_occ - 1]),) * 2 + (float(lam[n_occ]),) * 2
    sched = oracle.acc_schedule(-1.0, 1.0, *b)
    # the case is covered: step 2 is a stretched p = 1 step
    assert sched.p[2] == 1 and sched.alpha[2] > 1.1
    ref = oracle.sp2_acc(F, -1.0, 1.0, sched, tau=tau)
    assert ref.status == Status.OK
    rp, ci, bl = to_bsr_blocks(sps.csr_matrix(F), 32)
    assert ci.size == 8
    ctx = sp2.BsrContext(0)
    try:
        ctx.init_bsr(n, torch.from_numpy(rp).cuda(), torch.from_numpy(ci).cuda(),
                     torch.from_numpy(np.ascontiguousarray(bl)).cuda(), -1.0, 1.0, n_occ,
                     trunc_tau=tau)
        ctx.set_homo_lumo(*b)
        print_case("bsr acc, zero diagonal block under a stretch")
        st = ctx.run()
        D = ctx.get_density(as_fp64=True).cpu().numpy()
        n_it, _, _ = ctx.get_info()
        h = ctx.get_history()
    finally:
        ctx.close()
    assert st == sp2.OK
    assert h["p"][1:n_it + 1] == sched.p[1:n_it + 1]
    err = np.linalg.norm(D - ref.X) / math.sqrt(n_occ)
    worst = 0.0
    for k, (a, r) in enumerate(zip(h["v"], ref.v)):
        if r > 1e-2:
            worst = max(worst, abs(a - r) / r)
            assert abs(a - r) <= 1e-4 * r, (k, a, r)
    # the stop comes when the error stagnates at the working precision: the
    # oracle with FP32 storage and products stops where the GPU does (the
    # FP64 one two steps later, at its own rounding level)
    ref32 = oracle.sp2_acc(F, -1.0, 1.0, sched, tau=tau, working="fp32")
    print(f"  n_gpu={n_it} n_oracle={ref.n} (fp32 working: {ref32.n}) err={err:.2e} "
          f"worst history dev {worst:.2e}", flush=True)
    assert err < 1e-5
    assert abs(n_it - ref32.n) <= 1
