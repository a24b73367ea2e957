"""GPU parity of the dense SP2 path against the FP64 CPU oracle.

Every case is computed by the HIP library through its C ABI (via the ctypes
binding) and by the oracle on the same seeded input.
"""
import math

import numpy as np
import pytest

import oracle
from oracle import Status
from workloads import dense_instance, diagonal_instance, config_small
from tests.gpu_helpers import square_bound, print_case

pytestmark = pytest.mark.gpu

PRECS = ("fp64", "fp32", "bf16x3")
# Frobenius tolerance on ||D_gpu - D_oracle||_F / sqrt(n_occ), per precision.
D_TOL = {"fp64": 1e-11, "fp32": 2e-5, "bf16x3": 2e-4}


def _run(F, inst, **kw):
    import torch
    import paper_1507_02087_amd as sp2
    Ft = torch.from_numpy(np.ascontiguousarray(F)).to("cuda:0")
    res = sp2.run_dense(Ft, inst.lambda_min, inst.lambda_max, inst.n_occ, **kw)
    torch.cuda.synchronize()
    return res


def _configs():
    """(precision, 1-based kernel configuration id) of every compiled
    configuration; read from the library when it is built."""
    try:
        import paper_1507_02087_amd as sp2
        return [(c["precision"], c["id"]) for c in sp2.kernel_configs()]
    except Exception:
        return [(p, 0) for p in PRECS]


CONFIGS = _configs()


@pytest.mark.parametrize("prec,cfg", CONFIGS)
@pytest.mark.parametrize("n", [64, 300])
@pytest.mark.parametrize("split", [0, 1])
def test_diagonal_input_bit_exact(prec, cfg, n, split):
    """Diagonal (permuted) F: every entry of every square is one product plus
    exact zeros, so the GPU iterates equal the oracle's (same working
    precision) bit for bit, for every kernel configuration, with and without
    the split of tail tiles."""
    rng = np.random.default_rng(n)
    n_occ = n // 2
    d = np.concatenate([rng.uniform(-1, -0.05, n_occ), rng.uniform(0.05, 1, n - n_occ)])
    inst = diagonal_instance(d, n_occ, -1.0, 1.0, perm_seed=n + 1)
    steps = 10
    print_case(f"diagonal n={n} prec={prec} cfg={cfg} split={split} steps={steps}")
    res = _run(inst.F, inst, precision=prec, max_iter=steps, kernel_config=cfg,
               tail_split=split)
    ref = oracle.sp2(inst.F, -1.0, 1.0, n_occ, max_iter=steps, working=prec)
    assert res.status_name == "NOT_CONVERGED" and ref.status == Status.NOT_CONVERGED
    assert res.n == steps and res.p[:steps + 1] == ref.p
    D = res.D.cpu().numpy()
    assert np.array_equal(D, ref.X), float(np.max(np.abs(D - ref.X)))
    np.testing.assert_allclose(res.v, ref.v, rtol=1e-12, atol=0)


@pytest.mark.parametrize("prec,cfg", CONFIGS)
@pytest.mark.parametrize("n", [2, 31, 129, 300, 513])
@pytest.mark.parametrize("split", [0, 1, 3])
def test_one_square_elementwise(prec, cfg, n, split):
    """X~_1 after one fused square, element by element, against the oracle's
    step in the same working precision, within the worst-case rounding bound
    of two different summation orders."""
    n_occ = n // 2
    # asymmetric bounds keep Tr X_0 away from n_occ, so the first polynomial
    # choice is decided by the traces and not by rounding
    inst = dense_instance(n, n_occ, -1.0, 1.3, 0.1, seed=1000 + n)
    print_case(f"one square n={n} prec={prec} cfg={cfg} split={split}")
    res = _run(inst.F, inst, precision=prec, max_iter=1, kernel_config=cfg,
               tail_split=split)
    ref = oracle.sp2(inst.F, inst.lambda_min, inst.lambda_max, n_occ,
                     max_iter=1, working=prec)
    assert res.status_name == "NOT_CONVERGED" and res.n == 1
    assert res.p[1] == ref.p[1]
    D = res.D.cpu().numpy()
    tol = square_bound(n, prec) + (2.0 ** -22 if prec != "fp64" else 0.0)
    err = float(np.max(np.abs(D - ref.X)))
    assert err <= tol, (err, tol)
    assert np.array_equal(D, D.T)
    # traces of X~_1 inherit the element bound: |dTr| <= n tol,
    # |d sum x^2| <= sum |a - b||a + b| <= tol (2 sum|x| + n^2 tol)
    assert abs(res.t1[1] - ref.t1[1]) <= n * tol + 1e-12
    assert abs(res.t2[1] - ref.t2[1]) <= tol * (2 * np.abs(ref.X).sum() + n * n * tol) + 1e-12
    # v_0 = ||X~_0 - S||_F: the same element bound on S, summed in quadrature
    assert abs(res.v[0] - ref.v[0]) <= n * square_bound(n, prec) + 1e-6 * ref.v[0]


@pytest.mark.parametrize("prec", PRECS)
def test_one_square_padded_row_stride(prec):
    """N = 2048: the library stores the iterate with a row stride longer
    than the padded width (2048 is a multiple of 512), so this covers the
    affine start, the square, its transposed writes and the copy-out at that
    stride: X~_1 element by element against the oracle's step, symmetric,
    and the traces."""
    n = 2048
    n_occ = n // 2
    inst = dense_instance(n, n_occ, -1.0, 1.3, 0.1, seed=2048)
    print_case(f"one square padded stride n={n} prec={prec}")
    res = _run(inst.F, inst, precision=prec, max_iter=1)
    ref = oracle.sp2(inst.F, inst.lambda_min, inst.lambda_max, n_occ,
                     max_iter=1, working=prec)
    assert res.status_name == "NOT_CONVERGED" and res.n == 1
    assert res.p[1] == ref.p[1]
    D = res.D.cpu().numpy()
    tol = square_bound(n, prec) + (2.0 ** -22 if prec != "fp64" else 0.0)
    err = float(np.max(np.abs(D - ref.X)))
    assert err <= tol, (err, tol)
    assert np.array_equal(D, D.T)
    assert abs(res.t1[1] - ref.t1[1]) <= n * tol + 1e-12


@pytest.mark.parametrize("prec", PRECS)
def test_full_run_small_config(prec):
    """Dense N=512, gap 0.1, n_occ 256: the stop is detected automatically
    and D matches the FP64 oracle within the stated Frobenius tolerance."""
    inst = config_small()
    print_case(f"full run N=512 prec={prec}")
    ref = oracle.sp2(inst.F, inst.lambda_min, inst.lambda_max, inst.n_occ)
    res = _run(inst.F, inst, precision=prec)
    assert res.status_name == "OK", res.status_name
    D = res.D.cpu().numpy()
    err = np.linalg.norm(D - ref.X) / math.sqrt(inst.n_occ)
    print_case(f"  n_gpu={res.n} n_oracle={ref.n} err={err:.3e} ms={res.run_ms:.3f}")
    assert err < D_TOL[prec]
    assert abs(np.trace(D) - inst.n_occ) < (1e-9 if prec == "fp64" else 1e-3)
    if prec == "fp64":
        assert abs(res.n - ref.n) <= 6
    else:
        assert res.n <= ref.n + 2
    # the history matches the oracle while the error is well above rounding:
    # relative deviation within 100 k u_eff after k steps, u_eff being the
    # working precision's unit roundoff (bf16x3 carries 16 significant bits)
    u_eff = {"fp64": 2.0 ** -53, "fp32": 2.0 ** -24, "bf16x3": 2.0 ** -16}[prec]
    for k, (a, b) in enumerate(zip(res.v, ref.v)):
        if b > 1e-3:
            assert abs(a - b) <= 100 * (k + 1) * u_eff * b + 1e-13, (k, a, b)
    # stop at an alternation with a low observed order
    assert res.p[res.n] != res.p[res.n - 1] and res.r[res.n] < 1.8


@pytest.mark.parametrize("prec", PRECS)
def test_ragged_tiles_full_run(prec):
    inst = dense_instance(333, 170, -1.3, 0.9, 0.12, seed=333)
    print_case(f"full run N=333 prec={prec}")
    ref = oracle.sp2(inst.F, inst.lambda_min, inst.lambda_max, inst.n_occ)
    res = _run(inst.F, inst, precision=prec)
    assert res.status_name == "OK"
    D = res.D.cpu().numpy()
    err = np.linalg.norm(D - ref.X) / math.sqrt(inst.n_occ)
    assert err < D_TOL[prec], err
    D_exact = oracle.density_from_eigenvectors(inst.Q, inst.n_occ)
    assert np.linalg.norm(D - D_exact) / math.sqrt(inst.n_occ) < D_TOL[prec]


def test_trivial_occupations_and_idempotent_input():
    import torch
    import paper_1507_02087_amd as sp2
    inst = dense_instance(200, 100, -1.0, 1.0, 0.1, seed=5)
    F = torch.from_numpy(inst.F).cuda()
    r0 = sp2.run_dense(F, -1.0, 1.0, 0)
    assert r0.status == sp2.OK and r0.n == 0 and r0.n_squares == 0
    assert float(r0.D.abs().max()) == 0.0
    rN = sp2.run_dense(F, -1.0, 1.0, 200, precision="fp32")
    assert rN.status == sp2.OK and torch.equal(rN.D.cpu(), torch.eye(200, dtype=torch.float64))
    d = np.array([0.0] * 70 + [1.0] * 50)
    di = diagonal_instance(d, 70, 0.0, 1.0, perm_seed=3)
    r = sp2.run_dense(torch.from_numpy(di.F).cuda(), 0.0, 1.0, 70)
    assert r.status == sp2.OK and r.n == 0 and r.v == [0.0]


@pytest.mark.parametrize("prec", PRECS)
def test_smallest_inputs(prec):
    """N = 1 admits only n_occ = 0 or 1, where D is 0 or 1 with no square
    computed; N = 0 is rejected as an invalid argument."""
    import torch
    import paper_1507_02087_amd as sp2
    F = torch.tensor([[0.3]], dtype=torch.float64, device="cuda")
    for n_occ, d in ((0, 0.0), (1, 1.0)):
        r = sp2.run_dense(F, -1.0, 1.0, n_occ, precision=prec)
        assert r.status == sp2.OK and r.n == 0 and r.n_squares == 0
        assert r.D.shape == (1, 1) and float(r.D[0, 0]) == d
    with pytest.raises(sp2.SP2Error) as e:
        sp2.run_dense(torch.zeros((0, 0), dtype=torch.float64, device="cuda"),
                      -1.0, 1.0, 0, precision=prec)
    assert e.value.status == sp2.INVALID_ARG


def test_invalid_arguments_raise():
    import torch
    import paper_1507_02087_amd as sp2
    F = torch.eye(8, dtype=torch.float64, device="cuda")
    for kw in (dict(lambda_min=1.0, lambda_max=1.0, n_occ=4),
               dict(lambda_min=0.0, lambda_max=1.0, n_occ=9),
               dict(lambda_min=0.0, lambda_max=float("inf"), n_occ=4)):
        with pytest.raises(sp2.SP2Error) as e:
            sp2.run_dense(F, **kw)
        assert e.value.status == sp2.INVALID_ARG
    with pytest.raises(sp2.SP2Error):
        sp2.run_dense(F, 0.0, 1.0, 4, max_iter=1000)
    with pytest.raises(sp2.SP2Error):
        sp2.run_dense(F, 0.0, 1.0, 4, kernel_config=999)
    fp32_cfg = next(c["id"] for c in sp2.kernel_configs() if c["precision"] == "fp32")
    with pytest.raises(sp2.SP2Error):   # configuration of another precision
        sp2.run_dense(F, 0.0, 1.0, 4, precision="fp64", kernel_config=fp32_cfg)


def test_divergence_and_nan_reported():
    import torch
    import paper_1507_02087_amd as sp2
    inst = dense_instance(64, 32, -1.0, 1.0, 0.2, seed=2)
    F = torch.from_numpy(inst.F).cuda()
    ref = oracle.sp2(inst.F, -1.0, -0.99, 32)
    r = sp2.run_dense(F, -1.0, -0.99, 32)
    assert r.status == sp2.DIVERGED and ref.status == Status.DIVERGED
    assert r.n == ref.n
    Fn = inst.F.copy()
    Fn[3, 5] = Fn[5, 3] = np.nan
    r = sp2.run_dense(torch.from_numpy(Fn).cuda(), -1.0, 1.0, 32)
    assert r.status == sp2.DIVERGED and r.n == 0


def test_literal_branch_rule_option():
    inst = dense_instance(256, 128, -1.0, 1.0, 0.1, seed=77)
    ref = oracle.sp2(inst.F, -1.0, 1.0, 128, branch="literal", max_iter=12)
    res = _run(inst.F, inst, branch="literal", max_iter=12)
    assert res.p == ref.p


def test_max_iter_not_converged_returns_last_iterate():
    inst = dense_instance(256, 128, -1.0, 1.0, 0.001, seed=8)
    ref = oracle.sp2(inst.F, -1.0, 1.0, 128, max_iter=5)
    res = _run(inst.F, inst, max_iter=5)
    assert res.status_name == "NOT_CONVERGED" and res.n == 5 and res.n_squares == 5
    assert np.max(np.abs(res.D.cpu().numpy() - ref.X)) < 1e-12


def test_runs_are_bitwise_reproducible():
    inst = dense_instance(400, 200, -1.0, 1.0, 0.05, seed=4)
    a = _run(inst.F, inst, precision="bf16x3")
    b = _run(inst.F, inst, precision="bf16x3")
    assert a.n == b.n and a.v == b.v
    import torch
    assert torch.equal(a.D, b.D)


def test_truncation_matches_oracle():
    inst = dense_instance(256, 128, -1.0, 1.0, 0.1, seed=12)
    tau = 1e-4
    ref = oracle.sp2(inst.F, -1.0, 1.0, 128, tau=tau, max_iter=6)
    res = _run(inst.F, inst, trunc_tau=tau, max_iter=6)
    D = res.D.cpu().numpy()
    # entries far from the threshold agree; zeros where the oracle removed
    far = np.abs(np.abs(ref.X) - tau) > 1e-9
    assert np.max(np.abs(D - ref.X)[far]) < 1e-11
    assert np.all(D[(ref.X == 0) & far] == 0)
