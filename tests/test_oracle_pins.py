"""Pins of the FP64 oracle against facts the paper and mathematics fix.

None of these tests re-types the oracle's formulas: each one checks the
oracle against a value the paper prints, a closed form reached a different
way (the scalar recursion on known eigenvalues), an exact special case
(diagonal inputs), brute force, or an invariant of the exact density matrix.
"""
import json
import math
import os

import numpy as np
import pytest

import oracle
from oracle import sp2, Status
from workloads import (config_small, dense_instance, diagonal_instance,
                       e5_instance, symmetric_gaussian_perturbation)

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _gold(name):
    with open(os.path.join(GOLD, name)) as fh:
        return json.load(fh)


# ------------------------------------------------------------------ constants
def _brute_max(fun, lo=1e-6, hi=1 - 1e-6, n=2_000_001):
    x = np.linspace(lo, hi, n)
    y = fun(x)
    i = int(np.argmax(y))
    # refine around the grid maximum by golden-section search
    a, b = x[max(i - 2, 0)], x[min(i + 2, n - 1)]
    g = (math.sqrt(5) - 1) / 2
    for _ in range(200):
        c, d = b - g * (b - a), a + g * (b - a)
        if fun(np.array([c]))[0] > fun(np.array([d]))[0]:
            b = d
        else:
            a = c
    xm = 0.5 * (a + b)
    return float(fun(np.array([xm]))[0]), xm


def _g_two_step(outer, inner):
    # g(x) = (f - f^2)/(x - x^2)^2 with f the composition, written out here
    # from the polynomial definitions x^2 and 2x - x^2 of sec. 4.
    def fun(x):
        y = inner(x)
        f = outer(y)
        return (f - f * f) / (x - x * x) ** 2
    return fun


SQ = lambda x: x * x                       # noqa: E731
TWO = lambda x: 2 * x - x * x              # noqa: E731


def test_c_sp2_matches_paper_and_brute_force():
    gold = _gold("paper_constants.json")
    assert round(oracle.C_SP2, gold["C2_sp_printed_digits"]) == gold["C2_sp_printed"]
    m12, x12 = _brute_max(_g_two_step(SQ, TWO))      # p1(p2(x))
    m21, x21 = _brute_max(_g_two_step(TWO, SQ))      # p2(p1(x))
    assert abs(m12 - oracle.C_SP2) < 1e-12
    assert abs(m21 - oracle.C_SP2) < 1e-12
    # the two compositions are mirror images: maxima at x* and 1 - x*
    assert abs(x12 + x21 - 1.0) < 1e-6
    assert oracle.Q_TILDE == gold["q_tilde"]


def test_two_step_limits_at_end_points():
    # exact rational arithmetic avoids the cancellation of 1 - x near x = 1
    from fractions import Fraction
    gold = _gold("paper_constants.json")
    e = Fraction(1, 10**8)

    def g(outer, inner, x):
        f = outer(inner(x))
        return (f - f * f) / (x - x * x) ** 2

    assert abs(float(g(TWO, SQ, e)) - gold["p21_limit_at_0"]) < 1e-6
    assert abs(float(g(SQ, TWO, 1 - e)) - gold["p12_limit_at_1"]) < 1e-6
    assert abs(float(g(TWO, SQ, 1 - e)) - gold["p21_limit_at_1"]) < 1e-6
    assert abs(float(g(SQ, TWO, e)) - gold["p12_limit_at_0"]) < 1e-6


def test_theorem1_g_ratio_mcweeny():
    gold = _gold("paper_constants.json")
    pmw = lambda x: 3 * x * x - 2 * x ** 3          # noqa: E731
    m, xm = _brute_max(lambda x: oracle.g_ratio(pmw, x))
    assert abs(m - gold["mcweeny_C"]) < 1e-10 and abs(xm - 0.5) < 1e-6
    assert abs(oracle.g_ratio(pmw, 1e-7) - gold["mcweeny_limit_at_ends"]) < 1e-5


def test_single_sp2_polynomials_have_no_limit():
    # sec. 4: g for x^2 alone is unbounded near 1, for 2x - x^2 near 0
    assert oracle.g_ratio(oracle.p_sp1, 1 - 1e-9) > 1e6
    assert oracle.g_ratio(oracle.p_sp2, 1e-9) > 1e6


# ------------------------------------------------------------------ f0
def test_f0_spectrum_closed_form():
    inst = dense_instance(96, 40, -3.0, 2.0, 0.3, seed=5)
    X0 = oracle.f0(inst.F, inst.lambda_min, inst.lambda_max)
    ev = np.sort(np.linalg.eigvalsh(X0))
    want = np.sort((inst.lambda_max - inst.lam) / (inst.lambda_max - inst.lambda_min))
    assert np.max(np.abs(ev - want)) < 1e-13
    t1 = (96 * inst.lambda_max - np.trace(inst.F)) / (inst.lambda_max - inst.lambda_min)
    assert abs(np.trace(X0) - t1) < 1e-12


# ------------------------------------------------------------------ images
def scalar_sp2(x0, n_occ, steps):
    """Eigenvalue-domain SP2 (Remark after Theorem 1): the iterates are
    Q diag(x) Q^T, so traces and errors follow from the eigenvalues alone."""
    xs, ps = [x0.copy()], [-1]
    x = x0.copy()
    for _ in range(steps):
        p = 1 if x.sum() > n_occ else 0   # Alg. 2 trace test
        x = x * x if p == 1 else 2 * x - x * x
        xs.append(x.copy())
        ps.append(p)
    return xs, ps


def test_iterates_are_polynomial_images_of_eigenvalues():
    inst = dense_instance(160, 70, -1.0, 1.5, 0.2, seed=21)
    steps = 9   # well before stagnation for this gap
    res = sp2(inst.F, inst.lambda_min, inst.lambda_max, inst.n_occ, max_iter=steps)
    assert res.status == Status.NOT_CONVERGED and res.n == steps
    x0 = (inst.lambda_max - inst.lam) / (inst.lambda_max - inst.lambda_min)
    xs, ps = scalar_sp2(x0, inst.n_occ, steps)
    assert res.p == ps
    Qt = inst.Q
    for k in range(steps + 1):
        if k < steps:
            vk = math.sqrt(float(np.sum((xs[k] - xs[k] ** 2) ** 2)))
            assert abs(res.v[k] - vk) <= 1e-10 * vk + 1e-13
        assert abs(res.t1[k] - xs[k].sum()) < 1e-10
        assert abs(res.t2[k] - (xs[k] ** 2).sum()) < 1e-10
    M = Qt.T @ res.X @ Qt
    assert np.max(np.abs(M - np.diag(xs[steps]))) < 1e-11


def test_diagonal_input_is_bit_exact():
    rng = np.random.default_rng(3)
    d = np.concatenate([rng.uniform(-1, -0.05, 30), rng.uniform(0.05, 1, 34)])
    inst = diagonal_instance(d, 30, -1.0, 1.0, perm_seed=9)
    steps = 12
    res = sp2(inst.F, -1.0, 1.0, 30, max_iter=steps)
    x0 = (1.0 - d) / 2.0
    x = x0.copy()
    perm = np.random.default_rng(9).permutation(64)
    for i in range(1, steps + 1):
        # the oracle's branch at step i used its own traces; replay them
        x = x * x if res.p[i] == 1 else 2.0 * x - x * x
    want = np.zeros((64, 64))
    want[perm, perm] = x
    assert np.array_equal(res.X, want)


def test_literal_and_nearest_branch_agree_inside_unit_interval():
    rng = np.random.default_rng(0)
    for _ in range(20000):
        n = int(rng.integers(1, 50))
        x = rng.uniform(0, 1, n)
        n_occ = int(rng.integers(0, n + 1))
        t1, t2 = x.sum(), (x * x).sum()
        assert oracle.choose_polynomial(t1, t2, n_occ, "nearest") == \
            oracle.choose_polynomial(t1, t2, n_occ, "literal")
    # a tie goes to 2x - x^2, as the strict '>' does
    assert oracle.choose_polynomial(5.0, 4.0, 5, "nearest") == 0
    assert oracle.choose_polynomial(5.0, 4.0, 5, "literal") == 0


# ------------------------------------------------------------------ stop logic
def test_stop_needs_alternation_and_low_order():
    C = oracle.C_SP2
    v = [0.5, 0.4, 1e-3, 0.3, C * 1e-6 * 0.5]
    p = [-1, 0, 1, 1, 0]
    # k = 4: p4 != p3, r = log(v4/C)/log(v2) = log(0.5e-6)/log(1e-3) > 2 -> no stop
    assert not oracle.stop_fires(v, p, 4)
    v2 = list(v)
    v2[4] = C * 1e-5            # r = 5/3 < 1.8 -> stop
    assert oracle.stop_fires(v2, p, 4)
    p2 = list(p)
    p2[4] = 1                   # no alternation -> no stop
    assert not oracle.stop_fires(v2, p2, 4)
    assert not oracle.stop_fires(v2, p, 1)       # k < 2
    v3 = list(v2)
    v3[2] = 1.5                 # v_{k-2} >= 1: the order test is skipped
    assert not oracle.stop_fires(v3, p, 4)


def test_exact_arithmetic_order_never_below_two():
    # Theorem 1 with the composed SP2 polynomials: in exact arithmetic the
    # spectral-norm order over two alternating steps is >= 2. Check it on the
    # scalar recursion for many random spectra, away from rounding.
    rng = np.random.default_rng(11)
    for trial in range(200):
        n = int(rng.integers(2, 40))
        x = np.sort(rng.uniform(0, 1, n))
        n_occ = int(rng.integers(1, n))
        xs, ps = scalar_sp2(x, n_occ, 30)
        e = [float(np.max(xk - xk * xk)) for xk in xs]
        for k in range(2, len(xs)):
            if ps[k] != ps[k - 1] and 1e-6 < e[k - 2] < 1 and e[k] > 1e-12:
                r = math.log(e[k] / oracle.C_SP2) / math.log(e[k - 2])
                assert r >= 2.0 - 1e-9, (trial, k, r)


# ------------------------------------------------------------------ worked example
@pytest.mark.parametrize("norm,key", [("fro", "stop_iteration_frobenius"),
                                      ("spectral", "stop_iteration_spectral")])
def test_paper_worked_example_stop_iteration(norm, key):
    gold = _gold("paper_e5_stop.json")
    inst = e5_instance(seed=7)
    assert inst.n == gold["n"] and inst.n_occ == gold["n_occ"]
    rng = np.random.default_rng(107)
    pert = lambda i, X: symmetric_gaussian_perturbation(  # noqa: E731
        X.shape[0], gold["perturbation_spectral_norm"], rng)
    res = sp2(inst.F, inst.lambda_min, inst.lambda_max, inst.n_occ,
              norm=norm, perturb=pert)
    assert res.status == Status.OK
    assert res.n + 1 == gold[key]
    assert res.n_squares == gold[key]


# ------------------------------------------------------------------ final D
def test_final_density_invariants_small_config():
    inst = config_small()
    res = sp2(inst.F, inst.lambda_min, inst.lambda_max, inst.n_occ)
    assert res.status == Status.OK
    D = res.X
    D_exact = oracle.density_from_eigenvectors(inst.Q, inst.n_occ)
    assert np.linalg.norm(D - D_exact) < 1e-11 * math.sqrt(inst.n_occ)
    assert abs(np.trace(D) - inst.n_occ) < 1e-9
    assert np.linalg.norm(D - D @ D) < 1e-11
    assert np.linalg.norm(inst.F @ D - D @ inst.F) / np.linalg.norm(inst.F) < 1e-11
    D_eigh = oracle.density_from_eigh(inst.F, inst.n_occ)
    assert np.linalg.norm(D_eigh - D_exact) < 1e-10
    # no premature stop: the returned error is near the smallest seen
    assert res.v[res.n] <= 10 * min(res.v)
    # stop came at an alternation with a low observed order
    assert res.p[res.n] != res.p[res.n - 1]
    assert res.r[res.n] < oracle.Q_TILDE


def test_reduced_precision_modes_stop_and_stay_close():
    inst = dense_instance(256, 128, -1.0, 1.0, 0.1, seed=44)
    ref = sp2(inst.F, -1.0, 1.0, 128)
    D_exact = oracle.density_from_eigenvectors(inst.Q, 128)
    for working, tol in (("fp32", 2e-5), ("bf16x3", 2e-4)):
        res = sp2(inst.F, -1.0, 1.0, 128, working=working)
        assert res.status == Status.OK
        err = np.linalg.norm(res.X - D_exact) / math.sqrt(128)
        assert err < tol, (working, err)
        assert res.n <= ref.n + 2


def test_bf16_rounding_matches_torch():
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(1)
    a = (rng.standard_normal(100000) * 10.0 ** rng.uniform(-6, 3, 100000)).astype(np.float32)
    # include exact ties: low 16 bits == 0x8000
    ties = (rng.integers(0, 2**31, 1000, dtype=np.uint32) & 0xFFFF0000) | 0x8000
    a = np.concatenate([a, ties.view(np.float32)])
    a = a[np.isfinite(a)]
    from oracle.sp2 import _round_bf16
    ours = _round_bf16(a)
    want = torch.from_numpy(a).to(torch.bfloat16).to(torch.float32).numpy()
    assert np.array_equal(ours, want)


# ------------------------------------------------------------------ degenerate
def test_degenerate_occupations_and_bad_bounds():
    inst = dense_instance(40, 20, -1.0, 1.0, 0.2, seed=1)
    r0 = sp2(inst.F, -1.0, 1.0, 0)
    assert r0.status == Status.OK and r0.n == 0 and not r0.X.any()
    rN = sp2(inst.F, -1.0, 1.0, 40)
    assert rN.status == Status.OK and np.array_equal(rN.X, np.eye(40))
    assert sp2(inst.F, 1.0, 1.0, 20).status == Status.INVALID_ARG
    assert sp2(inst.F, 1.0, -1.0, 20).status == Status.INVALID_ARG
    assert sp2(inst.F, -1.0, 1.0, 41).status == Status.INVALID_ARG
    assert sp2(inst.F, -1.0, 1.0, -1).status == Status.INVALID_ARG
    Fn = inst.F.copy()
    Fn[3, 5] = Fn[5, 3] = np.nan
    assert sp2(Fn, -1.0, 1.0, 20).status == Status.DIVERGED


def test_bounds_not_enclosing_spectrum_diverge():
    inst = dense_instance(64, 32, -1.0, 1.0, 0.2, seed=2)
    # lambda_max far below the true maximum: X_0 has eigenvalues near -199,
    # which both polynomials blow up
    res = sp2(inst.F, -1.0, -0.99, 32)
    assert res.status == Status.DIVERGED
    assert res.n <= 12


def test_exactly_idempotent_input_stops_at_zero():
    d = np.array([0.0] * 5 + [1.0] * 7)
    inst = diagonal_instance(d, 5, 0.0, 1.0)
    res = sp2(inst.F, 0.0, 1.0, 5)
    assert res.status == Status.OK and res.n == 0 and res.v == [0.0]


def test_truncation_threshold_semantics():
    X = np.array([[1e-7, -2e-6], [-2e-6, 1e-6]])
    Y = oracle.truncate(X, 1e-6)
    assert Y[0, 0] == 0.0 and Y[1, 1] == 1e-6 and Y[0, 1] == -2e-6
    assert oracle.truncate(X, 0.0) is X
