"""Pins of the SP2-ACC oracle (Alg. 3 schedule, Alg. 4 expansion) against
facts the paper and the mathematics fix: the fold that defines the stretch,
Theorem 2 and its proof, the scalar images of the homo/lumo bounds, the
efficiency figure behind delta = 0.01, exact projectors of diagonal inputs,
and the density matrix of constructed spectra."""
import math

import numpy as np
import pytest

import oracle
from oracle import acc_polynomial, acc_schedule, sp2_acc
from workloads import (config_small, dense_instance, diagonal_instance,
                       e5_instance, symmetric_gaussian_perturbation)


def _homo_lumo(inst):
    ev = np.linalg.eigvalsh(inst.F)
    return ev[inst.n_occ - 1], ev[inst.n_occ]


def _random_bounds(rng):
    lmin, lmax = -rng.uniform(0.5, 3.0), rng.uniform(0.5, 3.0)
    c = rng.uniform(lmin + 0.2 * (lmax - lmin), lmax - 0.2 * (lmax - lmin))
    gap = rng.uniform(1e-4, 0.3) * (lmax - lmin)
    homo_in, lumo_in = c - gap / 2, c + gap / 2
    homo_out = homo_in - rng.uniform(0.0, homo_in - lmin)
    lumo_out = lumo_in + rng.uniform(0.0, lmax - lumo_in)
    return lmin, lmax, homo_out, homo_in, lumo_in, lumo_out


def _max_run_after_first_alternation(p):
    seq = p[1:]
    first = next((i for i in range(1, len(seq)) if seq[i] != seq[i - 1]), None)
    if first is None:
        return 0
    run = best = 1
    for i in range(first + 1, len(seq)):
        run = run + 1 if seq[i] == seq[i - 1] else 1
        best = max(best, run)
    return best


def test_fold_defines_the_stretch():
    """Scale-and-fold (sec. 4): with alpha = 2/(2 - gamma_low), x^2-type step
    maps 0 and gamma_low to one value (the unoccupied part is folded back);
    with alpha = 2/(2 - beta_low), the 2x - x^2-type step maps 1 and
    1 - beta_low to one value. Both keep [0, 1] inside [0, 1]."""
    rng = np.random.default_rng(11)
    xs = np.linspace(0.0, 1.0, 1001)
    for _ in range(200):
        s = acc_schedule(*_random_bounds(rng))
        assert s is not None
        for i in range(1, s.n_max + 1):
            p, a = s.p[i], s.alpha[i]
            assert 1.0 <= a <= 2.0
            ys = acc_polynomial(p, a, xs)
            assert ys.min() >= -1e-15 and ys.max() <= 1.0 + 1e-15
            if p == 1:
                g = s.gamma_low[i - 1] if i < s.n_min - 1 else 0.0
                # compare the roots |(1 - a) + a x|, which are O(1) accurate
                assert abs(math.sqrt(acc_polynomial(1, a, 0.0))
                           - math.sqrt(acc_polynomial(1, a, g))) < 1e-14
            else:
                b = s.beta_low[i - 1] if i < s.n_min - 1 else 0.0
                assert abs(acc_polynomial(0, a, 1.0) - acc_polynomial(0, a, 1.0 - b)) < 1e-14


def test_stretch_one_is_plain_sp2():
    """At alpha = 1 the two Alg. 4 polynomials are x^2 and 2x - x^2."""
    xs = np.linspace(-0.5, 1.5, 41)
    assert np.array_equal(acc_polynomial(1, 1.0, xs), oracle.p_sp1(xs))
    assert np.allclose(acc_polynomial(0, 1.0, xs), oracle.p_sp2(xs), rtol=0, atol=1e-15)


def test_theorem2_proof_sequence():
    """Proof of Theorem 2: starting from beta = gamma without acceleration,
    p_1 = 1, then p_2 = p_3 = 0 and p_4 = 1."""
    # lambda in [-1, 1], homo = -1/2, lumo = 1/2: beta_0 = gamma_0 = 1/4 exactly
    s = acc_schedule(-1.0, 1.0, -0.5, -0.5, 0.5, 0.5, accelerate=False)
    assert s.beta_up[0] == s.gamma_up[0] == 0.25
    assert s.p[1:5] == [1, 0, 0, 1]
    # and the scalar values the proof writes out
    g0 = 0.25
    assert s.gamma_up[1] == pytest.approx(g0 ** 2, rel=1e-15)
    assert s.beta_up[1] == pytest.approx(2 * g0 - g0 ** 2, rel=1e-15)
    assert s.gamma_up[2] == pytest.approx(2 * g0 ** 2 - g0 ** 4, rel=1e-14)
    assert s.beta_up[2] == pytest.approx((2 * g0 - g0 ** 2) ** 2, rel=1e-14)
    assert s.gamma_up[3] == pytest.approx(4 * g0 ** 2 - 6 * g0 ** 4 + 4 * g0 ** 6 - g0 ** 8,
                                          rel=1e-13)
    assert s.beta_up[3] == pytest.approx((2 * g0 - g0 ** 2) ** 4, rel=1e-13)


def test_theorem2_runs_of_one_polynomial():
    """Theorem 2: without acceleration, after both polynomials have been used,
    at most two subsequent steps use the same one; with acceleration at most
    three (the remark after the theorem)."""
    rng = np.random.default_rng(5)
    for _ in range(300):
        b = _random_bounds(rng)
        s0 = acc_schedule(*b, accelerate=False)
        s1 = acc_schedule(*b, accelerate=True)
        assert _max_run_after_first_alternation(s0.p) <= 2
        assert _max_run_after_first_alternation(s1.p) <= 3


def test_schedule_tracks_scalar_images():
    """The upper bounds follow the images of the inner homo/lumo bounds under
    the chosen polynomials: gamma_up_i = f_i(...f_1(x_lumo)) and
    beta_up_i = 1 - f_i(...f_1(x_homo)), with x = (lambda_max - lambda)/width
    (the spectrum of X_0, Alg. 2)."""
    rng = np.random.default_rng(9)
    for _ in range(100):
        lmin, lmax, ho, hi, li, lo = _random_bounds(rng)
        s = acc_schedule(lmin, lmax, ho, hi, li, lo)
        xh = (lmax - hi) / (lmax - lmin)
        xl = (lmax - li) / (lmax - lmin)
        for i in range(1, s.n_max + 1):
            xh = acc_polynomial(s.p[i], s.alpha[i], xh)
            xl = acc_polynomial(s.p[i], s.alpha[i], xl)
            if s.gamma_up[i] > 1e-6:
                assert xl == pytest.approx(s.gamma_up[i], rel=1e-9)
            if s.beta_up[i] > 1e-6:
                assert 1.0 - xh == pytest.approx(s.beta_up[i], rel=1e-9)
        # n_max: both images idempotent to eps_M (R18), the last step alternates
        assert xh * (1 - xh) <= 4 * oracle.EPS_M and xl * (1 - xl) <= 4 * oracle.EPS_M
        assert s.p[s.n_max] != s.p[s.n_max - 1]


def test_switch_off_and_n_min():
    """Alg. 3: once both lower bounds are below delta the stretch is 1 and the
    stop is checked from n_min on; without acceleration n_min = 2 (table
    tab:water_start_check_puri, first SCF cycle)."""
    rng = np.random.default_rng(21)
    for _ in range(100):
        b = _random_bounds(rng)
        s = acc_schedule(*b)
        assert 2 <= s.n_min <= s.n_max
        assert all(a == 1.0 for a in s.alpha[s.n_min - 1:])
        s0 = acc_schedule(*b, accelerate=False)
        assert s0.n_min == 2 and all(a == 1.0 for a in s0.alpha[1:])


def test_delta_efficiency_figure():
    """Figure fig:acc_efficiency: below 0.01 the stretched fold reduces an
    unoccupied eigenvalue by less than 1 percent more than x^2 does."""
    for lam in np.geomspace(1e-8, 0.01, 50):
        a = 2.0 / (2.0 - lam)
        gain = abs(lam ** 2 - acc_polynomial(1, a, lam)) / abs(lam - lam ** 2)
        assert gain < 0.01
    lam = 0.1
    a = 2.0 / (2.0 - lam)
    assert abs(lam ** 2 - acc_polynomial(1, a, lam)) / abs(lam - lam ** 2) > 0.01


def test_invalid_bounds():
    """R21: overlapping or unordered homo/lumo intervals, bounds on the
    spectral bounds, non-finite values give no schedule."""
    assert acc_schedule(-1, 1, -0.1, 0.1, 0.0, 0.2) is None     # homo_in >= lumo_in
    assert acc_schedule(-1, 1, 0.0, -0.1, 0.1, 0.2) is None     # homo_out > homo_in
    assert acc_schedule(-1, 1, -0.2, -0.1, 0.1, 0.05) is None   # lumo_out < lumo_in
    assert acc_schedule(-1, 1, -1.0, -1.0, 0.1, 0.2) is None    # homo_in = lambda_min
    assert acc_schedule(-1, 1, -0.2, -0.1, 1.0, 1.0) is None    # lumo_in = lambda_max
    assert acc_schedule(-1, 1, -1.2, -0.1, 0.1, 0.2) is None    # homo_out < lambda_min
    assert acc_schedule(-1, 1, -0.2, -0.1, 0.1, math.nan) is None
    assert sp2_acc(np.eye(3), -1, 1, None).status == oracle.Status.INVALID_ARG


@pytest.mark.parametrize("accelerate", [True, False])
def test_diagonal_projector(accelerate):
    """Diagonal F with a known spectrum: X~_n is the exact 0/1 projector onto
    the n_occ lowest states, within rounding, reached by n <= n_max."""
    rng = np.random.default_rng(3)
    d = np.concatenate([rng.uniform(-1.0, -0.05, 40), rng.uniform(0.05, 1.0, 24)])
    d[0], d[1] = -0.05, 0.05
    inst = diagonal_instance(d, 40, -1.0, 1.0, perm_seed=1)
    s = acc_schedule(-1.0, 1.0, -0.05, -0.05, 0.05, 0.05, accelerate=accelerate)
    res = sp2_acc(inst.F, -1.0, 1.0, s)
    assert res.status == oracle.Status.OK and res.n <= s.n_max
    occ = np.diag(inst.F) < 0
    assert np.max(np.abs(np.diag(res.X) - occ)) < 1e-14
    assert np.max(np.abs(res.X - np.diag(np.diag(res.X)))) == 0.0


def test_dense_density_and_fewer_steps():
    """Dense N = 512 construction (gap 0.1 in [-1, 1]): SP2-ACC reaches the
    exact D of the construction with exact and with loose outer bounds, with
    fewer steps than the unaccelerated schedule and than Alg. 2."""
    inst = config_small()
    D = inst.Q[:, :inst.n_occ] @ inst.Q[:, :inst.n_occ].T
    homo, lumo = _homo_lumo(inst)
    tol = 1e-12 * math.sqrt(inst.n_occ)
    s = acc_schedule(inst.lambda_min, inst.lambda_max, homo, homo, lumo, lumo)
    r = sp2_acc(inst.F, inst.lambda_min, inst.lambda_max, s)
    assert r.status == oracle.Status.OK and np.linalg.norm(r.X - D) < tol
    loose = acc_schedule(inst.lambda_min, inst.lambda_max, homo - 0.3, homo, lumo, lumo + 0.3)
    rl = sp2_acc(inst.F, inst.lambda_min, inst.lambda_max, loose)
    assert rl.status == oracle.Status.OK and np.linalg.norm(rl.X - D) < tol
    s0 = acc_schedule(inst.lambda_min, inst.lambda_max, homo, homo, lumo, lumo, accelerate=False)
    r0 = sp2_acc(inst.F, inst.lambda_min, inst.lambda_max, s0)
    assert r0.status == oracle.Status.OK and np.linalg.norm(r0.X - D) < tol
    r2 = oracle.sp2(inst.F, inst.lambda_min, inst.lambda_max, inst.n_occ)
    assert r.n < rl.n <= r0.n < r2.n
    # v_k = ||X~_k - X~_k^2||_F from the eigenvalue images while far above rounding
    x = (inst.lambda_max - inst.lam) / (inst.lambda_max - inst.lambda_min)
    for k in range(0, r.n + 1):
        if k:
            x = acc_polynomial(r.p[k], s.alpha[k], x)
        exact = math.sqrt(float(np.sum((x - x * x) ** 2)))
        if exact > 1e-8:
            assert r.v[k] == pytest.approx(exact, rel=1e-9)


def test_e5_with_noise_stops_on_alternation():
    """The sec. 4.1 example (N = 1000, perturbation of spectral norm 1e-5 per
    step) with the Alg. 3 schedule: the stop fires on an alternation at some
    i >= n_min with r_i < 1.8, before n_max, and far fewer steps are needed
    with acceleration; without it the stop comes where Alg. 2 stops
    (29 Frobenius / 31 spectral matrix multiplications in the paper, i.e.
    n = 28 / 30)."""
    inst = e5_instance(seed=7)
    homo, lumo = _homo_lumo(inst)
    out = {}
    for acc in (True, False):
        s = acc_schedule(inst.lambda_min, inst.lambda_max, homo, homo, lumo, lumo,
                         accelerate=acc)
        for norm in ("fro", "spectral"):
            rng = np.random.default_rng(1)
            pert = lambda i, X: symmetric_gaussian_perturbation(X.shape[0], 1e-5, rng)  # noqa: E731
            r = sp2_acc(inst.F, inst.lambda_min, inst.lambda_max, s, norm=norm, perturb=pert)
            assert r.status == oracle.Status.OK
            assert s.n_min <= r.n < s.n_max
            assert r.p[r.n] != r.p[r.n - 1] and r.r[r.n] < oracle.Q_TILDE
            out[(acc, norm)] = r.n
    assert out[(False, "fro")] == 28 and out[(False, "spectral")] == 30
    assert out[(True, "fro")] <= 18 and out[(True, "spectral")] <= 18


def test_fp32_working_precision():
    """FP32 squares and storage: same D to FP32 accuracy, stop not later than
    n_max."""
    inst = dense_instance(256, 128, -1.0, 1.0, 0.05, 17)
    D = inst.Q[:, :inst.n_occ] @ inst.Q[:, :inst.n_occ].T
    homo, lumo = _homo_lumo(inst)
    s = acc_schedule(inst.lambda_min, inst.lambda_max, homo, homo, lumo, lumo)
    r = sp2_acc(inst.F, inst.lambda_min, inst.lambda_max, s, working="fp32")
    assert r.status == oracle.Status.OK and r.n <= s.n_max
    assert np.linalg.norm(r.X - D) < 2e-5 * math.sqrt(inst.n_occ)
