"""Pins of the McWeeny / McW-ACC oracle against sec. 3 of the paper: the
constant C = 4 and the closed form behind it, the fold that defines the
stretch, the accelerated constant and its limit formula, the Frobenius
counterexample 2/sqrt(5), the K-ratio inequality of the regular expansion,
and whole runs against the scalar eigenvalue recursion and the exact D."""
import math

import numpy as np
import pytest

import oracle
from oracle.mcweeny import (C_MW, f0_mw, mcweeny, mw_gamma, mwa_alpha, p_mw, p_mwa)
from workloads import config_small, diagonal_instance


def _g(f, x):
    fx = f(x)
    return (fx - fx * fx) / (x - x * x) ** 2


def test_constant_and_closed_form():
    """(p_mw - p_mw^2)/(x - x^2)^2 = 3 + 4x - 4x^2 on (0, 1); its limits at
    0 and 1 are 3 and its maximum, C_2^mw, is 4 at x = 0.5."""
    # away from the end points, where p - p^2 and x - x^2 cancel
    x = np.linspace(0.01, 0.99, 20001)
    g = _g(p_mw, x)
    np.testing.assert_allclose(g, 3 + 4 * x - 4 * x * x, rtol=1e-10)
    assert g.max() == pytest.approx(4.0, abs=1e-12) and C_MW == 4.0
    assert x[np.argmax(g)] == pytest.approx(0.5, abs=1e-4)
    assert _g(p_mw, 1e-7) == pytest.approx(3.0, rel=1e-6)


def test_f0_spectrum():
    """f_0 maps the spectrum to (mu - lambda)/gamma + 0.5 in [0, 1]."""
    inst = config_small()
    mu = 0.5 * (inst.lam[inst.n_occ - 1] + inst.lam[inst.n_occ])
    X0 = f0_mw(inst.F, inst.lambda_min, inst.lambda_max, mu)
    g = mw_gamma(inst.lambda_min, inst.lambda_max, mu)
    ev = np.sort(np.linalg.eigvalsh(X0))
    ref = np.sort((mu - inst.lam) / g + 0.5)
    np.testing.assert_allclose(ev, ref, atol=1e-13)
    assert ev.min() >= -1e-13 and ev.max() <= 1 + 1e-13
    assert np.sum(ev > 0.5) == inst.n_occ


def test_stretch_folds_the_spectrum():
    """The stretch alpha(beta) makes p_mw take the same value at the image of
    0 and at the image of beta (the fold), so [0, beta] lands inside the
    image of [beta, 1 - beta]'s edge; alpha(0) = 1 and alpha(0.5) = sqrt(3)."""
    for beta in np.linspace(0.001, 0.499, 60):
        a = mwa_alpha(beta)
        assert p_mw(a * (0.0 - 0.5) + 0.5) == pytest.approx(p_mw(a * (beta - 0.5) + 0.5),
                                                            abs=1e-14)
        assert p_mwa(0.0, beta) == pytest.approx(p_mwa(beta, beta), abs=1e-14)
    assert mwa_alpha(0.0) == 1.0 and mwa_alpha(0.5) == pytest.approx(math.sqrt(3), rel=1e-15)


@pytest.mark.parametrize("beta", [0.05, 0.1, 0.3, 0.45])
def test_accelerated_constant(beta):
    """C_2^mwa = 4: g_1(x, beta) on [beta, 1 - beta] peaks at 4 at x = 0.5;
    g_2 on the outer intervals stays at or below g_1(beta, beta), whose
    value is the printed limit formula."""
    x = np.linspace(beta, 1 - beta, 40001)[1:-1]
    g1 = _g(lambda t: p_mwa(t, beta), x)
    assert g1.max() == pytest.approx(4.0, abs=1e-9)
    assert x[np.argmax(g1)] == pytest.approx(0.5, abs=1e-4)
    lim = 16 * (beta - 1.5) ** 2 * (beta - 0.75) ** 2 / ((beta - 1) ** 2 *
                                                          (4 * beta ** 2 - 6 * beta + 3) ** 3)
    assert _g(lambda t: p_mwa(t, beta), beta + 1e-9) == pytest.approx(lim, rel=1e-6)
    xo = np.concatenate([np.linspace(0, beta, 2001), np.linspace(1 - beta, 1, 2001)])
    fo = p_mwa(xo, beta)
    g2 = (fo - fo * fo) / (beta - beta * beta) ** 2
    assert g2.max() <= lim * (1 + 1e-9) and lim <= 4.0


def test_frobenius_counterexample():
    """sec. 3: for X = diag(0, 0, 0, beta, 1 - beta) the ratio that the
    Frobenius estimate needs to be >= 1 equals 2/sqrt(5) under McW-ACC."""
    for beta in (0.1, 0.3):
        lam = np.array([0.0, 0.0, 0.0, beta, 1 - beta])
        E = lam - lam * lam
        P = p_mwa(lam, beta)
        EP = P - P * P
        ratio = (np.linalg.norm(E) ** 2 * np.max(np.abs(EP))) / \
            (np.max(np.abs(E)) ** 2 * np.linalg.norm(EP))
        assert ratio == pytest.approx(2 / math.sqrt(5), rel=1e-12)


def test_regular_expansion_k_ratio():
    """sec. 3: for the regular expansion (||X - X^2||_F / ||X - X^2||_2)^2
    dominates the same ratio one step later, on random spectra in [0, 1]."""
    rng = np.random.default_rng(4)
    for _ in range(200):
        lam = rng.uniform(0, 1, rng.integers(2, 60))
        E = lam - lam * lam
        P = p_mw(lam)
        EP = P - P * P
        k0 = np.linalg.norm(E) / np.max(np.abs(E))
        k1 = np.linalg.norm(EP) / np.max(np.abs(EP))
        assert k0 ** 2 >= k1 * (1 - 1e-12)


@pytest.mark.parametrize("xi", [None, 0.1])
def test_diagonal_input_scalar_recursion(xi):
    """Diagonal F: every step equals the scalar recursion on its diagonal
    (bit for bit: each entry is one scalar polynomial evaluation in the same
    order), and the result is the 0/1 projector."""
    rng = np.random.default_rng(7)
    d = np.concatenate([rng.uniform(-1, -0.05, 30), rng.uniform(0.05, 1, 20)])
    d[0], d[1] = -0.05, 0.05
    inst = diagonal_instance(d, 30, -1.0, 1.0, perm_seed=None)
    res = mcweeny(inst.F, -1.0, 1.0, 0.0, xi=xi)
    assert res.status == oracle.Status.OK
    x = (0.0 - d) / mw_gamma(-1.0, 1.0, 0.0) + 0.5
    beta = 0.5 * (1 - xi / 2.0) if xi else 0.0
    for k in range(1, res.n + 1):
        a = res.p[k]
        on = bool(xi) and beta >= 0.01
        assert a == (mwa_alpha(beta) if on else 1.0)
        xs = a * (x - 0.5) + 0.5 if on else x
        s = xs * xs
        x = 3.0 * s - 2.0 * (xs * s)
        if xi and beta >= 0.01:
            beta = p_mw(a * (beta - 0.5) + 0.5)
    assert np.array_equal(np.diag(res.X), x)
    assert np.max(np.abs(np.diag(res.X) - (d < 0))) < 1e-14


def test_dense_runs():
    """N = 512 (gap 0.1): McWeeny and McW-ACC reach the exact D; the stop fires
    with r < 1.8; the error history equals the eigenvalue-domain images while
    far above rounding; the stretch takes fewer steps."""
    inst = config_small()
    D = oracle.density_from_eigenvectors(inst.Q, inst.n_occ)
    h, l = inst.lam[inst.n_occ - 1], inst.lam[inst.n_occ]
    mu = 0.5 * (h + l)
    g = mw_gamma(inst.lambda_min, inst.lambda_max, mu)
    out = {}
    for xi in (None, l - h):
        r = mcweeny(inst.F, inst.lambda_min, inst.lambda_max, mu, xi=xi)
        assert r.status == oracle.Status.OK
        assert np.linalg.norm(r.X - D) < 1e-12 * math.sqrt(inst.n_occ)
        assert r.r[r.n] < 1.8
        x = (mu - inst.lam) / g + 0.5
        for k in range(r.n + 1):
            if k:
                a = r.p[k]
                x = p_mw(a * (x - 0.5) + 0.5)
            exact = math.sqrt(float(np.sum((x - x * x) ** 2)))
            if exact > 1e-8:
                assert r.v[k] == pytest.approx(exact, rel=1e-9)
        out[xi] = r.n
    assert out[l - h] < out[None]
