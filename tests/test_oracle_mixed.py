"""Pins of the oracle's mixed norm (sec. 2: spectral norm of the matrix of
block Frobenius norms) and of the stop driven by it."""
import math

import numpy as np
import pytest

import oracle
from workloads import config_small, e5_instance, symmetric_gaussian_perturbation


def _sym(rng, n):
    A = rng.standard_normal((n, n))
    return A + A.T


def test_limits_of_the_block_size():
    """One block: the Frobenius norm. Blocks of one element: the spectral
    norm of |A|; for a diagonal A that is the spectral norm of A."""
    rng = np.random.default_rng(1)
    for n in (1, 7, 50):
        A = _sym(rng, n)
        assert oracle.mixed_norm(A, n) == pytest.approx(np.linalg.norm(A), rel=1e-14)
        assert oracle.mixed_norm(A, n + 13) == pytest.approx(np.linalg.norm(A), rel=1e-14)
        assert oracle.mixed_norm(A, 1) == pytest.approx(np.linalg.norm(np.abs(A), 2), rel=1e-12)
        d = rng.standard_normal(n)
        assert oracle.mixed_norm(np.diag(d), 1) == pytest.approx(np.max(np.abs(d)), rel=1e-14)


def test_between_spectral_and_frobenius():
    """e <= m <= v for every block size (sec. 2)."""
    rng = np.random.default_rng(2)
    for n in (5, 33, 64, 100):
        A = _sym(rng, n)
        e, v = np.linalg.norm(A, 2), np.linalg.norm(A)
        for b in (1, 2, 3, 8, 32, n):
            m = oracle.mixed_norm(A, b)
            assert e * (1 - 1e-13) <= m <= v * (1 + 1e-13), (n, b, e, m, v)


def test_block_diagonal_and_block_permutation():
    """Aligned block-diagonal A: the matrix of block norms is diagonal, so m
    is the largest block Frobenius norm; permuting whole blocks leaves m
    unchanged; zero padding leaves m unchanged."""
    rng = np.random.default_rng(3)
    b, nb = 8, 6
    blocks = [_sym(rng, b) * rng.uniform(0.1, 2.0) for _ in range(nb)]
    A = np.zeros((b * nb, b * nb))
    for k, B in enumerate(blocks):
        A[k * b:(k + 1) * b, k * b:(k + 1) * b] = B
    assert oracle.mixed_norm(A, b) == pytest.approx(max(np.linalg.norm(B) for B in blocks),
                                                    rel=1e-14)
    G = _sym(rng, b * nb)
    perm = rng.permutation(nb)
    idx = np.concatenate([np.arange(p * b, (p + 1) * b) for p in perm])
    assert oracle.mixed_norm(G[np.ix_(idx, idx)], b) == pytest.approx(oracle.mixed_norm(G, b),
                                                                      rel=1e-12)
    Z = np.zeros((b * nb + 5, b * nb + 5))
    Z[:b * nb, :b * nb] = G
    assert oracle.mixed_norm(Z, b) == pytest.approx(oracle.mixed_norm(G, b), rel=1e-14)


def test_stop_with_the_mixed_norm():
    """N = 512: the mixed-norm stop fires on an alternation with r < 1.8,
    between the Frobenius and the spectral stops (give or take rounding
    in stagnation), and returns D."""
    inst = config_small()
    D = oracle.density_from_eigenvectors(inst.Q, inst.n_occ)
    out = {}
    for norm in ("fro", "mixed", "spectral"):
        r = oracle.sp2(inst.F, inst.lambda_min, inst.lambda_max, inst.n_occ, norm=norm,
                       mixed_block=32)
        assert r.status == oracle.Status.OK
        assert np.linalg.norm(r.X - D) < 1e-12 * math.sqrt(inst.n_occ)
        assert r.p[r.n] != r.p[r.n - 1] and r.r[r.n] < oracle.Q_TILDE
        out[norm] = r
    assert out["fro"].n - 2 <= out["mixed"].n <= out["spectral"].n + 2
    # the error sequence itself lies between the other two at every step
    for k in range(min(len(out[x].v) for x in out)):
        if out["fro"].p[:k + 1] == out["mixed"].p[:k + 1] == out["spectral"].p[:k + 1]:
            assert out["spectral"].v[k] * (1 - 1e-9) <= out["mixed"].v[k] <= out["fro"].v[k] * (1 + 1e-9)


def test_mixed_norm_on_the_perturbed_example():
    """The sec. 4.1 example with the mixed norm (block 100): the stop fires
    in the same place as with the spectral norm or earlier, never before
    the Frobenius stop."""
    inst = e5_instance(seed=7)
    n = {}
    for norm in ("fro", "mixed", "spectral"):
        rng = np.random.default_rng(1)
        pert = lambda i, X: symmetric_gaussian_perturbation(X.shape[0], 1e-5, rng)  # noqa: E731
        r = oracle.sp2(inst.F, inst.lambda_min, inst.lambda_max, inst.n_occ, norm=norm,
                       perturb=pert, mixed_block=100)
        assert r.status == oracle.Status.OK
        n[norm] = r.n
    assert n["fro"] <= n["mixed"] <= n["spectral"]
