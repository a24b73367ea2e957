"""Pins of the sparse (CSR) FP64 oracle, oracle/sp2_sparse.py, that checks the
block-sparse workload at full size. It runs Alg. 2 with the truncation of
sec. 5 on CSR matrices; it is pinned against the dense oracle (itself
pinned against the paper and the mathematics in test_oracle_pins.py) on the
same inputs, bit for bit where both compute exact products, and against
the definitions of its norms."""
import math

import numpy as np
import pytest
import scipy.sparse as sps

import oracle
from oracle.sp2_sparse import fro_csr, mixed_norm_csr, sp2_csr, truncate_csr
from workloads import diagonal_instance
from workloads.decay_band import decay_band_instance


@pytest.fixture(scope="module")
def band512():
    return decay_band_instance(n=512, seed=3)


@pytest.mark.parametrize("tau", [0.0, 1e-6, 1e-4])
def test_same_run_as_dense_oracle(band512, tau):
    inst = band512
    a = sp2_csr(inst.F, inst.lambda_min, inst.lambda_max, inst.n_occ, tau=tau)
    b = oracle.sp2(inst.F.toarray(), inst.lambda_min, inst.lambda_max, inst.n_occ,
                   tau=tau)
    assert a.status == b.status == oracle.Status.OK
    assert a.n == b.n and a.p == b.p
    assert np.max(np.abs(a.X.toarray() - b.X)) < 1e-13
    for x, y in zip(a.v, b.v):
        if y > 1e-8:
            assert abs(x - y) <= 1e-10 * y
    np.testing.assert_allclose(a.t1, b.t1, rtol=1e-12, atol=1e-9)


def test_truncation_removes_entries_from_the_pattern(band512):
    inst = band512
    tau = 1e-4
    r = sp2_csr(inst.F, inst.lambda_min, inst.lambda_max, inst.n_occ, tau=tau)
    X = r.X
    assert X.nnz == np.count_nonzero(X.toarray())
    assert np.all(np.abs(X.data) >= tau)
    # and the truncation itself keeps |x| >= tau, drops |x| < tau
    A = sps.csr_matrix(np.array([[1e-5, -2e-4], [2e-4, -1e-4]]))
    T = truncate_csr(A, 1e-4).toarray()
    assert np.array_equal(T, np.array([[0.0, -2e-4], [2e-4, -1e-4]]))


def test_diagonal_input_bit_exact_with_dense_oracle():
    rng = np.random.default_rng(8)
    n, n_occ = 96, 40
    d = np.concatenate([rng.uniform(-1, -0.05, n_occ), rng.uniform(0.05, 1, n - n_occ)])
    inst = diagonal_instance(d, n_occ, -1.0, 1.0, perm_seed=4)
    a = sp2_csr(sps.csr_matrix(inst.F), -1.0, 1.0, n_occ, max_iter=12)
    b = oracle.sp2(inst.F, -1.0, 1.0, n_occ, max_iter=12)
    assert a.status == b.status and a.n == b.n and a.p == b.p
    assert np.array_equal(a.X.toarray(), b.X)
    # the norms sum the same squares in another order
    np.testing.assert_allclose(a.v, b.v, rtol=1e-14, atol=0)


def test_trivial_and_invalid_inputs():
    F = sps.identity(10, format="csr") * 0.3
    assert sp2_csr(F, -1.0, 1.0, 0).X.nnz == 0
    assert np.array_equal(sp2_csr(F, -1.0, 1.0, 10).X.toarray(), np.eye(10))
    assert sp2_csr(F, 1.0, 1.0, 5).status == oracle.Status.INVALID_ARG
    assert sp2_csr(F, -1.0, 1.0, 11).status == oracle.Status.INVALID_ARG


def test_norms_follow_their_definitions():
    rng = np.random.default_rng(2)
    A = rng.standard_normal((100, 100))
    A[np.abs(A) < 1.0] = 0.0
    S = sps.csr_matrix(A)
    assert fro_csr(S) == pytest.approx(float(np.linalg.norm(A)), rel=1e-14)
    for b in (1, 7, 32, 100):
        assert mixed_norm_csr(S, b) == pytest.approx(oracle.mixed_norm(A, b), rel=1e-12)


def test_mixed_norm_run_matches_dense_oracle(band512):
    inst = band512
    a = sp2_csr(inst.F, inst.lambda_min, inst.lambda_max, inst.n_occ, tau=1e-6,
                norm="mixed")
    b = oracle.sp2(inst.F.toarray(), inst.lambda_min, inst.lambda_max, inst.n_occ,
                   tau=1e-6, norm="mixed")
    assert a.n == b.n and a.p == b.p
    assert np.max(np.abs(a.X.toarray() - b.X)) < 1e-13
    assert math.isclose(a.v[3], b.v[3], rel_tol=1e-10)
