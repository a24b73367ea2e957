"""The regime the mixed norm exists for (sec. 2, after the Frobenius
estimate; sec. 5, the diagonal example of fig:num_test_diag_matrices): for a
large system perturbed in every step, ||X~ - X~^2||_F never falls below 1,
so the Frobenius form of the stopping test is never evaluated (reading R2)
and the run ends at max_iter, while the mixed norm with a fixed block size
stagnates below 1 and the test stops the run on an alternation with an
observed order below 1.8 at the exact projector within the noise.

The paper's example has dimension 1e8 with a perturbation of spectral norm
1e-3 and block size 1000. Scaled down here: dimension 1e6, diagonal, gap 0.1
centred at 0.5, equidistant eigenvalues in [0, 1], n_occ = N/2, a diagonal
normal perturbation of spectral norm 6e-3 in every step (Frobenius norm
about 1.1, so that it alone keeps v above 1), block size 1000."""
import math

import numpy as np
import pytest
import scipy.sparse as sps

import oracle
from oracle.sp2_sparse import sp2_csr

N = 1_000_000
SPEC = 6e-3
BLOCK = 1000


def _inputs():
    half = N // 2
    lo = np.linspace(0.0, 0.45, half)            # virtual side of X_0
    hi = np.linspace(0.55, 1.0, N - half)        # occupied side of X_0
    x0 = np.concatenate([lo, hi])
    # F = I - X_0 with bounds [0, 1], so that X_0 = (1 I - F) / 1
    F = sps.diags(1.0 - x0, format="csr")
    occ = (x0 > 0.5).astype(float)

    def perturb(i, X):
        rng = np.random.default_rng(1000 + i)
        e = rng.standard_normal(N)
        return sps.diags(e * (SPEC / np.max(np.abs(e))), format="csr")
    return F, occ, perturb


@pytest.fixture(scope="module")
def runs():
    F, occ, perturb = _inputs()
    fro = sp2_csr(F, 0.0, 1.0, N // 2, max_iter=40, perturb=perturb)
    mix = sp2_csr(F, 0.0, 1.0, N // 2, max_iter=40, perturb=perturb, norm="mixed",
                  mixed_block=BLOCK)
    return fro, mix, occ


def test_frobenius_error_never_below_one(runs):
    fro, _, _ = runs
    assert fro.status == oracle.Status.NOT_CONVERGED
    assert min(fro.v) > 1.0
    # the order test is never evaluated (R2: it needs v_{k-2} < 1)
    assert all(math.isnan(r) for r in fro.r)


def test_mixed_norm_stops_at_the_projector(runs):
    fro, mix, occ = runs
    assert mix.status == oracle.Status.OK
    k = mix.n
    assert mix.p[k] != mix.p[k - 1] and mix.r[k] < oracle.Q_TILDE
    assert 0.0 < mix.v[k - 2] < 1.0
    d = mix.X.diagonal()
    assert np.max(np.abs(d - occ)) < 10 * SPEC
    assert abs(float(d.sum()) - N // 2) < 10 * SPEC * math.sqrt(N)
    # spectral <= mixed <= Frobenius (sec. 2); for a diagonal error the
    # spectral norm is its largest entry
    for kk in range(1, k + 1):
        assert mix.v[kk] <= fro.v[kk] * (1 + 1e-12) or kk > len(fro.v)
    # the stop comes once the error has stagnated at the noise level: about
    # the largest Frobenius norm of a block of the perturbation, sigma
    # sqrt(block) with sigma ~ SPEC / sqrt(2 ln N)
    sigma = SPEC / math.sqrt(2.0 * math.log(N))
    assert mix.v[k] < 5 * sigma * math.sqrt(BLOCK)
