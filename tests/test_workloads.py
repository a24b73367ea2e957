"""CPU checks of the seeded input generators (no method arithmetic here)."""
import numpy as np
import pytest

from workloads import dense_instance, batch_instances, two_band_spectrum
from workloads.banded import banded_instance, to_bsr_blocks, givens_brick_wall


def test_dense_instance_spectrum_and_bounds_exact():
    inst = dense_instance(200, 90, -1.5, 1.0, 0.2, seed=3)
    ev = np.linalg.eigvalsh(inst.F)
    assert np.max(np.abs(ev - inst.lam)) < 1e-12
    assert inst.lam[0] == -1.5 and inst.lam[-1] == 1.0
    assert abs(inst.lumo - inst.homo - 0.2) < 1e-15
    assert np.array_equal(inst.F, inst.F.T)


def test_two_band_spectrum_counts_and_endpoints():
    rng = np.random.default_rng(0)
    lam = two_band_spectrum(11, 4, -2.0, 3.0, 0.5, rng)
    assert lam.size == 11 and np.all(np.diff(lam) >= 0)
    assert lam[3] == -0.25 and lam[4] == 0.25 and lam[0] == -2.0 and lam[-1] == 3.0


def test_batch_sizes_and_gaps_in_range():
    insts = batch_instances(count=6, n_lo=64, n_hi=120, seed=9)
    for i in insts:
        assert 64 <= i.n <= 120 and i.n_occ == i.n // 2
        assert 0.02 <= i.meta["gap"] <= 0.2


def test_givens_brick_wall_is_orthogonal_and_banded():
    Q = givens_brick_wall(64, 5, np.random.default_rng(1)).toarray()
    assert np.max(np.abs(Q @ Q.T - np.eye(64))) < 1e-13
    i, j = np.nonzero(Q)
    assert np.max(np.abs(i - j)) <= 5


def test_banded_instance_exact_spectrum_and_density():
    inst = banded_instance(n=256, layers=6, seed=4)
    F = inst.F.toarray()
    assert np.array_equal(F, F.T)
    i, j = np.nonzero(F)
    assert np.max(np.abs(i - j)) <= 2 * inst.layers
    assert np.max(np.abs(np.linalg.eigvalsh(F) - inst.lam)) < 1e-12
    D = inst.density_exact().toarray()
    assert abs(np.trace(D) - inst.n_occ) < 1e-10
    assert np.max(np.abs(D @ D - D)) < 1e-12
    _, V = np.linalg.eigh(F)
    Dref = V[:, :inst.n_occ] @ V[:, :inst.n_occ].T
    assert np.max(np.abs(D - Dref)) < 1e-10


def test_bsr_blocks_round_trip_with_padding():
    inst = banded_instance(n=100, layers=4, seed=2)
    rp, ci, bl = to_bsr_blocks(inst.F, 32)
    nb = 4
    assert rp[0] == 0 and rp[-1] == ci.size and rp.size == nb + 1
    E = np.zeros((128, 128))
    for r in range(nb):
        cols = ci[rp[r]:rp[r + 1]]
        assert np.all(np.diff(cols) > 0) and r in cols
        for q in range(rp[r], rp[r + 1]):
            E[32 * r:32 * r + 32, 32 * ci[q]:32 * ci[q] + 32] = bl[q]
    assert np.array_equal(E[:100, :100], inst.F.toarray())
    assert not E[100:].any() and not E[:, 100:].any()
    # the block pattern is symmetric
    pat = {(r, c) for r in range(nb) for c in ci[rp[r]:rp[r + 1]]}
    assert all((c, r) in pat for r, c in pat)


def test_decay_band_entries_and_structure():
    from workloads.decay_band import decay_band, alternating_diagonal
    A = decay_band(400, 40, 8.0, np.random.default_rng(6)).toarray()
    assert np.array_equal(A, A.T) and not np.any(np.diag(A))
    i, j = np.nonzero(A)
    assert np.max(np.abs(i - j)) == 40
    # scaled back by exp(|i - j| / 8) the entries are standard normal
    z = A[i, j] * np.exp(np.abs(i - j) / 8.0)
    assert abs(np.mean(z)) < 0.03 and abs(np.mean(z * z) - 1.0) < 0.05
    assert np.array_equal(alternating_diagonal(5), [-1.0, 1.0, -1.0, 1.0, -1.0])


@pytest.mark.parametrize("n,seed", [(512, 3), (1024, 11)])
def test_decay_band_instance_gap_bounds_and_inertia(n, seed):
    from workloads.decay_band import count_below, decay_band_instance
    inst = decay_band_instance(n=n, seed=seed)
    F = inst.F.toarray()
    ev = np.linalg.eigvalsh(F)
    k = inst.n_occ
    assert k == n // 2
    assert abs(ev[k - 1] - inst.homo) < 1e-12 and abs(ev[k] - inst.lumo) < 1e-12
    assert abs(inst.gap - 0.1) <= 1e-4
    assert inst.lambda_min <= ev[0] and inst.lambda_max >= ev[-1]
    assert ev[0] - inst.lambda_min < 1e-5 and inst.lambda_max - ev[-1] < 1e-5
    d = np.diag(F)
    assert np.all(d[0::2] == -inst.delta) and np.all(d[1::2] == inst.delta)
    for s in (-3.0, inst.homo - 1e-3, 0.5 * (inst.homo + inst.lumo), 2.5):
        assert count_below(inst.F, s) == int(np.count_nonzero(ev < s))
