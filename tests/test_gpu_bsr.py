"""GPU parity of the block-sparse (BSR, 32 x 32 FP32 blocks) SP2 path with
element-magnitude truncation against the FP64 oracle run with the same
truncation on the dense form of the same matrix."""
import math

import numpy as np
import pytest

import oracle
from oracle import Status
from workloads.banded import banded_instance, to_bsr_blocks
from workloads import diagonal_instance
from tests.gpu_helpers import print_case

pytestmark = pytest.mark.gpu


def _dev(rp, ci, bl):
    import torch
    return (torch.from_numpy(rp).cuda(), torch.from_numpy(ci).cuda(),
            torch.from_numpy(np.ascontiguousarray(bl)).cuda())


def _run_bsr(F_sparse, n, lmin, lmax, n_occ, tau, **kw):
    import paper_1507_02087_amd as sp2
    rp, ci, bl = to_bsr_blocks(F_sparse, 32)
    ctx = sp2.BsrContext(0)
    ctx.init_bsr(n, *_dev(rp, ci, bl), lmin, lmax, n_occ, trunc_tau=tau, **kw)
    st = ctx.run()
    D = ctx.get_density(as_fp64=True).cpu().numpy()
    n_it, n_sq, ms = ctx.get_info()
    hist = ctx.get_history()
    bsr = ctx.get_bsr()
    ctx.close()
    return st, D, n_it, n_sq, ms, hist, bsr


@pytest.mark.parametrize("n,layers,tau", [(1024, 12, 1e-6), (1000, 20, 1e-6),
                                          (2048, 32, 1e-5)])
def test_banded_matches_truncated_oracle(n, layers, tau):
    import paper_1507_02087_amd as sp2
    inst = banded_instance(n=n, layers=layers, seed=7 + n)
    print_case(f"bsr n={n} layers={layers} tau={tau}")
    st, D, n_it, n_sq, ms, hist, bsr = _run_bsr(
        inst.F, n, inst.lambda_min, inst.lambda_max, inst.n_occ, tau)
    assert st == sp2.OK
    Fd = inst.F.toarray()
    ref = oracle.sp2(Fd, inst.lambda_min, inst.lambda_max, inst.n_occ, tau=tau)
    assert ref.status == Status.OK
    err = np.linalg.norm(D - ref.X) / math.sqrt(inst.n_occ)
    D_exact = inst.density_exact().toarray()
    err_exact = np.linalg.norm(D - D_exact) / math.sqrt(inst.n_occ)
    print_case(f"  n_gpu={n_it} n_oracle={ref.n} err={err:.2e} exact={err_exact:.2e} ms={ms:.2f}")
    assert err < 1e-4
    assert err_exact < 1e-3
    assert abs(np.trace(D) - inst.n_occ) < 1e-3 * math.sqrt(n)
    assert hist["p"][n_it] != hist["p"][n_it - 1] and hist["r"][n_it] < 1.8
    # the block-sparse result: sorted columns, only nonzero blocks, and it
    # expands to the dense result
    rp, ci, bl = (t.cpu().numpy() for t in bsr)
    nb = (n + 31) // 32
    assert rp[0] == 0 and rp[-1] == ci.size
    E = np.zeros((nb * 32, nb * 32))
    for r in range(nb):
        cols = ci[rp[r]:rp[r + 1]]
        assert np.all(np.diff(cols) > 0)
        for q in range(rp[r], rp[r + 1]):
            assert np.any(bl[q] != 0)
            E[r * 32:(r + 1) * 32, cols[q - rp[r]] * 32:(cols[q - rp[r]] + 1) * 32] = bl[q]
    assert np.array_equal(E[:n, :n], D)
    assert np.array_equal(D, D.T)


def test_truncation_zero_matches_dense_oracle_closely():
    import paper_1507_02087_amd as sp2
    inst = banded_instance(n=512, layers=8, seed=3)
    st, D, n_it, *_ = _run_bsr(inst.F, 512, inst.lambda_min, inst.lambda_max,
                               inst.n_occ, 0.0)
    ref = oracle.sp2(inst.F.toarray(), inst.lambda_min, inst.lambda_max, inst.n_occ)
    assert st == sp2.OK
    assert np.linalg.norm(D - ref.X) / math.sqrt(inst.n_occ) < 2e-5


def test_block_diagonal_input_bit_exact():
    """A diagonal F: every block product is one scalar product plus exact
    zeros, so the iterates equal the oracle's FP32 working precision bit for
    bit (only diagonal blocks are ever stored)."""
    import scipy.sparse as sps
    import paper_1507_02087_amd as sp2
    rng = np.random.default_rng(5)
    n, n_occ = 200, 90
    d = np.concatenate([rng.uniform(-1, -0.05, n_occ), rng.uniform(0.05, 1, n - n_occ)])
    rng.shuffle(d)
    inst = diagonal_instance(d, n_occ, -1.0, 1.0)
    F = sps.csr_matrix(np.diag(d))
    # store all diagonal blocks (a diagonal with zeros is still block-diagonal)
    rp, ci, bl = to_bsr_blocks(F, 32)
    ctx = sp2.BsrContext(0)
    ctx.init_bsr(n, *_dev(rp, ci, bl), -1.0, 1.0, n_occ, max_iter=9)
    st = ctx.run()
    D = ctx.get_density(as_fp64=True).cpu().numpy()
    h = ctx.get_history()
    ctx.close()
    ref = oracle.sp2(inst.F, -1.0, 1.0, n_occ, max_iter=9, working="fp32")
    assert st == sp2.NOT_CONVERGED and h["p"] == ref.p
    assert np.array_equal(D, ref.X)


def test_invalid_patterns_rejected():
    import torch
    import paper_1507_02087_amd as sp2
    ctx = sp2.BsrContext(0)
    bl = torch.zeros((3, 32, 32), dtype=torch.float64, device="cuda")
    cases = [
        ([0, 2, 3], [0, 1, 1]),     # (0,1) stored, (1,0) missing: asymmetric
        ([0, 1, 2], [1, 0]),        # diagonal blocks missing
        ([0, 2, 3], [1, 0, 1]),     # columns not sorted
    ]
    for rp, ci in cases:
        rpt = torch.tensor(rp, dtype=torch.int32, device="cuda")
        cit = torch.tensor(ci, dtype=torch.int32, device="cuda")
        with pytest.raises(sp2.SP2Error) as e:
            ctx.init_bsr(64, rpt, cit, bl[:len(ci)], -1.0, 1.0, 32)
        assert e.value.status == sp2.INVALID_ARG
    ctx.close()


def test_long_rows_and_ragged_tail():
    """Every block present (dense F as BSR, N = 2390: 75 block rows, the last
    ragged), so each row of the iterate holds 75 blocks and the product
    kernel walks its column lists in two chunks of at most 64; against the
    FP64 oracle on the dense form (no truncation)."""
    import scipy.sparse as sps
    import paper_1507_02087_amd as sp2
    from workloads import dense_instance
    inst = dense_instance(2390, 1100, -1.0, 1.0, 0.1, seed=2390)
    print_case("bsr n=2390, all 75 x 75 blocks stored")
    st, D, n_it, n_sq, ms, hist, _ = _run_bsr(sps.csr_matrix(inst.F), 2390,
                                             inst.lambda_min, inst.lambda_max,
                                             inst.n_occ, 0.0)
    assert st == sp2.OK
    ref = oracle.sp2(inst.F, inst.lambda_min, inst.lambda_max, inst.n_occ)
    err = np.linalg.norm(D - ref.X) / math.sqrt(inst.n_occ)
    De = oracle.density_from_eigenvectors(inst.Q, inst.n_occ)
    err_exact = np.linalg.norm(D - De) / math.sqrt(inst.n_occ)
    print(f"  n_gpu={n_it} n_oracle={ref.n} err={err:.2e} exact={err_exact:.2e} "
          f"{ms:.2f} ms", flush=True)
    assert err_exact < 2e-5
    assert abs(n_it - ref.n) <= 2
    for k, (a, r) in enumerate(zip(hist["v"], ref.v)):
        if r > 1e-2:
            assert abs(a - r) <= 1e-4 * r, (k, a, r)


def test_fill_beyond_capacity_reported():
    """A block-tridiagonal F without truncation fills in (the pattern of X^2
    has twice the block bandwidth of X's) until a pattern needs more blocks
    than the library keeps room for (min(nb^2, 16 nnzb + 64 nb) = 28640 for
    nb = 256): the fill kernel finds the total over capacity before writing
    anything and the run stops with SP2_OUT_OF_MEMORY."""
    import scipy.sparse as sps
    import paper_1507_02087_amd as sp2
    nb = 256
    n = 32 * nb
    rng = np.random.default_rng(256)
    offs = list(range(0, 33))
    B = sps.diags([rng.standard_normal(n - k) for k in offs], offs, shape=(n, n),
                  format="csr")
    F = (B + B.T).tocsr()
    R = float(np.max(np.asarray(abs(F).sum(axis=1)).ravel()))
    rp, ci, bl = to_bsr_blocks(F, 32)
    assert rp[-1] == 3 * nb - 2          # block tridiagonal
    print_case(f"bsr n={n} block-tridiagonal, tau=0, capacity overflow")
    ctx = sp2.BsrContext(0)
    ctx.init_bsr(n, *_dev(rp, ci, bl), -R, R, n // 2, trunc_tau=0.0)
    with pytest.raises(sp2.SP2Error) as e:
        ctx.run()
    assert e.value.status == sp2.OUT_OF_MEMORY
    assert "capacity" in str(e.value)
    ctx.close()
