"""Banded symmetric matrices with an exactly known spectrum (block-sparse
workload).

The paper's sparse inputs (Fock matrices in sec. 5 and sec. 6) are not
available. Their stand-in here is a banded matrix whose eigenvectors are a
product of L layers of random Givens rotations between neighbouring indices
("brick wall": layer l rotates the pairs (i, i+1) with i = l mod 2), so that
Q is orthogonal with bandwidth L, and F = Q diag(lambda) Q^T is symmetric
with bandwidth 2 L and entries that decay away from the diagonal. The
eigenvalues are the two-band spectrum of the dense workloads (gap at the
Fermi level, bounds exact), placed on the diagonal positions in a seeded
random order, so occupied and virtual states are mixed along the chain.
The exact density matrix D = Q diag(occupations) Q^T is banded as well and
is available at any size.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np
import scipy.sparse as sps

from .dense import two_band_spectrum


@dataclass
class BandedInstance:
    F: sps.csr_matrix        # (n, n) float64, symmetric, bandwidth 2 L
    lam: np.ndarray          # eigenvalues, ascending
    n_occ: int
    lambda_min: float
    lambda_max: float
    layers: int
    seed: int
    Q: sps.csr_matrix = None          # eigenvectors, column order of `order`
    order: np.ndarray = None          # diagonal position of each eigenvalue
    meta: dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return self.F.shape[0]

    def density_exact(self) -> sps.csr_matrix:
        """D = Q diag(occ) Q^T with the n_occ lowest eigenvalues occupied."""
        occ = np.zeros(self.n)
        occ[self.order[:self.n_occ]] = 1.0
        D = (self.Q @ sps.diags(occ) @ self.Q.T).tocsr()
        D.sum_duplicates()
        return D


def givens_brick_wall(n: int, layers: int, rng: np.random.Generator) -> sps.csr_matrix:
    """Q = G_L ... G_1, G_l rotating the pairs (i, i+1), i = l mod 2, by
    seeded uniform angles. Orthogonal, bandwidth `layers`."""
    Q = sps.identity(n, format="csr")
    for layer in range(layers):
        i = np.arange(layer % 2, n - 1, 2)
        th = rng.uniform(0.0, 2.0 * np.pi, size=i.size)
        c, s = np.cos(th), np.sin(th)
        diag = np.ones(n)
        diag[i] = c
        diag[i + 1] = c
        rows = np.concatenate([np.arange(n), i, i + 1])
        cols = np.concatenate([np.arange(n), i + 1, i])
        vals = np.concatenate([diag, -s, s])
        G = sps.csr_matrix((vals, (rows, cols)), shape=(n, n))
        Q = (G @ Q).tocsr()
    return Q


def banded_instance(n: int = 32768, layers: int = 48, gap: float = 0.1,
                    lo: float = -1.0, hi: float = 1.0, seed: int = 5001,
                    n_occ: int | None = None) -> BandedInstance:
    rng = np.random.default_rng(seed)
    n_occ = n // 2 if n_occ is None else n_occ
    lam = two_band_spectrum(n, n_occ, lo, hi, gap, rng)
    order = rng.permutation(n)          # diagonal position of lam[k]
    diag = np.empty(n)
    diag[order] = lam
    Q = givens_brick_wall(n, layers, rng)
    F = (Q @ sps.diags(diag) @ Q.T).tocsr()
    F = ((F + F.T) * 0.5).tocsr()
    F.sum_duplicates()
    return BandedInstance(F=F, lam=lam, n_occ=n_occ, lambda_min=lo,
                          lambda_max=hi, layers=layers, seed=seed, Q=Q,
                          order=order, meta=dict(gap=gap))


def to_bsr_blocks(A: sps.spmatrix, bs: int = 32, tau: float = 0.0):
    """Block-sparse row form with bs x bs blocks: (row_ptr, col_idx, blocks)
    with blocks of shape (nnzb, bs, bs), keeping every block that holds an
    entry with |x| >= tau (all stored blocks when tau = 0). The dimension is
    padded with zeros to a multiple of bs."""
    n = A.shape[0]
    nb = (n + bs - 1) // bs
    A = A.tocoo()
    keep = np.abs(A.data) >= tau if tau > 0 else np.ones(A.nnz, bool)
    bi, bj = A.row[keep] // bs, A.col[keep] // bs
    key = np.unique(bi.astype(np.int64) * nb + bj)
    rows, cols = key // nb, key % nb
    row_ptr = np.zeros(nb + 1, np.int32)
    np.add.at(row_ptr, rows + 1, 1)
    row_ptr = np.cumsum(row_ptr).astype(np.int32)
    blocks = np.zeros((key.size, bs, bs))
    pos = np.searchsorted(key, A.row.astype(np.int64) // bs * nb + A.col // bs)
    ok = (pos < key.size)
    ok[ok] &= key[pos[ok]] == (A.row[ok].astype(np.int64) // bs * nb + A.col[ok] // bs)
    blocks[pos[ok], A.row[ok] % bs, A.col[ok] % bs] = A.data[ok]
    return row_ptr, cols.astype(np.int32), blocks
