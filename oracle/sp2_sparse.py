"""Alg. 2 on sparse matrices (CSR), plain FP64 with scipy.sparse.

Test infrastructure: only the tests, their golden-value scripts and the
benchmark's CPU-baseline leg use this module. The library never does.

The same recursion and stopping rule as ``oracle.sp2.sp2`` (readings R1-R10
of that module), for inputs whose dense form is too large: at N = 32768 a
dense FP64 iterate takes 8.6 GB and a dense square 7e13 flops, while the
truncated iterates of a matrix with decaying entries keep a few hundred
nonzeros per row (sec. 5: removing entries below a threshold keeps the
iterates sparse; the paper's sparse runs, sec. 6, use this truncation).

Each step is written with library primitives only: the sparse product
X @ X, its symmetrisation (S + S^T) / 2 (R9), the Frobenius norm of X - S,
the polynomial, and the truncation of entries with |x| < tau (R10), which
also drops them from the sparsity pattern.
"""
from __future__ import annotations

import math

import numpy as np
import scipy.sparse as sps

from .sp2 import (SP2Result, Status, choose_polynomial, observed_order,
                  stop_fires)


def f0_csr(F: sps.spmatrix, lambda_min: float, lambda_max: float) -> sps.csr_matrix:
    """Alg. 2, initial step X_0 = (lambda_max I - F) / (lambda_max - lambda_min)."""
    n = F.shape[0]
    X = (lambda_max * sps.identity(n, format="csr") - F) / (lambda_max - lambda_min)
    return sps.csr_matrix(X)


def truncate_csr(X: sps.csr_matrix, tau: float) -> sps.csr_matrix:
    """E_i of sec. 5: entries with |x| < tau are removed (R10), from the
    values and from the pattern."""
    X = sps.csr_matrix(X, copy=True)
    if tau > 0.0:
        X.data[np.abs(X.data) < tau] = 0.0
    X.eliminate_zeros()
    return X


def fro_csr(A: sps.spmatrix) -> float:
    """||A||_F of a sparse matrix (its stored values)."""
    A = sps.csr_matrix(A)
    A.sum_duplicates()
    return float(np.sqrt(np.sum(A.data * A.data)))


def mixed_norm_csr(A: sps.spmatrix, block: int = 32) -> float:
    """Mixed norm (sec. 2): the spectral norm of the matrix of the Frobenius
    norms of the block x block blocks of A (zero padding at the end)."""
    A = sps.coo_matrix(A)
    n = A.shape[0]
    nb = -(-n // block)
    M = sps.coo_matrix((A.data * A.data, (A.row // block, A.col // block)),
                       shape=(nb, nb)).toarray()
    return float(np.linalg.norm(np.sqrt(M), 2))


def sp2_csr(F: sps.spmatrix, lambda_min: float, lambda_max: float, n_occ: int,
            tau: float = 0.0, branch: str = "nearest", max_iter: int = 100,
            norm: str = "fro", mixed_block: int = 32,
            perturb=None) -> SP2Result:
    """Alg. 2 (original SP2 with the new stopping criterion) on CSR matrices
    in FP64; arguments and result as ``oracle.sp2.sp2`` (res.X is CSR).
    norm: "fro" (R1) or "mixed" (block edge ``mixed_block``). ``perturb(i, X)``
    returns a sparse E_i added after the truncation of X~_i (the experiments
    of sec. 4.1 and sec. 5 perturb every iterate)."""
    F = sps.csr_matrix(F, dtype=np.float64)
    if F.ndim != 2 or F.shape[0] != F.shape[1] or F.shape[0] == 0:
        return SP2Result(None, 0, Status.INVALID_ARG)
    N = F.shape[0]
    if not (0 <= n_occ <= N) or not (lambda_max > lambda_min) \
            or not math.isfinite(lambda_max - lambda_min) or max_iter < 1:
        return SP2Result(None, 0, Status.INVALID_ARG)
    if norm not in ("fro", "mixed"):
        raise ValueError(f"unknown norm {norm!r}")
    if n_occ == 0:                                     # R7
        return SP2Result(sps.csr_matrix((N, N)), 0, Status.OK)
    if n_occ == N:
        return SP2Result(sps.identity(N, format="csr"), 0, Status.OK)

    def error(A):
        return fro_csr(A) if norm == "fro" else mixed_norm_csr(A, mixed_block)

    X = truncate_csr(f0_csr(F, lambda_min, lambda_max), tau)   # X~_0
    if perturb is not None:
        X = (X + perturb(0, X)).tocsr()
    res = SP2Result(None, 0, Status.NOT_CONVERGED)
    res.p.append(-1)
    res.t1.append(float(X.diagonal().sum()))
    res.t2.append(float(np.sum(X.data * X.data)))
    if not (math.isfinite(res.t1[0]) and math.isfinite(res.t2[0])):
        res.status, res.X = Status.DIVERGED, X
        return res

    for i in range(1, max_iter + 1):
        S = X @ X
        S = ((S + S.T) * 0.5).tocsr()                  # R9
        k = i - 1
        vk = error(X - S)
        res.v.append(vk)
        res.r.append(observed_order(vk, res.v[k - 2]) if k >= 2 else float("nan"))
        if not math.isfinite(vk):
            res.status, res.X, res.n = Status.DIVERGED, X, k
            return res
        if vk == 0.0:                                  # R6
            res.status, res.X, res.n = Status.OK, X, k
            return res
        if stop_fires(res.v, res.p, k):                # Alg. 2 stop
            res.status, res.X, res.n = Status.OK, X, k
            return res
        pi = choose_polynomial(res.t1[k], res.t2[k], n_occ, branch)
        res.p.append(pi)
        Xi = S if pi == 1 else (2.0 * X - S).tocsr()   # Alg. 2, X_i
        X = truncate_csr(Xi, tau)                      # X~_i = X_i + E_i
        if perturb is not None:
            X = (X + perturb(i, X)).tocsr()
        t1n, t2n = float(X.diagonal().sum()), float(np.sum(X.data * X.data))
        res.t1.append(t1n)
        res.t2.append(t2n)
        if not (math.isfinite(t1n) and math.isfinite(t2n)) or t2n > t1n + N:
            res.status, res.X, res.n = Status.DIVERGED, X, i
            return res
    res.X, res.n = X, max_iter
    return res


__all__ = ["f0_csr", "truncate_csr", "fro_csr", "mixed_norm_csr", "sp2_csr"]
