"""SP2 purification with the parameterless stopping criterion, plain FP64.

Test infrastructure: only the tests, the smoke check and the benchmark's
CPU-baseline leg use this module. The library never does.

Each function cites the part of Kruchinina, Rudberg, Rubensson (2015) that it
follows. Where the paper is silent or ambiguous, the reading taken here is
named in the docstring (readings R1-R12 of the design notes):

* R1  the idempotency error fed to the stop is the Frobenius norm
      v_i = ||X_i - X_i^2||_F (sec. 2, eq. eq:frobnorm); the spectral norm of
      Alg. 2 is available as an option for small N.
* R2  the order test is evaluated only when 0 < v_{k-2} < 1 (sec. 2: the
      Frobenius estimate of the order is valid only below one).
* R3  polynomial choice: x^2 is taken iff the trace it produces is nearer to
      n_occ than the trace 2x - x^2 produces. This is Alg. 2's
      "Tr X > n_occ" whenever Tr X^2 <= Tr X (true for any spectrum inside
      [0,1]); the literal rule is kept as an option.
* R4  n is the index of the returned iterate; n + 1 squares were computed.
* R5  the returned matrix is X~_n, not the already computed X_{n+1}.
* R6  v_k == 0 exactly stops with n = k.
* R7  n_occ = 0 returns 0 and n_occ = N returns I (n = 0); bounds with
      lambda_max <= lambda_min are rejected; non-finite traces or errors, or
      Tr X^2 > Tr X + N, report divergence.
* R8  at most max_iter squares (default 100); otherwise NOT_CONVERGED and
      the last iterate X~_{max_iter}.
* R9  the computed square is symmetrised, S <- (S + S^T)/2.
* R10 truncation E_i removes entries with |x| < tau, applied to X_0 and to
      every X_i after the polynomial is applied, before traces and errors.
"""
from __future__ import annotations

import enum
import math
from dataclasses import dataclass, field
from typing import Callable, Optional

import numpy as np

# Alg. 2 and sec. 4 (derivation of C_2^sp): the smallest constant such that the
# observed order over two alternating SP2 steps is at least 2 in exact
# arithmetic, C = max_x g(x, 0) for p(x) = p1(p2(x)) or p2(p1(x)).
C_SP2 = (71.0 + 17.0 * math.sqrt(17.0)) / 32.0
# Sec. 2: tolerance q~ used in place of the order q = 2.
Q_TILDE = 1.8


class Status(enum.IntEnum):
    """Outcome codes; the numeric values match the C library's enum."""

    OK = 0
    INVALID_ARG = 1
    OUT_OF_MEMORY = 2
    HIP_ERROR = 3
    NOT_CONVERGED = 4
    DIVERGED = 5
    BAD_STATE = 6


@dataclass
class SP2Result:
    X: Optional[np.ndarray]          # X~_n, the returned approximation of D
    n: int                           # index of X~_n (n + 1 squares computed)
    status: Status
    v: list = field(default_factory=list)    # v[k] = ||X~_k - X~_k^2||
    t1: list = field(default_factory=list)   # t1[k] = Tr X~_k
    t2: list = field(default_factory=list)   # t2[k] = ||X~_k||_F^2
    p: list = field(default_factory=list)    # p[i], i >= 1 (p[0] = -1)
    r: list = field(default_factory=list)    # r[k] = log(v_k/C)/log(v_{k-2})

    @property
    def n_squares(self) -> int:
        return len(self.v)


# ---------------------------------------------------------------- polynomials
def p_sp1(x):
    """SP2 polynomial x^2 (sec. 4, first polynomial)."""
    return x * x


def p_sp2(x):
    """SP2 polynomial 2x - x^2 (sec. 4, second polynomial)."""
    return 2.0 * x - x * x


def g_ratio(f: Callable, x, q: float = 2.0):
    """Theorem 1 with a = 0: g(x) = (f(x) - f(x)^2) / (x - x^2)^q."""
    fx = f(x)
    return (fx - fx * fx) / (x - x * x) ** q


# ---------------------------------------------------------------- steps
def f0(F: np.ndarray, lambda_min: float, lambda_max: float) -> np.ndarray:
    """Alg. 2, initial step: X_0 = (lambda_max I - F)/(lambda_max - lambda_min).

    Maps the spectrum of F into [0, 1] in reverse order so that occupied
    states (lowest eigenvalues of F) end up near 1.
    """
    n = F.shape[0]
    return (lambda_max * np.eye(n) - F) / (lambda_max - lambda_min)


def truncate(X: np.ndarray, tau: float) -> np.ndarray:
    """Truncation E_i by element magnitude (sec. 5): entries with |x| < tau
    are removed (set to zero); entries with |x| >= tau are kept (R10)."""
    if tau <= 0.0:
        return X
    Y = X.copy()
    Y[np.abs(Y) < tau] = 0.0
    return Y


def choose_polynomial(t1: float, t2: float, n_occ: int,
                      rule: str = "nearest") -> int:
    """Polynomial for the next step (Alg. 2, the trace test on the branch).

    t1 = Tr X, t2 = Tr X^2. Returns 1 for x^2 and 0 for 2x - x^2.
    ``literal``: x^2 iff Tr X > n_occ.
    ``nearest`` (R3): x^2 iff |Tr X^2 - n_occ| < |Tr(2X - X^2) - n_occ|;
    a tie gives 0, as the strict '>' of the literal rule does.
    """
    if rule == "literal":
        return 1 if t1 > n_occ else 0
    if rule == "nearest":
        return 1 if abs(t2 - n_occ) < abs(2.0 * t1 - t2 - n_occ) else 0
    raise ValueError(f"unknown branch rule {rule!r}")


def observed_order(v_k: float, v_km2: float) -> float:
    """r_k = log(v_k / C) / log(v_{k-2}) (sec. 2, eq. eq:Cq_relation; Alg. 2
    uses the error two steps back because C is derived for a composition of
    the two SP2 polynomials). NaN where it is not defined (R2)."""
    if not (0.0 < v_km2 < 1.0) or not (v_k > 0.0):
        return float("nan")
    return math.log(v_k / C_SP2) / math.log(v_km2)


def stop_fires(v: list, p: list, k: int) -> bool:
    """Alg. 2 stopping test at step k: k >= 2, the polynomials of steps k and
    k-1 differ, and the observed order r_k is below q~ = 1.8 (R2: only when
    0 < v_{k-2} < 1)."""
    if k < 2 or p[k] == p[k - 1]:
        return False
    r = observed_order(v[k], v[k - 2])
    return (not math.isnan(r)) and r < Q_TILDE


# ---------------------------------------------------------------- precision
def _round_bf16(a: np.ndarray) -> np.ndarray:
    """Round float32 values to bfloat16 (round to nearest, ties to even),
    returned as float32. NaN/Inf are not expected here."""
    b = np.ascontiguousarray(a, dtype=np.float32).view(np.uint32).astype(np.uint64)
    lsb = (b >> 16) & 1
    b = (b + 0x7FFF + lsb) & 0xFFFF0000
    return b.astype(np.uint32).view(np.float32)


def _square(X: np.ndarray, working: str) -> np.ndarray:
    """The matrix square in the requested working precision.

    ``fp64``: plain float64 product. ``fp32``: the product of the float32
    rounding of X, accumulated in float32. ``bf16x3``: X (float32) is split
    into H = bf16(X) and L = bf16(X - H); S = H H + H L + L H accumulated in
    float32 (the L L term is dropped). The result is returned in float64.
    """
    if working == "fp64":
        return X @ X
    X32 = X.astype(np.float32)
    if working == "fp32":
        return (X32 @ X32).astype(np.float64)
    if working == "bf16x3":
        H = _round_bf16(X32)
        L = _round_bf16(X32 - H)
        S = H @ H
        S += H @ L
        S += L @ H
        return S.astype(np.float64)
    raise ValueError(f"unknown working precision {working!r}")


def _store(X: np.ndarray, working: str) -> np.ndarray:
    """Round an iterate to the precision it is stored in."""
    if working == "fp64":
        return X
    return X.astype(np.float32).astype(np.float64)


def _spectral_error(X: np.ndarray, S: np.ndarray) -> float:
    return float(np.max(np.abs(np.linalg.eigvalsh(X - S))))


def mixed_norm(A: np.ndarray, block: int) -> float:
    """Mixed norm (sec. 2, after eq. eq:estim_order_using_frob_norm): A is
    cut into square blocks of edge ``block`` (zero padding at the end), and
    the result is the spectral norm of the matrix of the blocks' Frobenius
    norms. It lies between the spectral and the Frobenius norm of A."""
    n = A.shape[0]
    nb = -(-n // block)
    P = np.zeros((nb * block, nb * block))
    P[:n, :n] = A
    M = np.sqrt(np.einsum("ibjc->ij", (P * P).reshape(nb, block, nb, block)))
    return float(np.linalg.norm(M, 2))


def _error(X: np.ndarray, S: np.ndarray, norm: str, mixed_block: int) -> float:
    """||X - S|| in the requested norm (R1; 'mixed' for large N, sec. 2)."""
    if norm == "fro":
        return float(np.linalg.norm(X - S, "fro"))         # eq. eq:frobnorm
    if norm == "spectral":
        return _spectral_error(X, S)                        # Alg. 2, e_k
    if norm == "mixed":
        return mixed_norm(X - S, mixed_block)
    raise ValueError(f"unknown norm {norm!r}")


# ---------------------------------------------------------------- algorithm
def sp2(F: np.ndarray, lambda_min: float, lambda_max: float, n_occ: int,
        norm: str = "fro", branch: str = "nearest", tau: float = 0.0,
        max_iter: int = 100,
        perturb: Optional[Callable[[int, np.ndarray], np.ndarray]] = None,
        working: str = "fp64", mixed_block: int = 32) -> SP2Result:
    """Alg. 2 (original SP2 with the new stopping criterion), FP64.

    F: symmetric (N, N); lambda_min <= lambda_1 and lambda_max >= lambda_N
    (sec. 3, bounds of the extremal eigenvalues); n_occ: number of occupied
    states. ``perturb(i, X)`` returns E_i, added after truncation (the
    paper's experiments of sec. 4.1 and sec. 5 perturb every iterate).
    ``working`` selects the precision of the matrix square and of the stored
    iterate ("fp64", "fp32", "bf16x3"); traces, errors and the stop test
    stay in float64 in every mode. ``norm`` = "fro", "spectral" or "mixed"
    (block edge ``mixed_block``); the stop formula is the same for each,
    with the error two steps back required in (0, 1) (R2).

    Loop structure, per step i >= 1: the square S = X~_{i-1}^2 is computed
    once and serves both v_{i-1} = ||X~_{i-1} - S|| (the error that the stop
    test at k = i - 1 needs) and the next iterate X_i = S or 2 X~_{i-1} - S.
    """
    F = np.asarray(F, dtype=np.float64)
    if F.ndim != 2 or F.shape[0] != F.shape[1] or F.shape[0] == 0:
        return SP2Result(None, 0, Status.INVALID_ARG)
    N = F.shape[0]
    if not (0 <= n_occ <= N) or not (lambda_max > lambda_min) \
            or not math.isfinite(lambda_max - lambda_min) or max_iter < 1:
        return SP2Result(None, 0, Status.INVALID_ARG)
    if norm not in ("fro", "spectral", "mixed") or mixed_block < 1:
        raise ValueError(f"unknown norm {norm!r} / block {mixed_block}")
    if n_occ == 0:                                     # R7
        return SP2Result(np.zeros((N, N)), 0, Status.OK)
    if n_occ == N:
        return SP2Result(np.eye(N), 0, Status.OK)

    X = f0(F, lambda_min, lambda_max)                  # Alg. 2: X_0
    X = _store(truncate(X, tau), working)              # X~_0 = X_0 + E_0
    if perturb is not None:
        X = _store(X + perturb(0, X), working)

    res = SP2Result(None, 0, Status.NOT_CONVERGED)
    res.p.append(-1)
    res.t1.append(float(np.trace(X)))
    res.t2.append(float(np.sum(X * X)))
    if not (math.isfinite(res.t1[0]) and math.isfinite(res.t2[0])):
        res.status = Status.DIVERGED
        res.X = X
        return res

    for i in range(1, max_iter + 1):
        S = _square(X, working)
        S = 0.5 * (S + S.T)                            # R9
        k = i - 1
        vk = _error(X, S, norm, mixed_block)
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
        t1, t2 = res.t1[k], res.t2[k]
        pi = choose_polynomial(t1, t2, n_occ, branch)
        res.p.append(pi)
        Xi = S if pi == 1 else 2.0 * X - S             # Alg. 2, X_i
        Xi = truncate(_store(Xi, working), tau)        # X~_i = X_i + E_i
        if perturb is not None:
            Xi = _store(Xi + perturb(i, Xi), working)
        X = Xi
        t1n, t2n = float(np.trace(X)), float(np.sum(X * X))
        res.t1.append(t1n)
        res.t2.append(t2n)
        if not (math.isfinite(t1n) and math.isfinite(t2n)) or t2n > t1n + N:
            res.status, res.X, res.n = Status.DIVERGED, X, i
            return res
    res.X, res.n = X, max_iter
    return res


# ---------------------------------------------------------------- exact D
def density_from_eigenvectors(Q: np.ndarray, n_occ: int) -> np.ndarray:
    """eq. eq:D_def: D = sum over the n_occ lowest eigenpairs of x x^T, given
    the eigenvectors sorted by ascending eigenvalue."""
    Qo = Q[:, :n_occ]
    return Qo @ Qo.T


def density_from_eigh(F: np.ndarray, n_occ: int) -> np.ndarray:
    """eq. eq:D_def via a LAPACK eigendecomposition of F."""
    _, V = np.linalg.eigh(F)
    return density_from_eigenvectors(V, n_occ)
