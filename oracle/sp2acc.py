"""SP2-ACC: SP2 with a polynomial schedule fixed in advance from bounds of the
homo and lumo eigenvalues, scale-and-fold acceleration and the parameterless
stopping criterion. Plain FP64 (optionally FP32-rounded squares).

Test infrastructure: only the tests, the smoke check and the benchmark's
CPU-baseline leg use this module. The library never does.

Follows Alg. 3 (determination of the polynomials) and Alg. 4 (the SP2-ACC
expansion) of Kruchinina, Rudberg, Rubensson (2015), sec. 4, with the
switch-off of the acceleration discussed after the derivation of C_2^sp.
Readings taken where the text is garbled or silent:

* R16 the loop of Alg. 3 continues while the bound estimates are not yet
      idempotent to eps_M OR the last two polynomials are equal (read with
      'and' it would end at the first alternation); an undefined p (steps 0
      and -1) counts as equal, so a schedule has at least two steps and ends
      on an alternation, where the stop test of Alg. 4 can fire.
* R18 eps_M is the FP64 machine epsilon whatever precision the squares use:
      n_max is an upper estimate of the iteration count; the stop decides.
* R19 if the stop has not fired at i = n_max, X~_{n_max} is returned with
      n = n_max (the loop of Alg. 4 ends there).
* R20 if the acceleration is never switched off inside the loop of Alg. 3,
      n_min = n_max.
* R21 the bounds must satisfy lambda_min <= homo_out <= homo_in < lumo_in
      <= lumo_out <= lambda_max with homo_in > lambda_min and lumo_in <
      lambda_max (the homo/lumo intervals may not overlap, sec. 6; Theorem 2
      needs nonzero upper bounds); ``accelerate=False`` runs Alg. 3 with the
      lower bounds set to zero (alpha_i = 1), the setting of Theorem 2.
* R1, R2, R6, R7, R9, R10 and the max_iter cap are as in ``oracle.sp2``.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import Callable, Optional

import numpy as np

from .sp2 import (C_SP2, Q_TILDE, SP2Result, Status, _error, _square,
                  _store, f0, observed_order, truncate)

EPS_M = float(np.finfo(np.float64).eps)   # R18
DELTA = 0.01                              # Alg. 3 switch-off threshold


@dataclass
class Schedule:
    """Output of Alg. 3. p[i], alpha[i] for i = 1..n_max (index 0 unused)."""

    n_min: int
    n_max: int
    p: list = field(default_factory=list)
    alpha: list = field(default_factory=list)
    beta_up: list = field(default_factory=list)    # after step i (index 0: start)
    gamma_up: list = field(default_factory=list)
    beta_low: list = field(default_factory=list)
    gamma_low: list = field(default_factory=list)


def bounds_valid(lambda_min, lambda_max, homo_out, homo_in, lumo_in, lumo_out) -> bool:
    """R21."""
    vals = (lambda_min, lambda_max, homo_out, homo_in, lumo_in, lumo_out)
    if not all(math.isfinite(v) for v in vals):
        return False
    return (lambda_min <= homo_out <= homo_in < lumo_in <= lumo_out <= lambda_max
            and homo_in > lambda_min and lumo_in < lambda_max)


def acc_schedule(lambda_min: float, lambda_max: float, homo_out: float,
                 homo_in: float, lumo_in: float, lumo_out: float,
                 accelerate: bool = True, eps: float = EPS_M,
                 delta: float = DELTA, max_len: int = 200) -> Optional[Schedule]:
    """Alg. 3: the polynomial p_i and stretch alpha_i of every step, n_min
    (first step where the stop is checked) and n_max (length).

    beta is the distance of the homo image from 1 and gamma that of the lumo
    image from 0 in the spectrum of X_0; 'up'/'low' are the upper and lower
    bounds of these distances given by the inner/outer eigenvalue bounds.
    Each step folds the side that is further from its target: x^2 with the
    stretch alpha = 2/(2 - gamma_low) when gamma_up >= beta_up, otherwise
    2x - x^2 with alpha = 2/(2 - beta_low); both bounds of both sides are
    mapped through the chosen polynomial. Returns None for bounds that R21
    rejects or a schedule longer than max_len.
    """
    if not bounds_valid(lambda_min, lambda_max, homo_out, homo_in, lumo_in, lumo_out):
        return None
    w = lambda_max - lambda_min
    b_up = 1.0 - (lambda_max - homo_in) / w
    b_lo = 1.0 - (lambda_max - homo_out) / w
    g_up = (lambda_max - lumo_in) / w
    g_lo = (lambda_max - lumo_out) / w
    if not accelerate:
        b_lo = g_lo = 0.0
    sched = Schedule(n_min=-1, n_max=0, p=[-1], alpha=[1.0], beta_up=[b_up],
                     gamma_up=[g_up], beta_low=[b_lo], gamma_low=[g_lo])
    d = delta
    i = 0

    def same_as_previous(i: int) -> bool:     # R16: undefined counts as equal
        return i < 2 or sched.p[i] == sched.p[i - 1]

    while (b_up - b_up * b_up > eps or g_up - g_up * g_up > eps) or same_as_previous(i):
        i += 1
        if i > max_len:
            return None
        if b_lo < d and g_lo < d:              # switch the acceleration off
            b_lo = 0.0
            g_lo = 0.0
            sched.n_min = i + 1
            d = 0.0
        if g_up >= b_up:
            p = 1
            a = 2.0 / (2.0 - g_lo)
            # unoccupied side: folded by ((1 - a) + a x)^2
            g_lo = ((1.0 - a) + a * g_lo) ** 2
            g_up = ((1.0 - a) + a * g_up) ** 2
            # occupied side: distance from 1 after the same polynomial
            b_lo = 2.0 * a * b_lo - (a * b_lo) ** 2
            b_up = 2.0 * a * b_up - (a * b_up) ** 2
        else:
            p = 0
            a = 2.0 / (2.0 - b_lo)
            g_lo = 2.0 * a * g_lo - (a * g_lo) ** 2
            g_up = 2.0 * a * g_up - (a * g_up) ** 2
            b_lo = ((1.0 - a) + a * b_lo) ** 2
            b_up = ((1.0 - a) + a * b_up) ** 2
        sched.p.append(p)
        sched.alpha.append(a)
        sched.beta_up.append(b_up)
        sched.gamma_up.append(g_up)
        sched.beta_low.append(b_lo)
        sched.gamma_low.append(g_lo)
    sched.n_max = i
    if sched.n_min < 0 or sched.n_min > sched.n_max:   # R20
        sched.n_min = sched.n_max
    return sched


def acc_polynomial(p: int, alpha: float, x):
    """Alg. 4: ((1 - a) + a x)^2 for p = 1, 2 a x - (a x)^2 for p = 0; maps
    [0, 1] into [0, 1] for 1 <= a <= 2 and reduces to the SP2 polynomials at
    a = 1."""
    if p == 1:
        y = (1.0 - alpha) + alpha * x
        return y * y
    y = alpha * x
    return 2.0 * y - y * y


def sp2_acc(F: np.ndarray, lambda_min: float, lambda_max: float,
            sched: Schedule, norm: str = "fro", tau: float = 0.0,
            max_iter: int = 100,
            perturb: Optional[Callable[[int, np.ndarray], np.ndarray]] = None,
            working: str = "fp64", mixed_block: int = 32) -> SP2Result:
    """Alg. 4 with the schedule of Alg. 3.

    Per step i = 1..n_max: X_i = ((1 - a_i) I + a_i X~_{i-1})^2 (p_i = 1) or
    2 a_i X~_{i-1} - (a_i X~_{i-1})^2 (p_i = 0), X~_i = X_i + E_i (truncation,
    then ``perturb``), e_i = ||X~_i - X~_i^2||, and the stop at i >= n_min
    when p_i != p_{i-1} and log(e_i / C) / log(e_{i-2}) < 1.8. The matrix
    products are formed exactly as written (a product for the polynomial and
    a second one for the error). ``working`` = "fp64" or "fp32" rounds the
    stored iterates and the products to that precision.

    Result fields as in ``oracle.sp2.sp2``; res.p holds p_1.. with p[0] = -1,
    and ``max_iter`` counts squares the way the library does: X~_i is
    returned with NOT_CONVERGED once i reaches max_iter before the stop.
    """
    F = np.asarray(F, dtype=np.float64)
    if F.ndim != 2 or F.shape[0] != F.shape[1] or F.shape[0] == 0 or sched is None:
        return SP2Result(None, 0, Status.INVALID_ARG)
    if not (lambda_max > lambda_min) or max_iter < 1:
        return SP2Result(None, 0, Status.INVALID_ARG)
    if working not in ("fp64", "fp32"):
        raise ValueError(f"unknown working precision {working!r}")
    if norm not in ("fro", "spectral", "mixed") or mixed_block < 1:
        raise ValueError(f"unknown norm {norm!r} / block {mixed_block}")
    N = F.shape[0]
    eye = np.eye(N)

    def error(X):
        S = _square(X, working)
        S = 0.5 * (S + S.T)                           # R9
        return _error(X, S, norm, mixed_block)

    X = _store(truncate(f0(F, lambda_min, lambda_max), tau), working)
    if perturb is not None:
        X = _store(X + perturb(0, X), working)
    res = SP2Result(None, 0, Status.NOT_CONVERGED)
    res.p.append(-1)
    res.t1.append(float(np.trace(X)))
    res.t2.append(float(np.sum(X * X)))
    if not (math.isfinite(res.t1[0]) and math.isfinite(res.t2[0])):
        res.status, res.X = Status.DIVERGED, X
        return res
    e0 = error(X)                                     # e_0
    res.v.append(e0)
    res.r.append(float("nan"))
    if not math.isfinite(e0):
        res.status, res.X = Status.DIVERGED, X
        return res
    if e0 == 0.0:                                     # R6
        res.status, res.X = Status.OK, X
        return res

    for i in range(1, sched.n_max + 1):
        p, a = sched.p[i], sched.alpha[i]
        if p == 1:
            M = _store((1.0 - a) * eye + a * X, working)
            Xi = _square(M, working)
        else:
            M = _store(a * X, working)
            Xi = 2.0 * M - _square(M, working)
        Xi = 0.5 * (Xi + Xi.T)                        # R9
        Xi = truncate(_store(Xi, working), tau)       # X~_i = X_i + E_i
        if perturb is not None:
            Xi = _store(Xi + perturb(i, Xi), working)
        X = Xi
        res.p.append(p)
        t1, t2 = float(np.trace(X)), float(np.sum(X * X))
        res.t1.append(t1)
        res.t2.append(t2)
        if not (math.isfinite(t1) and math.isfinite(t2)) or t2 > t1 + N:
            res.status, res.X, res.n = Status.DIVERGED, X, i
            return res
        if i >= max_iter:
            res.status, res.X, res.n = Status.NOT_CONVERGED, X, i
            return res
        ei = error(X)                                 # e_i
        res.v.append(ei)
        r = observed_order(ei, res.v[i - 2]) if i >= 2 else float("nan")
        res.r.append(r)
        if not math.isfinite(ei):
            res.status, res.X, res.n = Status.DIVERGED, X, i
            return res
        if ei == 0.0:                                 # R6
            res.status, res.X, res.n = Status.OK, X, i
            return res
        if i >= sched.n_min and p != res.p[i - 1] and not math.isnan(r) and r < Q_TILDE:
            res.status, res.X, res.n = Status.OK, X, i   # Alg. 4 stop
            return res
    res.status, res.X, res.n = Status.OK, X, sched.n_max   # R19
    return res


__all__ = ["EPS_M", "DELTA", "Schedule", "bounds_valid", "acc_schedule",
           "acc_polynomial", "sp2_acc", "C_SP2"]
