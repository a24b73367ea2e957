"""McWeeny and McW-ACC purification with the parameterless stopping criterion,
plain FP64 (optionally FP32-rounded products).

Test infrastructure: only the tests, the smoke check and the benchmark's
CPU-baseline leg use this module. The library never does.

Follows sec. 3 of Kruchinina, Rudberg, Rubensson (2015): the regular McWeeny
expansion (the general recursive expansion with f_0 centred at mu and
f_i = p_mw(x) = 3x^2 - 2x^3) and the accelerated one, Alg. McW-ACC, with the
stop log(e_i / 4) / log(e_{i-1}) < 1.8 at every step (C_2^mw = C_2^mwa = 4).
Readings:

* R23 mu and the gap estimate xi are inputs (the paper's Alg. McW-ACC takes
      them as given); gamma = 2 max(lambda_max - mu, mu - lambda_min).
* R24 with the Frobenius or mixed norm the accelerated scheme switches the
      stretch off (alpha = 1) once beta_{i-1} < delta = 0.01 and tests the
      stop only from the step after the switch-off (sec. 3: the Frobenius
      estimate can stop too early while the stretch is on); with the spectral
      norm the stop is tested from i = 1 as printed.
* R2 (only when 0 < e_{i-1} < 1), R6, R7 (bounds, divergence), R9, R10 and
  the max_iter cap as in ``oracle.sp2``.
"""
from __future__ import annotations

import math
from typing import Callable, Optional

import numpy as np

from .sp2 import SP2Result, Status, _error, _square, _store, truncate

C_MW = 4.0        # sec. 3: C_2^mw = max over [0,1] of 3 + 4x - 4x^2
Q_TILDE = 1.8
DELTA_MW = 0.01   # R24


def p_mw(x):
    """McWeeny polynomial 3x^2 - 2x^3 (sec. 3)."""
    return 3.0 * x * x - 2.0 * x * x * x


def mw_gamma(lambda_min: float, lambda_max: float, mu: float) -> float:
    """2 max(lambda_max - mu, mu - lambda_min) (sec. 3, f_0)."""
    return 2.0 * max(lambda_max - mu, mu - lambda_min)


def f0_mw(F: np.ndarray, lambda_min: float, lambda_max: float, mu: float) -> np.ndarray:
    """f_0(x) = (mu - x)/gamma + 0.5 applied to F (sec. 3): maps the spectrum
    into [0, 1], occupied states (below mu) above 0.5."""
    n = F.shape[0]
    g = mw_gamma(lambda_min, lambda_max, mu)
    return (mu * np.eye(n) - F) / g + 0.5 * np.eye(n)


def mwa_alpha(beta: float) -> float:
    """Alg. McW-ACC stretch: 3 / sqrt(12 beta^2 - 18 beta + 9)."""
    return 3.0 / math.sqrt(12.0 * beta * beta - 18.0 * beta + 9.0)


def p_mwa(x, beta: float):
    """p_mw(3 (12 beta^2 - 18 beta + 9)^(-1/2) (x - 0.5) + 0.5) (sec. 3)."""
    return p_mw(mwa_alpha(beta) * (x - 0.5) + 0.5)


def mw_order(e_k: float, e_km1: float) -> float:
    """log(e_k / 4) / log(e_{k-1}), NaN where undefined (R2)."""
    if not (0.0 < e_km1 < 1.0) or not (e_k > 0.0):
        return float("nan")
    return math.log(e_k / C_MW) / math.log(e_km1)


def mcweeny(F: np.ndarray, lambda_min: float, lambda_max: float, mu: float,
            xi: Optional[float] = None, norm: str = "fro", tau: float = 0.0,
            max_iter: int = 100,
            perturb: Optional[Callable[[int, np.ndarray], np.ndarray]] = None,
            working: str = "fp64", mixed_block: int = 32) -> SP2Result:
    """McWeeny expansion (xi None) or McW-ACC with gap estimate xi.

    Per step i: X_s = alpha (X~_{i-1} - 0.5 I) + 0.5 I (alpha = 1 for the
    regular expansion), X_i = 3 X_s^2 - 2 X_s^3 with the products formed as
    written, X~_i = X_i + E_i, e_i = ||X~_i - X~_i^2||, stop when
    log(e_i / 4) / log(e_{i-1}) < 1.8. The stretch follows
    beta_s = alpha (beta_{i-1} - 0.5) + 0.5, beta_i = p_mw(beta_s) from
    beta_0 = 0.5 (1 - xi / gamma). Result fields as in ``oracle.sp2.sp2``;
    ``p`` holds the stretch alpha_i per step (alpha_0 = 1 placeholder) and
    ``r`` the observed orders.
    """
    F = np.asarray(F, dtype=np.float64)
    if F.ndim != 2 or F.shape[0] != F.shape[1] or F.shape[0] == 0:
        return SP2Result(None, 0, Status.INVALID_ARG)
    N = F.shape[0]
    if not (lambda_max > lambda_min) or not (lambda_min <= mu <= lambda_max) \
            or max_iter < 1:
        return SP2Result(None, 0, Status.INVALID_ARG)
    gam = mw_gamma(lambda_min, lambda_max, mu)
    accelerate = xi is not None
    if accelerate and not (0.0 < xi <= gam):
        return SP2Result(None, 0, Status.INVALID_ARG)
    if working not in ("fp64", "fp32"):
        raise ValueError(f"unknown working precision {working!r}")
    eye = np.eye(N)

    def error(X):
        S = _square(X, working)
        S = 0.5 * (S + S.T)                             # R9
        return _error(X, S, norm, mixed_block)

    X = _store(truncate(f0_mw(F, lambda_min, lambda_max, mu), tau), working)
    if perturb is not None:
        X = _store(X + perturb(0, X), working)
    res = SP2Result(None, 0, Status.NOT_CONVERGED)
    res.p.append(1.0)
    res.t1.append(float(np.trace(X)))
    res.t2.append(float(np.sum(X * X)))
    if not (math.isfinite(res.t1[0]) and math.isfinite(res.t2[0])):
        res.status, res.X = Status.DIVERGED, X
        return res
    e0 = error(X)
    res.v.append(e0)
    res.r.append(float("nan"))
    if not math.isfinite(e0):
        res.status, res.X = Status.DIVERGED, X
        return res
    if e0 == 0.0:                                       # R6
        res.status, res.X = Status.OK, X
        return res
    beta = 0.5 * (1.0 - xi / gam) if accelerate else 0.0
    stretch_on = accelerate
    first_test = 1 if (not accelerate or norm == "spectral") else None
    for i in range(1, max_iter + 1):
        if stretch_on and norm != "spectral" and beta < DELTA_MW:   # R24
            stretch_on = False
            first_test = i + 1
        a = mwa_alpha(beta) if stretch_on else 1.0
        # the regular expansion applies p_mw to X~ itself; the stretch of
        # Alg. McW-ACC shifts and scales it first
        Xs = _store(a * (X - 0.5 * eye) + 0.5 * eye, working) if stretch_on else X
        S = _square(Xs, working)
        S = _store(0.5 * (S + S.T), working)
        T = Xs @ S if working == "fp64" else \
            (Xs.astype(np.float32) @ S.astype(np.float32)).astype(np.float64)
        T = 0.5 * (T + T.T)
        Xi = truncate(_store(3.0 * S - 2.0 * T, working), tau)
        if perturb is not None:
            Xi = _store(Xi + perturb(i, Xi), working)
        if stretch_on:
            bs = a * (beta - 0.5) + 0.5
            beta = p_mw(bs)
        X = Xi
        res.p.append(a)
        t1, t2 = float(np.trace(X)), float(np.sum(X * X))
        res.t1.append(t1)
        res.t2.append(t2)
        if not (math.isfinite(t1) and math.isfinite(t2)) or t2 > t1 + N:
            res.status, res.X, res.n = Status.DIVERGED, X, i
            return res
        if i >= max_iter:
            res.status, res.X, res.n = Status.NOT_CONVERGED, X, i
            return res
        ei = error(X)
        res.v.append(ei)
        r = mw_order(ei, res.v[i - 1])
        res.r.append(r)
        if not math.isfinite(ei):
            res.status, res.X, res.n = Status.DIVERGED, X, i
            return res
        if ei == 0.0:                                   # R6
            res.status, res.X, res.n = Status.OK, X, i
            return res
        if first_test is not None and i >= first_test and not math.isnan(r) \
                and r < Q_TILDE:
            res.status, res.X, res.n = Status.OK, X, i
            return res
    return res


__all__ = ["C_MW", "DELTA_MW", "p_mw", "mw_gamma", "f0_mw", "mwa_alpha", "p_mwa",
           "mw_order", "mcweeny"]
