"""Replay of the scalar decisions of a run on the history the GPU returned.

The finalize kernel takes three kinds of scalar decisions per step from the
FP64 values it accumulated: the observed order r_k (sec. 2), the polynomial
of the next step (Alg. 2's trace test, or the schedule of Alg. 3), and the
stop (Alg. 2 / Alg. 4, or the McWeeny test of sec. 3). Given the run's own
history (v or the error in the norm the stop read, the traces t1, t2, the
polynomials p, the orders r), each of these decisions is fixed exactly by
the oracle's scalar functions. This module replays them and asserts that the
device took the same ones at every step: no earlier firing of the stop was
missed, the stop fired where the run ended, and every polynomial choice is
the one the rule gives for the GPU's own traces. Test code only.
"""
from __future__ import annotations

import math
from types import SimpleNamespace

import oracle
from oracle.mcweeny import mw_order

# r_k is log(e_k / C) / log(e_{k-2}) on both sides; the device's log may
# differ from the host's by an ulp.
ORDER_RTOL = 1e-12
# stop decisions within this distance of q~ = 1.8 are not replayed (the
# two logarithms could legitimately round to opposite sides)
EDGE = 1e-12


def _hist(res):
    if isinstance(res, dict):
        return SimpleNamespace(**res)
    return res


def _order(e, k, method):
    if method == "mcweeny":
        return mw_order(e[k], e[k - 1]) if k >= 1 else float("nan")
    return oracle.observed_order(e[k], e[k - 2]) if k >= 2 else float("nan")


def replay(res, n_occ, *, n=None, status=None, branch="nearest", e=None,
           schedule=None, method="sp2", mw_first=1):
    """Asserts that the run's orders, polynomial choices and stop equal the
    oracle's decisions on the run's own history.

    res: a Result of the binding (or a dict/namespace with v, t1, t2, p, r
    and, unless given as arguments, n and status). e: the error history the
    stop read (the mixed or spectral norm; default the Frobenius v).
    schedule: an Alg. 3 schedule (oracle.acc_schedule) for SP2-ACC runs.
    method: "sp2" (Alg. 2 / Alg. 4) or "mcweeny" (sec. 3), whose stop is
    tested from step mw_first on. Returns the number of steps replayed.
    """
    h = _hist(res)
    n = h.n if n is None else n
    status = h.status if status is None else status
    v = list(h.v)
    e = v if e is None else list(e)
    p, r, t1, t2 = list(h.p), list(h.r), list(h.t1), list(h.t2)
    ok = (status == 0)
    if not v:                     # n_occ = 0 or n: no square was computed
        assert n == 0
        return 0
    assert len(e) >= len(v) and len(r) >= len(v)
    if ok and v[n] != 0.0:
        assert len(v) == n + 1, (len(v), n)

    # observed orders
    for k in range(len(v)):
        exp = _order(e, k, method)
        got = r[k]
        if math.isnan(exp) or not math.isfinite(e[k]):
            assert math.isnan(got) or not math.isfinite(e[k]), (k, got, exp)
        else:
            assert abs(got - exp) <= ORDER_RTOL * abs(exp), (k, got, exp)

    # polynomial choices: p[k + 1] was chosen from the traces of X~_k
    if method == "sp2":
        for k in range(len(p) - 1):
            if p[k + 1] < 0:
                continue
            if schedule is not None:
                want = (schedule.p[k + 1] if k + 1 <= schedule.n_max
                        else 1 - p[k])
            else:
                want = oracle.choose_polynomial(t1[k], t2[k], n_occ, branch)
            assert p[k + 1] == want, (k + 1, p[k + 1], want, t1[k], t2[k])

    # stop decisions: the test ran at every k < len(v) and fired only at n
    kmin = schedule.n_min if schedule is not None else 2
    for k in range(len(v)):
        rk = _order(e, k, method)
        if not math.isnan(rk) and abs(rk - oracle.Q_TILDE) < EDGE:
            continue
        if method == "mcweeny":
            fires = k >= mw_first and not math.isnan(rk) and rk < oracle.Q_TILDE
        else:
            fires = (k >= kmin and p[k] != p[k - 1] and not math.isnan(rk)
                     and rk < oracle.Q_TILDE)
        if ok and k == n:
            special = v[k] == 0.0 or (schedule is not None and k >= schedule.n_max)
            assert fires or special, ("stop did not fire where the run ended", k, rk)
        else:
            assert not fires, ("the stop fires at a step the run went past", k, rk, n)
    return len(v)


def mcweeny_first_step(lambda_min, lambda_max, mu, xi, norm="fro") -> int:
    """First step whose error the McWeeny stop tests (sec. 3, reading R24):
    1 for the regular expansion and for McW-ACC with the spectral norm;
    otherwise the step after the one where beta first falls below 0.01
    (the stretch is switched off there), following the scalar recursion
    beta_i = p_mw(alpha_i (beta_{i-1} - 1/2) + 1/2) from
    beta_0 = (1 - xi / gamma) / 2."""
    from oracle.mcweeny import DELTA_MW, mw_gamma, mwa_alpha, p_mw
    if xi is None or norm == "spectral":
        return 1
    beta = 0.5 * (1.0 - xi / mw_gamma(lambda_min, lambda_max, mu))
    for i in range(1, 400):
        if beta < DELTA_MW:
            return i + 1
        a = mwa_alpha(beta)
        beta = p_mw(a * (beta - 0.5) + 0.5)
    raise AssertionError("McW-ACC stretch never switches off")


def replay_run(res, lambda_min, lambda_max, n_occ, opts):
    """replay() with the rule set a run_dense / run_batch call selected:
    opts are that call's keyword arguments (branch, norm, homo_lumo with
    accelerate, mcweeny)."""
    norm = opts.get("norm", "fro")
    e = res.m if norm != "fro" else None
    schedule, method, first = None, "sp2", 1
    if opts.get("homo_lumo") is not None:
        schedule = oracle.acc_schedule(lambda_min, lambda_max, *opts["homo_lumo"],
                                       accelerate=opts.get("accelerate", True))
    if opts.get("mcweeny") is not None:
        mu, xi = opts["mcweeny"]
        method = "mcweeny"
        first = mcweeny_first_step(lambda_min, lambda_max, mu, xi, norm)
    return replay(res, n_occ, branch=opts.get("branch", "nearest"), e=e,
                  schedule=schedule, method=method, mw_first=first)


def replay_batch(results, lambda_min, lambda_max, n_occ, opts):
    """replay_run() for every instance of a run_batch call."""
    hl = opts.get("homo_lumo")
    mw = opts.get("mcweeny")
    total = 0
    for b, res in enumerate(results):
        o = dict(opts)
        if hl is not None:
            o["homo_lumo"] = tuple(seq[b] for seq in hl)
        if mw is not None:
            o["mcweeny"] = (mw[0][b], None if mw[1] is None else mw[1][b])
        total += replay_run(res, lambda_min[b], lambda_max[b], n_occ[b], o)
    return total
