"""The replay of a run's scalar decisions (tests/stop_replay.py) that every
GPU run of the suite goes through: it accepts the oracle's own histories
(Alg. 2, Alg. 4, the McWeeny expansion of sec. 3) and rejects histories with
a planted wrong decision: a polynomial that the trace test does not pick, an
order that is not log(v_k/C)/log(v_{k-2}), a run that goes past a firing of
the stop, and a run that ends where the stop does not fire."""
import copy

import pytest

import oracle
from oracle.mcweeny import mcweeny
from tests.stop_replay import mcweeny_first_step, replay
from workloads import config_small, dense_instance


@pytest.fixture(scope="module")
def small():
    return config_small()


@pytest.mark.parametrize("working", ["fp64", "fp32", "bf16x3"])
def test_oracle_runs_replay(small, working):
    ref = oracle.sp2(small.F, small.lambda_min, small.lambda_max, small.n_occ,
                     working=working)
    assert ref.status == oracle.Status.OK
    assert replay(ref, small.n_occ) == ref.n + 1


def test_literal_rule_and_not_converged_replay(small):
    ref = oracle.sp2(small.F, small.lambda_min, small.lambda_max, small.n_occ,
                     branch="literal", max_iter=12)
    assert ref.status == oracle.Status.NOT_CONVERGED
    replay(ref, small.n_occ, branch="literal")


def test_schedule_and_mcweeny_runs_replay(small):
    h, l = float(small.lam[small.n_occ - 1]), float(small.lam[small.n_occ])
    sched = oracle.acc_schedule(small.lambda_min, small.lambda_max, h, h, l, l)
    ref = oracle.sp2_acc(small.F, small.lambda_min, small.lambda_max, sched)
    assert ref.status == oracle.Status.OK
    replay(ref, small.n_occ, schedule=sched)
    mu, xi = 0.5 * (h + l), l - h
    for x in (None, xi):
        mw = mcweeny(small.F, small.lambda_min, small.lambda_max, mu, x)
        assert mw.status == oracle.Status.OK
        first = mcweeny_first_step(small.lambda_min, small.lambda_max, mu, x)
        assert (first == 1) == (x is None)
        replay(mw, small.n_occ, method="mcweeny", mw_first=first)


def test_planted_wrong_decisions_are_caught():
    inst = dense_instance(256, 128, -1.0, 1.0, 0.1, seed=21)
    ref = oracle.sp2(inst.F, inst.lambda_min, inst.lambda_max, inst.n_occ)
    assert ref.status == oracle.Status.OK and ref.n > 6
    replay(ref, inst.n_occ)
    # a polynomial the trace test does not pick
    bad = copy.deepcopy(ref)
    bad.p[3] = 1 - bad.p[3]
    with pytest.raises(AssertionError):
        replay(bad, inst.n_occ)
    # an observed order that is not the one of the returned errors
    bad = copy.deepcopy(ref)
    bad.r[ref.n - 1] *= 1.0 + 1e-9
    with pytest.raises(AssertionError):
        replay(bad, inst.n_occ)
    # the run went on past the step where the stop fires
    bad = copy.deepcopy(ref)
    bad.status = oracle.Status.NOT_CONVERGED
    with pytest.raises(AssertionError, match="went past"):
        replay(bad, inst.n_occ)
    # the run ends one step before the stop fires
    bad = copy.deepcopy(ref)
    bad.n = ref.n - 1
    bad.v, bad.r = ref.v[:ref.n], ref.r[:ref.n]
    with pytest.raises(AssertionError, match="did not fire"):
        replay(bad, inst.n_occ)
