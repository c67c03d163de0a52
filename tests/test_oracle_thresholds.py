"""Pins for the oracle's Boltzmann thresholds T(dE) = ceil(2^32 exp(-beta dE)).

The pre-tabulated Boltzmann factors of Sec. 2 are integer thresholds on a
32-bit uniform; they are checked against mpmath at 60 digits for every
temperature of the workloads and at the special points beta = 0 and infinity.
"""
import math

import mpmath as mp
import pytest

BETAS = [0.4406868, 0.2216546, 0.4, 0.5 * math.log(1 + math.sqrt(2)), 0.05, 1.0, 3.0]
BETAS += [0.5 + 2.5 * k / 31 for k in range(32)]  # the batched spin-glass temperature set


def exact_threshold(beta, dE):
    with mp.workdps(60):
        x = mp.ldexp(mp.e ** (-mp.mpf(beta) * mp.mpf(dE)), 32)
        return min(int(mp.ceil(x)), 2 ** 32)


@pytest.mark.parametrize("beta", BETAS)
def test_thresholds_match_mpmath(oracle_mod, beta):
    for m in range(1, 7):
        for J0 in (1.0, 0.5):
            dE = 2.0 * J0 * m
            assert oracle_mod.threshold(beta, dE) == exact_threshold(beta, dE), (beta, dE)


def test_threshold_special_cases(oracle_mod):
    assert oracle_mod.threshold(0.0, 8.0) == 2 ** 32          # beta = 0: always accept
    assert oracle_mod.threshold(float("inf"), 4.0) == 0       # beta = inf: never uphill
    assert oracle_mod.threshold(1.0, 0.0) == 2 ** 32          # dE <= 0: always
    assert oracle_mod.threshold(1.0, -4.0) == 2 ** 32
    assert oracle_mod.threshold(1e-12, 4.0) == 2 ** 32        # rounds up to 2^32


def test_known_values(oracle_mod):
    # values at the critical temperature of the 2D workload, rederived here
    assert oracle_mod.threshold(0.4406868, 4.0) == exact_threshold(0.4406868, 4.0)
    # monotone in dE
    for beta in BETAS:
        ts = [oracle_mod.threshold(beta, 4.0 * k) for k in range(1, 4)]
        assert ts[0] >= ts[1] >= ts[2]
