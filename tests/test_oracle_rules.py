"""Pins of the oracle's heat-bath rule and tiled k-hit schedule (Sec. 2).

* Heat-bath thresholds equal ceil(2^32 / (1 + exp(-2 beta h))) evaluated in
  mpmath.
* The plain Metropolis schedule of the rule/schedule code reproduces the
  oracle's pinned Metropolis chain step for step.
* Heat bath forgets the old spin: two states that differ only on colour 0
  are identical after one sweep (Metropolis keeps them apart).
* One heat-bath update in a frozen field gives +1 with probability p_+.
* Heat bath, and both rules under the tiled k-hit schedule, sample the
  Boltzmann distribution of the 4 x 4 torus: long-run means of E and |M|
  equal the exact enumeration within their errors.
"""
import math

import mpmath as mp
import numpy as np
import pytest

import oracle.exact as ex


@pytest.mark.parametrize("beta,h", [(0.3, 4), (0.4406868, -2), (1.7, 2), (0.05, -6), (2.5, 0)])
def test_heatbath_threshold_matches_mpmath(oracle_mod, beta, h):
    with mp.workdps(50):
        want = int(mp.ceil(mp.ldexp(1 / (1 + mp.e ** (-2 * mp.mpf(beta) * h)), 32)))
    assert oracle_mod.threshold_hb(beta, h) == min(want, 2 ** 32)
    assert oracle_mod.threshold_hb(float("inf"), 2) == 2 ** 32
    assert oracle_mod.threshold_hb(float("inf"), -2) == 0
    assert oracle_mod.threshold_hb(0.0, 3) == 2 ** 31


@pytest.mark.parametrize("d,L,kind", [(2, 16, 0), (3, 8, 1), (2, 10, 1)])
def test_plain_metropolis_equals_the_pinned_chain(oracle_mod, d, L, kind):
    a = oracle_mod.OracleLattice(d, 1, L, 4, J_kind=kind)
    b = oracle_mod.OracleLattice(d, 1, L, 4, J_kind=kind)
    a.sweep(0.44, 7)
    b.sweep_rule(0.44, 7, "metropolis")
    assert np.array_equal(a.s, b.s)


def _colour0(d, L):
    i = np.arange(L ** d)
    x, y, z = i % L, (i // L) % L, i // (L * L) if d == 3 else 0 * i
    return ((x + y + z) & 1) == 0


def test_heatbath_forgets_the_old_spin(oracle_mod):
    d, L = 2, 32
    base = oracle_mod.OracleLattice(d, 1, L, 5)
    c0 = _colour0(d, L)
    s_b = base.s.copy()
    s_b[c0] = -s_b[c0]
    for rule, same in (("heatbath", True), ("metropolis", False)):
        a = oracle_mod.OracleLattice(d, 1, L, 5, spins=base.s)
        b = oracle_mod.OracleLattice(d, 1, L, 5, spins=s_b)
        a.sweep_rule(0.5, 1, rule)
        b.sweep_rule(0.5, 1, rule)
        assert np.array_equal(a.s, b.s) == same, rule


def test_heatbath_update_in_a_frozen_field(oracle_mod):
    d, L, beta = 2, 256, 0.2
    lat = oracle_mod.OracleLattice(d, 1, L, 6, init="cold")
    lat.sweep_rule(beta, 1, "heatbath")
    c0 = _colour0(d, L)
    up = (lat.s[c0] > 0).mean()
    p = 1 / (1 + math.exp(-2 * beta * 4))  # all four neighbours +1
    se = math.sqrt(p * (1 - p) / c0.sum())
    assert abs(up - p) < 5 * se


def _binned(x, nb=50):
    x = np.asarray(x, dtype=np.float64)
    m = len(x) // nb
    b = x[: m * nb].reshape(nb, m).mean(axis=1)
    return b.mean(), b.std(ddof=1) / math.sqrt(nb)


@pytest.mark.parametrize("rule,tile,hits", [("heatbath", 0, 1), ("heatbath", 2, 3),
                                            ("metropolis", 2, 4)])
def test_rules_and_schedules_sample_the_boltzmann_distribution(oracle_mod, rule, tile, hits):
    L, beta = 4, 0.35
    E_all, M_all = ex.enumerate_torus(L)
    e_ex, m_ex, _, _ = ex.canonical_means(E_all, M_all, beta, L * L)
    lat = oracle_mod.OracleLattice(2, 1, L, 17)
    lat.sweep_rule(beta, 200, rule, tile, hits)
    es, ms = [], []
    for _ in range(30000):
        lat.sweep_rule(beta, 1, rule, tile, hits)
        o = lat.measure()
        es.append(o.E_int / 16)
        ms.append(o.absM / 16)
    e, se = _binned(es)
    m, sm = _binned(ms)
    assert abs(e - e_ex) < 5 * se, (e, e_ex, se)
    assert abs(m - m_ex) < 5 * sm, (m, m_ex, sm)
