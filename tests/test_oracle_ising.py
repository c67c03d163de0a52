"""Pins for the oracle's Ising chain (CPU only).

Each check fixes a different part of the oracle against something other than
itself:
* beta = 0 (every move accepted: one sweep maps s -> -s exactly) and
  beta = infinity (energy never rises; the ground state is a fixed point);
* the integer identity E(after) - E(before) = 2 * sum of accepted m_i per
  half-sweep, tying the update's local field to the bond-sum energy of Eq. (1);
* E mod 4 and M mod 2 invariants;
* the oracle's energy of random 4 x 4 states equals brute-force enumeration,
  itself pinned to Kaufman's exact partition function;
* the distribution of oracle chains after a few sweeps from a fixed start
  equals exact propagation of Eq. (2) over all 2^16 (or 2^8) states (chi^2);
* detailed balance / stationarity of the exact chain itself;
* long-run averages against enumeration (4 x 4) and Kaufman (8 x 8, 16 x 16).
"""
import numpy as np
import pytest
from scipy.stats import chi2

import oracle.exact as ex

BETA_C2 = 0.4406868


def _lat(oracle_mod, d, L, seed=1, **kw):
    return oracle_mod.OracleLattice(d, 1, L, seed, **kw)


@pytest.mark.parametrize("d,L,kind", [(2, 8, 0), (2, 6, 1), (3, 4, 0), (3, 2, 1), (2, 2, 0)])
def test_beta_zero_flips_everything(oracle_mod, d, L, kind):
    lat = _lat(oracle_mod, d, L, J_kind=kind)
    s0 = lat.s.copy()
    o0 = lat.measure()
    _, st = lat.sweep(0.0, 1)
    assert np.array_equal(lat.s, -s0)
    o1 = lat.measure()
    assert o1.E_int == o0.E_int and o1.M_int == -o0.M_int
    assert st.n_accept == st.n_attempt == lat.N


@pytest.mark.parametrize("d,L", [(2, 16), (3, 6)])
def test_beta_infinity_quench(oracle_mod, d, L):
    lat = _lat(oracle_mod, d, L, seed=7)
    e_prev = lat.measure().E_int
    for t in range(20):
        for c in (0, 1):
            lat.half_sweep(float("inf"), c, t)
            e = lat.measure().E_int
            assert e <= e_prev
            e_prev = e
    cold = _lat(oracle_mod, d, L, init="cold")
    s0 = cold.s.copy()
    cold.sweep(float("inf"), 3)
    assert np.array_equal(cold.s, s0)


@pytest.mark.parametrize("d,L,kind,beta", [(2, 8, 0, BETA_C2), (2, 10, 1, 0.7), (3, 4, 0, 0.2216546),
                                           (3, 6, 1, 1.0), (2, 2, 0, 0.3), (3, 2, 1, 0.5)])
def test_energy_identity_per_half_sweep(oracle_mod, d, L, kind, beta):
    lat = _lat(oracle_mod, d, L, seed=3, J_kind=kind)
    for t in range(10):
        for c in (0, 1):
            e0 = lat.measure()
            st = lat.half_sweep(beta, c, t)
            e1 = lat.measure()
            assert e1.E_int - e0.E_int == 2 * st.dE_units
            assert st.n_attempt == lat.N // 2
            assert e1.E_int % 4 == e0.E_int % 4
            assert (e1.M_int - lat.N) % 2 == 0


def test_energy_of_states_matches_enumeration(oracle_mod):
    E, M = ex.enumerate_torus(4)
    rng = np.random.default_rng(0)
    for idx in rng.choice(len(E), size=300, replace=False):
        spins = np.array([1 - 2 * ((idx >> i) & 1) for i in range(16)], dtype=np.int8)
        lat = _lat(oracle_mod, 2, 4, spins=spins)
        o = lat.measure()
        assert o.E_int == E[idx] and o.M_int == M[idx]


def test_enumeration_matches_kaufman():
    E, M = ex.enumerate_torus(4)
    for beta in (0.2, BETA_C2, 0.7):
        lnZ = ex.canonical_means(E, M, beta, 16)[3]
        assert abs(lnZ - float(ex.kaufman_lnZ(4, 4, beta))) < 1e-12
        assert abs(ex.canonical_means(E, M, beta, 16)[0] - ex.kaufman_energy(4, beta)) < 1e-12


def test_onsager_limits():
    assert abs(ex.onsager_beta_c() - 0.440686793509772) < 1e-15
    assert abs(ex.onsager_energy(0.4) - ex.kaufman_energy(256, 0.4)) < 1e-12
    assert abs(ex.onsager_energy(ex.onsager_beta_c() + 1e-9) + np.sqrt(2)) < 1e-6


def test_exact_chain_is_stationary_and_balanced():
    for chain in (ex.SmallLatticeChain(2, 4, BETA_C2), ex.SmallLatticeChain(3, 2, 0.3)):
        pi = chain.boltzmann()
        for c in (0, 1):
            assert np.abs(chain.half_sweep(pi, c) - pi).max() < 1e-15
        # detailed balance of one half-sweep on a handful of state pairs
        rng = np.random.default_rng(1)
        for x in rng.integers(0, len(pi), size=20):
            delta = np.zeros(len(pi))
            delta[x] = 1.0
            row = chain.half_sweep(delta, 0)  # P_0(x, .)
            for y in np.nonzero(row > 0)[0][:10]:
                dy = np.zeros(len(pi))
                dy[y] = 1.0
                back = chain.half_sweep(dy, 0)[x]  # P_0(y, x)
                assert abs(pi[x] * row[y] - pi[y] * back) <= 1e-12 * max(pi[x] * row[y], 1e-300)


def _chi2_states(samples_idx, p_exact, min_expected=5.0):
    n = len(samples_idx)
    counts = np.bincount(samples_idx, minlength=len(p_exact)).astype(np.float64)
    exp_c = p_exact * n
    big = exp_c >= min_expected
    obs = np.append(counts[big], counts[~big].sum())
    expv = np.append(exp_c[big], exp_c[~big].sum())
    keep = expv > 0
    stat = ((obs[keep] - expv[keep]) ** 2 / expv[keep]).sum()
    dof = keep.sum() - 1
    return stat, dof


@pytest.mark.parametrize("d,L,kind,beta,sweeps", [(2, 4, 0, BETA_C2, 1), (2, 4, 0, BETA_C2, 3),
                                                  (2, 4, 1, 0.8, 2), (3, 2, 0, 0.3, 2)])
def test_ensemble_matches_exact_propagation(oracle_mod, d, L, kind, beta, sweeps):
    lat = _lat(oracle_mod, d, L, seed=11, J_kind=kind)
    J = None if kind == 0 else lat.J
    chain = ex.SmallLatticeChain(d, L, beta, J=J)
    start = ex.state_index(lat.s)
    pi = np.zeros(1 << lat.N)
    pi[start] = 1.0
    for _ in range(sweeps):
        pi = chain.sweep(pi)
    n_chains = 200_000
    out = lat.ensemble(beta, sweeps, n_chains)
    idx = ex.state_index(out)
    stat, dof = _chi2_states(idx, pi)
    assert stat < chi2.ppf(1 - 1e-4, dof), (stat, dof)


def _binned_mean(x, nbins=50):
    x = np.asarray(x, dtype=np.float64)
    m = len(x) // nbins
    b = x[: m * nbins].reshape(nbins, m).mean(axis=1)
    return b.mean(), b.std(ddof=1) / np.sqrt(nbins)


def test_long_run_4x4_against_enumeration(oracle_mod):
    E, M = ex.enumerate_torus(4)
    e_ex, m_ex, _, _ = ex.canonical_means(E, M, BETA_C2, 16)
    lat = _lat(oracle_mod, 2, 4, seed=21)
    lat.sweep(BETA_C2, 200)
    series, _ = lat.sweep(BETA_C2, 100_000, 1)
    e = [o.E_int / 16 for o in series]
    m = [o.absM / 16 for o in series]
    me, se = _binned_mean(e)
    mm, sm = _binned_mean(m)
    assert abs(me - e_ex) < 4 * se, (me, e_ex, se)
    assert abs(mm - m_ex) < 4 * sm, (mm, m_ex, sm)


@pytest.mark.parametrize("L,beta,sweeps", [(8, 0.4, 40_000), (16, BETA_C2, 30_000)])
def test_long_run_against_kaufman(oracle_mod, L, beta, sweeps):
    lat = _lat(oracle_mod, 2, L, seed=31)
    lat.sweep(beta, 2000)
    series, _ = lat.sweep(beta, sweeps, 1)
    e = [o.E_int / L ** 2 for o in series]
    me, se = _binned_mean(e, nbins=40)
    ek = ex.kaufman_energy(L, beta)
    assert abs(me - ek) < 4 * se, (me, ek, se)


def test_long_run_3d_l2_against_enumeration(oracle_mod):
    chain = ex.SmallLatticeChain(3, 2, 0.3)
    pi = chain.boltzmann()
    e_ex = float((pi * chain.E).sum()) / 8
    lat = _lat(oracle_mod, 3, 2, seed=41)
    series, _ = lat.sweep(0.3, 100_000, 1)
    me, se = _binned_mean([o.E_int / 8 for o in series])
    assert abs(me - e_ex) < 4 * se


def test_bond_correlations_sum_and_mean(oracle_mod):
    lat = _lat(oracle_mod, 2, 4, seed=51)
    acc = np.zeros((2, 16), dtype=np.int64)
    lat.bond_accumulate(acc)
    assert acc.sum() == -lat.measure().E_int
    # long-run per-bond mean equals the exact nearest-neighbour correlation
    E, M = ex.enumerate_torus(4)
    e_ex = ex.canonical_means(E, M, BETA_C2, 16)[0]
    nn_exact = -e_ex / 2  # every bond is equivalent on the torus
    acc[:] = 0
    n = 20_000
    per = []
    for k in range(n):
        lat.sweep(BETA_C2, 1)
        before = acc.copy()
        lat.bond_accumulate(acc)
        per.append((acc - before).mean())
    mb, sb = _binned_mean(per)
    assert abs(acc.mean() / n - nn_exact) < 4 * sb + 1e-12
    assert abs(mb - nn_exact) < 4 * sb
