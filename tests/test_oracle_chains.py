"""Pins of the real-coupling chains of the oracle (derivatives of ln Z).

* The enumeration of bond moments with per-bond couplings reduces, for J = 1,
  to the energy of an independent enumeration and of Kaufman's exact ln Z.
* Its derivatives obey d ln Z / d J_b = beta <x_b> and
  d <x_a> / d J_b = beta Cov(x_a, x_b) (checked by central differences of
  the enumeration itself, so a wrong sign, index or transposition fails).
* The oracle's chains reproduce the exact means and covariances at L = 4
  within their statistical errors, and follow the single-lattice chains
  (replica k) step for step.
"""
import numpy as np
import pytest

import oracle.exact as ex

L4 = 4


@pytest.fixture(scope="module")
def x4():
    return ex.torus_bond_products(L4)


def test_uniform_couplings_reduce_to_enumerated_and_kaufman_energy(x4):
    beta = 0.37
    mean, _, lnZ = ex.exact_bond_moments(L4, np.ones((2, 16)), beta, x4)
    E, M = ex.enumerate_torus(L4)
    e, _, _, lnZ_enum = ex.canonical_means(E, M, beta, 16)
    assert abs(-mean.sum() / 16 - e) < 1e-12
    assert abs(lnZ - lnZ_enum) < 1e-10
    assert abs(-mean.sum() / 16 - ex.kaufman_energy(L4, beta)) < 1e-12


def test_derivatives_of_ln_z_by_central_differences(x4):
    rng = np.random.default_rng(3)
    J = rng.normal(1.0, 0.3, size=(2, 16))
    beta, eps = 0.41, 1e-5
    mean, cov, _ = ex.exact_bond_moments(L4, J, beta, x4)
    for b in (0, 7, 16, 31):
        Jp, Jm = J.copy(), J.copy()
        Jp.reshape(-1)[b] += eps
        Jm.reshape(-1)[b] -= eps
        mp_, _, lp = ex.exact_bond_moments(L4, Jp, beta, x4)
        mm_, _, lm = ex.exact_bond_moments(L4, Jm, beta, x4)
        assert abs((lp - lm) / (2 * eps) - beta * mean.reshape(-1)[b]) < 1e-8
        fd = (mp_ - mm_).reshape(-1) / (2 * eps)
        assert np.abs(fd - beta * cov[:, b]).max() < 1e-8
    # d ln Z / d beta = sum_b J_b <x_b>
    _, _, lp = ex.exact_bond_moments(L4, J, beta + eps, x4)
    _, _, lm = ex.exact_bond_moments(L4, J, beta - eps, x4)
    assert abs((lp - lm) / (2 * eps) - (J * mean).sum()) < 1e-7


def test_bond_covariance_is_the_sample_covariance(oracle_mod):
    rng = np.random.default_rng(5)
    s = rng.choice(np.array([-1, 1], dtype=np.int8), size=(3, 50, 2, 9))
    g = rng.normal(size=(2, 9))
    got = oracle_mod.bond_covariance(s, g)
    X = s.reshape(150, 18).astype(np.float64)
    G = X @ g.reshape(-1)
    want = np.cov(np.vstack([G, X.T]), bias=True)[0, 1:]
    assert np.allclose(got.reshape(-1), want, rtol=0, atol=1e-12)


def test_chains_follow_single_lattice_chains(oracle_mod):
    d, L, seed, beta, n = 2, 8, 17, 0.45, 12
    rng = np.random.default_rng(8)
    J = rng.normal(1.0, 0.2, size=(d, L ** d)).astype(np.float32)
    s0 = np.stack([oracle_mod.init_ising(d, L, seed, replica=10 + k) for k in range(3)])
    out, bsum, samples, _ = oracle_mod.chains_ising(d, L, seed, J, beta, s0, n, t0=5,
                                                    replica0=10, want_samples=True)
    assert np.array_equal(samples.astype(np.int64).sum(axis=(0, 1)), bsum)
    for k in range(3):
        ref = oracle_mod.OracleLattice(d, 1, L, seed, J_kind=2, J=J, replica=10 + k, spins=s0[k])
        ref.t = 5
        for w in range(n):
            ref.sweep(beta, 1)
            acc = np.zeros((d, L ** d), dtype=np.int64)
            ref.bond_accumulate(acc)
            assert np.array_equal(samples[k, w].astype(np.int64), acc), (k, w)
        assert np.array_equal(ref.s, out[k])


def test_chains_reproduce_exact_moments_at_L4(oracle_mod, x4):
    rng = np.random.default_rng(11)
    J = rng.normal(1.0, 0.3, size=(2, 16)).astype(np.float32)
    beta, nch, nsw = 0.35, 48, 1500
    mean, cov, _ = ex.exact_bond_moments(L4, J.astype(np.float64), beta, x4)
    s0 = np.stack([oracle_mod.init_ising(2, L4, 2, replica=k) for k in range(nch)])
    st, _, _, _ = oracle_mod.chains_ising(2, L4, 2, J, beta, s0, 100)  # burn-in
    _, bsum, samples, _ = oracle_mod.chains_ising(2, L4, 2, J, beta, st, nsw, t0=100,
                                                  want_samples=True)
    per_chain = samples.astype(np.float64).mean(axis=1)  # [nch, 2, 16]
    est = per_chain.mean(axis=0)
    err = per_chain.std(axis=0, ddof=1) / np.sqrt(nch)
    assert np.allclose(est, bsum / (nch * nsw))
    assert np.all(np.abs(est - mean) < 5 * err + 1e-12), np.max(np.abs(est - mean) / err)
    g = rng.normal(size=(2, 16))
    want = (cov @ g.reshape(-1)).reshape(2, 16)
    parts = np.stack([oracle_mod.bond_covariance(samples[k::8], g) for k in range(8)])
    got = oracle_mod.bond_covariance(samples, g)
    cerr = parts.std(axis=0, ddof=1) / np.sqrt(8)
    assert np.all(np.abs(got - want) < 5 * cerr + 1e-3), np.max(np.abs(got - want) / cerr)
