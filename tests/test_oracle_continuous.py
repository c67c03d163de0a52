"""Pins for the oracle's XY / Heisenberg updates (CPU only).

* Single spin in a frozen field: only colour 0 is updated, so every colour-0
  spin sees the fixed field h = 2 d J of its aligned colour-1 neighbours; its
  long-time mean along h must be tanh(beta h) (Ising), I1/I0(beta h) (XY) or
  coth(beta h) - 1/(beta h) (Heisenberg).  This fixes the proposal's symmetry
  and the acceptance rule of Eq. (2) for continuous spins.
* beta = 0: every proposal is accepted, so one half-sweep shows the proposal
  distribution itself: XY rotation angles uniform in [-delta, delta],
  Heisenberg cos(angle) uniform in [cos delta, 1]; lengths preserved.
* Energy identity: E(after) - E(before) = sum of accepted dE.
* |s| = 1 after renormalisation.
* Small-beta expansion of the lattice energy.
"""
import numpy as np
import pytest
from scipy.stats import kstest

import oracle.exact as ex


def _frozen_field_mean(oracle_mod, d, n, L, beta, delta, steps, seed=5):
    lat = oracle_mod.OracleLattice(d, n, L, seed, init="cold", delta=delta, renorm_every=0)
    N = L ** d
    col0 = np.array([sum((i // L ** a) % L for a in range(d)) % 2 == 0 for i in range(N)])
    acc = np.zeros(col0.sum())
    for t in range(200):  # equilibrate
        lat.half_sweep(beta, 0, t)
    for t in range(200, 200 + steps):
        lat.half_sweep(beta, 0, t)
        proj = lat.s[col0] if n == 1 else lat.s[0][col0]
        acc += proj
    per_site = acc / steps
    return per_site.mean(), per_site.std(ddof=1) / np.sqrt(len(per_site))


@pytest.mark.parametrize("d,n,L,beta,delta,exact", [
    (2, 1, 32, 0.1, 0.0, lambda bh: ex.ising_single_spin_mean(bh)),
    (2, 2, 32, 0.3, 1.0, lambda bh: ex.xy_single_spin_mean(bh)),
    (2, 2, 32, 0.15, 2.5, lambda bh: ex.xy_single_spin_mean(bh)),
    (3, 3, 8, 0.2, 1.5, lambda bh: ex.heisenberg_single_spin_mean(bh)),
    (2, 3, 32, 0.25, 1.0, lambda bh: ex.heisenberg_single_spin_mean(bh)),
])
def test_single_spin_in_frozen_field(oracle_mod, d, n, L, beta, delta, exact):
    m, se = _frozen_field_mean(oracle_mod, d, n, L, beta, delta, steps=3000)
    want = exact(beta * 2 * d)
    assert abs(m - want) < 4 * se + 1e-12, (m, want, se)


def test_xy_beta_zero_rotation_is_uniform(oracle_mod):
    delta = 0.7
    lat = oracle_mod.OracleLattice(2, 2, 64, 9, delta=delta, renorm_every=0)
    s0 = lat.s.copy()
    st = lat.half_sweep(0.0, 0, 0)
    assert st.n_accept == st.n_attempt
    N = 64 * 64
    col0 = np.array([((i % 64) + (i // 64)) % 2 == 0 for i in range(N)])
    ang = np.arctan2(s0[0] * lat.s[1] - s0[1] * lat.s[0], (s0 * lat.s).sum(axis=0))[col0]
    assert np.all(np.abs(ang) <= delta + 1e-12)
    assert kstest(ang, "uniform", args=(-delta, 2 * delta)).pvalue > 1e-4
    assert np.allclose(np.sqrt((lat.s ** 2).sum(axis=0)), np.sqrt((s0 ** 2).sum(axis=0)),
                       atol=1e-14)
    assert np.array_equal(lat.s[:, ~col0], s0[:, ~col0])


def test_heisenberg_beta_zero_cap_is_uniform(oracle_mod):
    delta = 1.2
    lat = oracle_mod.OracleLattice(3, 3, 16, 13, delta=delta, renorm_every=0)
    s0 = lat.s.copy()
    lat.half_sweep(0.0, 1, 0)
    N = 16 ** 3
    col1 = np.array([((i % 16) + (i // 16) % 16 + i // 256) % 2 == 1 for i in range(N)])
    n0 = np.sqrt((s0 ** 2).sum(axis=0))
    cosang = ((s0 * lat.s).sum(axis=0) / n0 / np.sqrt((lat.s ** 2).sum(axis=0)))[col1]
    assert kstest(cosang, "uniform", args=(np.cos(delta), 1 - np.cos(delta))).pvalue > 1e-4
    assert np.allclose(np.sqrt((lat.s ** 2).sum(axis=0)), 1.0, atol=1e-6)
    # the azimuth about s0 is uniform: the mean of s' - (s'.s0) s0 vanishes
    perp = (lat.s - (lat.s * s0).sum(axis=0) * s0)[:, col1]
    assert np.all(np.abs(perp.mean(axis=1)) < 4 * perp.std(axis=1) / np.sqrt(col1.sum()))


@pytest.mark.parametrize("d,n,L,beta,delta,kind", [(2, 2, 16, 1.12, 1.0, 0), (3, 3, 8, 0.693, 1.0, 0),
                                                   (2, 3, 12, 0.8, 0.6, 2), (3, 2, 6, 0.5, 2.0, 1)])
def test_continuous_energy_identity(oracle_mod, d, n, L, beta, delta, kind):
    lat = oracle_mod.OracleLattice(d, n, L, 17, delta=delta, J_kind=kind, J0=1.0, J_sigma=0.2)
    for t in range(6):
        for c in (0, 1):
            e0 = lat.measure().E
            st = lat.half_sweep(beta, c, t)
            e1 = lat.measure().E
            assert abs((e1 - e0) - st.dE) < 1e-9 * max(1.0, abs(e0))
            assert 0 < st.n_accept < st.n_attempt


def test_renormalisation_restores_unit_length(oracle_mod):
    lat = oracle_mod.OracleLattice(2, 3, 16, 3, delta=1.0, renorm_every=5)
    lat.s *= 1.001
    lat.sweep(0.7, 5)
    assert np.allclose(np.sqrt((lat.s ** 2).sum(axis=0)), 1.0, atol=1e-12)


@pytest.mark.parametrize("d,n,single", [(2, 2, ex.xy_single_spin_mean),
                                        (3, 3, ex.heisenberg_single_spin_mean)])
def test_small_beta_energy(oracle_mod, d, n, single):
    beta = 0.05
    L = 32 if d == 2 else 12
    lat = oracle_mod.OracleLattice(d, n, L, 23, delta=3.0)
    lat.sweep(beta, 50)
    series, _ = lat.sweep(beta, 400, 1)
    e = np.array([o.E for o in series]) / L ** d
    m = e.mean()
    se = e.std(ddof=1) / np.sqrt(len(e)) * 3  # generous: allow autocorrelation
    want = -d * single(beta)  # leading order of the high-temperature expansion
    assert abs(m - want) < 4 * se + 5 * beta ** 3, (m, want, se)
