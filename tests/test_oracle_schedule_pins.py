"""Pins of three oracle parts that other tests take on trust (CPU only).

* `ising_sweep_sites` (the site-by-site update that supplies the expected
  spins of the full-size late-counter GPU test) equals a whole sweep of the
  oracle's pinned chain on every site, for several shapes, coupling kinds and
  sweep counters up to 2^32 - 1.
* Bond accumulation for continuous spins and real couplings: on hand-built
  twisted states every bond product has a closed form (cos of the twist for
  XY, sin^2 a cos(twist) + cos^2 a for a tilted Heisenberg spiral), and
  sum_b J_b acc_b = -E of Eq. (1) on random states.
* The tiled k-hit schedule of Sec. 2 (two-level checkerboard, k updates of
  the inner checkerboard per tile colour):
  - at beta = 0 every attempt is accepted, so one tiled sweep maps s to
    (-1)^k s -- every site attempted exactly k times;
  - one tile-colour pass leaves the sites of the other tile colour as they
    were, and the two passes in order make one sweep;
  - on 4 x 4 (and 4 x 4 x 4) with 2-site tiles and k = 2 the schedule is
    written out here step by step from the description (tile colour 0 then 1;
    k times colour 0 then colour 1 inside the active tiles; each stage
    updated site by site in a random order, which the checkerboard makes
    equivalent to a simultaneous update), with the random numbers drawn by
    the Philox block function and the thresholds of the pinned tables; the
    oracle must agree, and a schedule with the hit and tile-colour loops
    swapped must not.
"""

import numpy as np
import pytest

import inputs

M32 = 0xFFFFFFFF


def _coords(d, L):
    i = np.arange(L ** d)
    x, y = i % L, (i // L) % L
    z = i // (L * L) if d == 3 else np.zeros_like(i)
    return x, y, z


# ---------------------------------------------------------------------------
# ising_sweep_sites against whole sweeps
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("d,L,kind,t,beta", [
    (2, 16, 0, 0, 0.4406868), (2, 32, 1, 77, 0.7), (3, 8, 0, 123456, 0.2216546),
    (3, 6, 1, 2 ** 32 - 1, 0.5), (2, 12, 2, 5, 0.9), (2, 4, 0, 9, 0.3), (2, 2, 0, 3, 0.3),
    (3, 4, 2, 40000, 0.4)])
def test_sweep_sites_equal_a_whole_sweep(oracle_mod, d, L, kind, t, beta):
    ref = oracle_mod.OracleLattice(d, 1, L, 31, J_kind=kind, J_sigma=0.3)
    sites = np.arange(L ** d)
    got = oracle_mod.ising_sweep_sites(ref, beta, t, sites)
    s_before = ref.s.copy()
    ref.t = t
    ref.sweep(beta, 1)
    assert np.array_equal(got, ref.s)
    # the selection is honoured in any order and with repeats
    sel = np.random.default_rng(d + L).permutation(sites)[: max(3, len(sites) // 3)]
    sel = np.concatenate([sel, sel[:2]])
    again = oracle_mod.OracleLattice(d, 1, L, 31, J_kind=kind, J_sigma=0.3, spins=s_before,
                                     J=ref.J)
    assert np.array_equal(oracle_mod.ising_sweep_sites(again, beta, t, sel), ref.s[sel])
    assert np.array_equal(again.s, s_before)  # the input state is left alone


# ---------------------------------------------------------------------------
# bond accumulation: closed forms and the energy identity
# ---------------------------------------------------------------------------
def test_bond_products_of_a_twisted_xy_state(oracle_mod):
    d, L = 2, 6
    x, y, _ = _coords(d, L)
    th = 2 * np.pi * (x + 2 * y) / L  # +x twist 60 degrees, +y twist 120 degrees
    s = np.stack([np.cos(th), np.sin(th)])
    lat = oracle_mod.OracleLattice(d, 2, L, 1, spins=s, delta=1.0)
    acc = np.zeros((d, L ** d))
    lat.bond_accumulate(acc)
    # the components are cos and sin rounded to double: a few ulp
    assert np.abs(acc[0] - 0.5).max() < 1e-14
    assert np.abs(acc[1] + 0.5).max() < 1e-14
    lat.bond_accumulate(acc)  # accumulates
    assert np.abs(acc[0] - 1.0).max() < 2e-14 and np.abs(acc[1] + 1.0).max() < 2e-14


def test_bond_products_of_a_tilted_heisenberg_spiral(oracle_mod):
    d, L, a = 3, 4, np.pi / 3
    x, y, z = _coords(d, L)
    th = 2 * np.pi * (x + y + 2 * z) / L  # twists 90, 90 and 180 degrees
    s = np.stack([np.sin(a) * np.cos(th), np.sin(a) * np.sin(th), np.full(th.shape, np.cos(a))])
    lat = oracle_mod.OracleLattice(d, 3, L, 1, spins=s, delta=1.0)
    acc = np.zeros((d, L ** d))
    lat.bond_accumulate(acc)
    want = [np.cos(a) ** 2, np.cos(a) ** 2, np.cos(2 * a)]  # 0.25, 0.25, -0.5
    for mu in range(d):
        assert np.abs(acc[mu] - want[mu]).max() < 1e-14, mu


@pytest.mark.parametrize("d,n,L,kind", [(2, 2, 8, 0), (2, 2, 6, 2), (3, 3, 4, 1), (3, 3, 6, 2),
                                         (2, 1, 8, 2), (3, 1, 4, 2), (2, 3, 10, 1)])
def test_bond_sums_give_the_energy(oracle_mod, d, n, L, kind):
    N = L ** d
    if n == 1:
        s = inputs.random_ising(N, seed=L + d)
    else:
        s = inputs.random_unit_vectors(n, N, seed=L + d + n)
    lat = oracle_mod.OracleLattice(d, n, L, 5, J_kind=kind, J0=1.3, J_sigma=0.4, spins=s,
                                   delta=1.0)
    acc = np.zeros((d, N), dtype=np.int64 if n == 1 else np.float64)
    lat.bond_accumulate(acc)
    if kind == 0:
        Jb = np.full((d, N), 1.3)
    elif kind == 1:
        Jb = 1.3 * lat.J.astype(np.float64)
    else:
        Jb = lat.J.astype(np.float64)
    E = lat.measure().E
    assert abs((Jb * acc).sum() + E) <= 1e-12 * max(1.0, abs(E))
    # the products themselves: s_i . s_{i+mu} from the arrays directly
    x, y, z = _coords(d, L)
    for mu in range(d):
        nb = [(x + 1) % L + L * y + L * L * z, x + L * ((y + 1) % L) + L * L * z,
              x + L * y + L * L * ((z + 1) % L)][mu]
        sv = s.reshape(n, N) if n > 1 else s.reshape(1, N).astype(np.float64)
        prod = (sv * sv[:, nb]).sum(axis=0)
        assert np.abs(acc[mu] - prod).max() <= 1e-15


# ---------------------------------------------------------------------------
# tiled k-hit schedule
# ---------------------------------------------------------------------------
def _tile_colour(d, L, T):
    x, y, z = _coords(d, L)
    return (x // T + y // T + (z // T if d == 3 else 0)) & 1


@pytest.mark.parametrize("d,L,T,k", [(2, 8, 2, 1), (2, 8, 2, 2), (2, 8, 4, 3), (3, 8, 2, 3),
                                     (3, 4, 2, 2), (2, 16, 4, 5), (2, 32, 16, 4)])
def test_tiled_sweep_at_beta_zero_flips_every_site_k_times(oracle_mod, d, L, T, k):
    lat = oracle_mod.OracleLattice(d, 1, L, 8)
    s0 = lat.s.copy()
    lat.sweep_rule(0.0, 1, "metropolis", T, k)
    assert np.array_equal(lat.s, s0 * (-1) ** k)


@pytest.mark.parametrize("d,L,T,k,rule,kind", [(2, 8, 2, 2, "metropolis", 0),
                                               (2, 12, 2, 3, "heatbath", 1),
                                               (3, 8, 2, 2, "metropolis", 1),
                                               (2, 16, 4, 1, "heatbath", 0)])
def test_one_tile_colour_pass(oracle_mod, d, L, T, k, rule, kind):
    tcol = _tile_colour(d, L, T)
    lat = oracle_mod.OracleLattice(d, 1, L, 12, J_kind=kind)
    full = oracle_mod.OracleLattice(d, 1, L, 12, J_kind=kind)
    s0 = lat.s.copy()
    for t in range(3):
        before = lat.s.copy()
        lat.tile_pass(0.5, T, k, 0, rule, t=t)
        assert np.array_equal(lat.s[tcol == 1], before[tcol == 1])
        assert not np.array_equal(lat.s[tcol == 0], before[tcol == 0])
        mid = lat.s.copy()
        lat.tile_pass(0.5, T, k, 1, rule, t=t)
        assert np.array_equal(lat.s[tcol == 0], mid[tcol == 0])
    full.sweep_rule(0.5, 3, rule, T, k)
    assert np.array_equal(lat.s, full.s)
    # beta = 0, one Metropolis pass of tile colour 0 with k = 1 flips exactly those sites
    z = oracle_mod.OracleLattice(d, 1, L, 12, J_kind=kind, spins=s0, J=lat.J)
    z.tile_pass(0.0, T, 1, 0, "metropolis", t=0)
    assert np.array_equal(z.s, np.where(tcol == 0, -s0, s0))


def _draw(oracle_mod, seed, block, t, replica, tag):
    return oracle_mod.philox4x32_10([block, t, replica, tag], [seed & M32, seed >> 32])


def _new_spin(oracle_mod, lat, s, i, t, c, h, rule, beta):
    """One attempt at natural site i from the description: the local sum of
    the neighbours, the 32-bit uniform (prefix byte of the 16-site block, then
    the 24-bit refinement of the site's own block), the rule's threshold."""
    d, L, N = lat.d, lat.L, lat.N
    x = [i % L, (i // L) % L, i // (L * L)]
    tot = 0
    for mu in range(d):
        for step in (1, -1):
            q = list(x)
            q[mu] = (q[mu] + step) % L
            nb = q[0] + L * q[1] + (L * L * q[2] if d == 3 else 0)
            bond_site = i if step == 1 else nb  # bond (i, i+mu) is stored at i
            sign = 1 if lat.J is None else int(lat.J[mu, bond_site])
            tot += sign * int(s[nb])
    j = i >> 1
    seed, rep = int(lat.p.seed), int(lat.p.replica)
    wp = _draw(oracle_mod, seed, j >> 4, t, rep, c | (0 << 1) | (h << 8))
    wr = _draw(oracle_mod, seed, j, t, rep, c | (1 << 1) | (h << 8))
    prefix = (wp[(j >> 2) & 3] >> (8 * (j & 3))) & 0xFF
    u32 = (prefix << 24) | (wr[0] & 0xFFFFFF)
    J0 = float(lat.p.J0)
    if rule == "heatbath":
        return 1 if u32 < oracle_mod.threshold_hb(beta, J0 * tot) else -1
    m = int(s[i]) * tot
    return -int(s[i]) if u32 < oracle_mod.threshold(beta, 2.0 * J0 * m) else int(s[i])


def _written_out_sweep(oracle_mod, lat, s, t, beta, T, k, rule, rng, swapped=False):
    d, L = lat.d, lat.L
    x, y, z = _coords(d, L)
    colour = (x + y + z) & 1
    tcol = _tile_colour(d, L, T)
    stages = ([(tc, h) for tc in (0, 1) for h in range(k)] if not swapped
              else [(tc, h) for h in range(k) for tc in (0, 1)])
    for tc, h in stages:
        for c in (0, 1):
            for i in rng.permutation(np.nonzero((colour == c) & (tcol == tc))[0]):
                s[i] = _new_spin(oracle_mod, lat, s, int(i), t, c, h, rule, beta)
    return s


@pytest.mark.parametrize("d,rule,kind", [(2, "metropolis", 0), (2, "heatbath", 0),
                                         (2, "metropolis", 1), (3, "metropolis", 0),
                                         (3, "heatbath", 1)])
def test_tiled_schedule_written_out_step_by_step(oracle_mod, d, rule, kind):
    L, T, k, beta = 4, 2, 2, 0.44
    lat = oracle_mod.OracleLattice(d, 1, L, 3, J_kind=kind, J0=0.8 if kind else 1.0, replica=5)
    rng = np.random.default_rng(d)
    s = lat.s.astype(np.int64)
    swapped = s.copy()
    differs = False
    for t in range(3):
        s = _written_out_sweep(oracle_mod, lat, s, 10 + t, beta, T, k, rule, rng)
        swapped = _written_out_sweep(oracle_mod, lat, swapped, 10 + t, beta, T, k, rule, rng,
                                     swapped=True)
        lat.t = 10 + t
        lat.sweep_rule(beta, 1, rule, T, k)
        assert np.array_equal(lat.s, s), t
        differs |= not np.array_equal(s, swapped)
    assert differs, "the swapped loop order should give another chain"
    # and the plain schedule (tile 0, one hit) is the plain sweep of the chain
    plain = oracle_mod.OracleLattice(d, 1, L, 3, J_kind=kind, J0=0.8 if kind else 1.0, replica=5,
                                     J=lat.J)
    sp = plain.s.astype(np.int64)
    x, y, z = _coords(d, L)
    colour = (x + y + z) & 1
    for c in (0, 1):
        for i in rng.permutation(np.nonzero(colour == c)[0]):
            sp[i] = _new_spin(oracle_mod, plain, sp, int(i), 0, c, 0, rule, beta)
    plain.sweep_rule(beta, 1, rule)
    assert np.array_equal(plain.s, sp)
