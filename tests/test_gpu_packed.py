"""GPU parity of the bit-packed Ising kernels (one bit per site): the same
chain as the int8 kernels and the oracle, bit for bit."""
import numpy as np
import pytest

import layout

pytestmark = pytest.mark.gpu

BETA_C = 0.4406868


def unpack_nat(smc_gpu, words, d, L):
    flat = smc_gpu.unpack_spins(words.contiguous().view(-1)).cpu().numpy()
    return layout.to_natural(flat.reshape(-1, 2, L ** d // 2), d, L)


def nat(smc_gpu, lat):
    return unpack_nat(smc_gpu, lat.spins, lat.d, lat.L)[0]


def test_pack_unpack_round_trip(smc_gpu):
    import torch
    g = torch.Generator().manual_seed(3)
    a = (torch.randint(0, 2, (4096,), generator=g) * 2 - 1).to(torch.int8).cuda()
    w = smc_gpu.pack_spins(a)
    assert w.numel() == 128
    b = smc_gpu.unpack_spins(w)
    assert torch.equal(a, b)
    # bit k & 31 of word k >> 5 is site k, set for -1
    ref = np.zeros(128, dtype=np.int64)
    an = a.cpu().numpy()
    for k in range(4096):
        if an[k] < 0:
            ref[k >> 5] |= 1 << (k & 31)
    assert np.array_equal(w.cpu().numpy().astype(np.int64) & 0xFFFFFFFF, ref)


@pytest.mark.parametrize("d,L,kind", [(2, 64, 0), (2, 128, 1), (3, 64, 0), (3, 64, 1)])
def test_init_matches_oracle(smc_gpu, oracle_mod, d, L, kind):
    lat = smc_gpu.Lattice(d, 1, L, seed=21, J_kind=kind, packed=True)
    ref = oracle_mod.OracleLattice(d, 1, L, 21, J_kind=kind)
    assert np.array_equal(nat(smc_gpu, lat), ref.s)
    if kind == 1:
        J = unpack_nat(smc_gpu, lat.J, d, L)
        assert np.array_equal(J, ref.J)


SHAPES = [  # d, L, J_kind, beta, sweeps
    (2, 64, 0, BETA_C, 30),
    (2, 128, 1, 0.8, 20),
    (2, 192, 0, 0.3, 10),    # 3 words per plane row
    (3, 64, 0, 0.2216546, 6),
    (3, 64, 1, 0.9, 5),
    (2, 64, 0, 2.0, 30),     # low temperature: mostly refusable moves
]


@pytest.mark.parametrize("ties", ["wave", "lane", "fallback"])
@pytest.mark.parametrize("d,L,kind,beta,n", SHAPES)
def test_sweeps_match_oracle(smc_gpu, oracle_mod, d, L, kind, beta, n, ties, monkeypatch):
    monkeypatch.setenv("SMC_PACKED_TIES", ties)
    print(f"packed sweeps d={d} L={L} kind={kind} beta={beta} ties={ties}", flush=True)
    lat = smc_gpu.Lattice(d, 1, L, seed=L + kind, J_kind=kind, packed=True)
    assert lat.kernel()[0] == "ising_packed"
    ref = oracle_mod.OracleLattice(d, 1, L, L + kind, J_kind=kind)
    lat.sweep(beta, n)
    ref.sweep(beta, n)
    assert np.array_equal(nat(smc_gpu, lat), ref.s)
    o, r = lat.measure(), ref.measure()
    assert (o.E_int, o.M_int) == (r.E_int, r.M_int)


@pytest.mark.parametrize("ties", ["wave", "lane", "fallback"])
@pytest.mark.parametrize("rows", ["1", "4", "16", "64"])
def test_band_heights_give_the_same_chain(smc_gpu, oracle_mod, rows, ties, monkeypatch):
    monkeypatch.setenv("SMC_PACKED_ROWS", rows)
    monkeypatch.setenv("SMC_PACKED_TIES", ties)
    lat = smc_gpu.Lattice(2, 1, 128, seed=4, packed=True)
    assert lat.kernel() == ("ising_packed", int(rows))
    ref = oracle_mod.OracleLattice(2, 1, 128, 4)
    lat.sweep(BETA_C, 8)
    ref.sweep(BETA_C, 8)
    assert np.array_equal(nat(smc_gpu, lat), ref.s)


@pytest.mark.parametrize("ties", ["wave", "lane", "fallback"])
@pytest.mark.parametrize("d,L", [(2, 128), (3, 64)])
def test_sweep_measure_matches_oracle(smc_gpu, oracle_mod, d, L, ties, monkeypatch):
    import torch
    monkeypatch.setenv("SMC_PACKED_TIES", ties)
    lat = smc_gpu.Lattice(d, 1, L, seed=33, packed=True)
    ref = oracle_mod.OracleLattice(d, 1, L, 33)
    slots = torch.zeros((3, 8), dtype=torch.int64, device=lat.device)
    for k, n in enumerate((1, 4, 0)):
        lat.sweep_measure(0.5, n, slots[k])
    got = smc_gpu.Lattice.decode_obs(slots)
    for k, n in enumerate((1, 4, 0)):
        ref.sweep(0.5, n)
        r = ref.measure()
        assert (got[k].E_int, got[k].M_int) == (r.E_int, r.M_int), k
    assert [o.sweep for o in got] == [1, 5, 5]


@pytest.mark.parametrize("ties", ["wave", "lane", "fallback"])
def test_many_ties_per_wave(smc_gpu, oracle_mod, ties, monkeypatch):
    """Bands of 64 rows at beta = 2 on a 2D L=4096 lattice (a wave is one
    plane row's 64 word columns): a lane meets a tied word every 8 to 25 words
    (a refusable site ties with probability 2^-8, and 30-90 % of the sites are
    refusable), so a wave ends its band with about 100-190 queued words --
    more than one round of the wave's resolution -- and some lanes resolve a
    full queue on the spot."""
    monkeypatch.setenv("SMC_PACKED_ROWS", "64")
    monkeypatch.setenv("SMC_PACKED_TIES", ties)
    L = 4096
    print(f"packed many ties L={L} ties={ties}", flush=True)
    import torch
    lat = smc_gpu.Lattice(2, 1, L, seed=7, packed=True)
    assert lat.kernel() == ("ising_packed", 64)
    ref = oracle_mod.OracleLattice(2, 1, L, 7)
    lat.sweep(2.0, 2)
    ref.sweep(2.0, 2)
    assert np.array_equal(nat(smc_gpu, lat), ref.s)
    # a measured sweep: the tie flips' share of E and M
    slot = torch.zeros((1, 8), dtype=torch.int64, device=lat.device)
    lat.sweep_measure(2.0, 1, slot[0])
    ref.sweep(2.0, 1)
    got, r = smc_gpu.Lattice.decode_obs(slot)[0], ref.measure()
    assert (got.E_int, got.M_int) == (r.E_int, r.M_int)
    assert np.array_equal(nat(smc_gpu, lat), ref.s)


@pytest.mark.parametrize("kind", [0, 1])
def test_wave_uniform_bands_match_oracle(smc_gpu, oracle_mod, kind):
    """2D L=4096: a plane row is 64 words, so every wave lies inside one band
    and the kernel keeps the band's row arithmetic in scalar registers; plain
    and measured sweeps with uniform and +-1 couplings, bit for bit."""
    import torch
    L = 4096
    print(f"packed wave-uniform bands L={L} kind={kind}", flush=True)
    lat = smc_gpu.Lattice(2, 1, L, seed=21 + kind, J_kind=kind, packed=True)
    assert lat.kernel()[0] == "ising_packed"
    ref = oracle_mod.OracleLattice(2, 1, L, 21 + kind, J_kind=kind)
    lat.sweep(BETA_C, 2)
    ref.sweep(BETA_C, 2)
    slot = torch.zeros((1, 8), dtype=torch.int64, device=lat.device)
    lat.sweep_measure(BETA_C, 1, slot[0])
    ref.sweep(BETA_C, 1)
    got, r = smc_gpu.Lattice.decode_obs(slot)[0], ref.measure()
    assert (got.E_int, got.M_int) == (r.E_int, r.M_int)
    assert np.array_equal(nat(smc_gpu, lat), ref.s)


@pytest.mark.parametrize("rows", ["2", "4"])
@pytest.mark.parametrize("kind", [0, 1])
def test_wave_parity_bands_3d_match_oracle(smc_gpu, oracle_mod, rows, kind, monkeypatch):
    """3D L=128: a plane row is 2 words, so a wave holds 32 bands; with an even
    band height they lie in one z-plane and share their rows' parity, which
    the kernel then takes as a compile-time constant.  Plain and measured
    sweeps, uniform and +-1 couplings, bit for bit."""
    import torch
    monkeypatch.setenv("SMC_PACKED_ROWS", rows)
    L = 128
    print(f"packed wave-parity bands 3D L={L} rows={rows} kind={kind}", flush=True)
    lat = smc_gpu.Lattice(3, 1, L, seed=41 + kind, J_kind=kind, packed=True)
    assert lat.kernel() == ("ising_packed", int(rows))
    ref = oracle_mod.OracleLattice(3, 1, L, 41 + kind, J_kind=kind)
    lat.sweep(0.2216546, 2)
    ref.sweep(0.2216546, 2)
    slot = torch.zeros((1, 8), dtype=torch.int64, device=lat.device)
    lat.sweep_measure(0.2216546, 1, slot[0])
    ref.sweep(0.2216546, 1)
    got, r = smc_gpu.Lattice.decode_obs(slot)[0], ref.measure()
    assert (got.E_int, got.M_int) == (r.E_int, r.M_int)
    assert np.array_equal(nat(smc_gpu, lat), ref.s)


def test_special_temperatures(smc_gpu, oracle_mod):
    for beta in (0.0, float("inf")):
        lat = smc_gpu.Lattice(2, 1, 64, seed=9, packed=True)
        ref = oracle_mod.OracleLattice(2, 1, 64, 9)
        lat.sweep(beta, 3)
        ref.sweep(beta, 3)
        assert np.array_equal(nat(smc_gpu, lat), ref.s), beta


def test_full_size_2d_matches_oracle(smc_gpu, oracle_mod):
    L = 16384
    print("packed full size 2D L=16384, 2 sweeps", flush=True)
    lat = smc_gpu.Lattice(2, 1, L, seed=2, packed=True)
    ref = oracle_mod.OracleLattice(2, 1, L, 2)
    lat.sweep(BETA_C, 2)
    ref.sweep(BETA_C, 2)
    o, r = lat.measure(), ref.measure()
    assert (o.E_int, o.M_int) == (r.E_int, r.M_int)
    assert np.array_equal(nat(smc_gpu, lat), ref.s)


def test_full_size_3d_matches_oracle(smc_gpu, oracle_mod):
    L = 512
    print("packed full size 3D L=512, 2 sweeps", flush=True)
    lat = smc_gpu.Lattice(3, 1, L, seed=3, packed=True)
    ref = oracle_mod.OracleLattice(3, 1, L, 3)
    lat.sweep(0.2216546, 2)
    ref.sweep(0.2216546, 2)
    o, r = lat.measure(), ref.measure()
    assert (o.E_int, o.M_int) == (r.E_int, r.M_int)
    assert np.array_equal(nat(smc_gpu, lat), ref.s)


def test_packed_and_int8_chains_agree(smc_gpu):
    import torch
    a = smc_gpu.Lattice(3, 1, 128, seed=12, J_kind=1, packed=True)
    b = smc_gpu.Lattice(3, 1, 128, seed=12, J_kind=1)
    a.sweep(0.7, 4)
    b.sweep(0.7, 4)
    assert torch.equal(smc_gpu.unpack_spins(a.spins.view(-1)), b.spins.view(-1))


def test_bond_correlations_refused(smc_gpu):
    lat = smc_gpu.Lattice(2, 1, 64, seed=1, packed=True)
    with pytest.raises(smc_gpu.SmcError):
        lat.bond_reset()


@pytest.mark.parametrize("d,L,kind,J0,beta,n", [(2, 64, 0, -1.0, BETA_C, 10), (3, 64, 0, -1.0, 0.25, 5),
                                                (2, 64, 1, -0.7, 0.6, 10), (2, 64, 0, 0.5, 0.9, 10),
                                                (3, 64, 1, 2.0, 0.15, 4)])
@pytest.mark.parametrize("packed", [True, False])
def test_coupling_scale_and_sign_match_oracle(smc_gpu, oracle_mod, d, L, kind, J0, beta, n, packed):
    """Uniform or +-1 couplings scaled by J0, including J0 < 0 (the refusable
    moves are then those with more than d unsatisfied bonds), bit for bit in
    both spin layouts."""
    print(f"J0 sweeps d={d} L={L} kind={kind} J0={J0} packed={packed}", flush=True)
    lat = smc_gpu.Lattice(d, 1, L, seed=9 + kind, J_kind=kind, J0=J0, packed=packed)
    ref = oracle_mod.OracleLattice(d, 1, L, 9 + kind, J_kind=kind, J0=J0)
    lat.sweep(beta, n)
    ref.sweep(beta, n)
    got = nat(smc_gpu, lat) if packed else layout.to_natural(lat.spins.cpu().numpy(), d, L)
    assert np.array_equal(got, ref.s)
    o, r = lat.measure(), ref.measure()
    assert o.M_int == r.M_int and o.E == r.E, (o.E, r.E)
