"""GPU parity of the heat-bath rule and of the tiled k-hit schedule (Sec. 2)
against the oracle, bit for bit."""
import numpy as np
import pytest

import layout

pytestmark = pytest.mark.gpu

BETA_C = 0.4406868


def nat(lat):
    return layout.to_natural(lat.spins.cpu().numpy(), lat.d, lat.L)


@pytest.mark.parametrize("d,L,kind,beta,n", [(2, 32, 0, BETA_C, 20), (2, 20, 1, 0.9, 15),
                                             (3, 8, 1, 0.3, 10), (3, 16, 0, 0.2216546, 6),
                                             (2, 64, 0, float("inf"), 3)])
def test_heatbath_plain_sweeps_match_oracle(smc_gpu, oracle_mod, d, L, kind, beta, n):
    print(f"heat bath d={d} L={L} kind={kind}", flush=True)
    lat = smc_gpu.Lattice(d, 1, L, seed=L + 3, J_kind=kind, heatbath=True)
    ref = oracle_mod.OracleLattice(d, 1, L, L + 3, J_kind=kind)
    lat.sweep(beta, n)
    ref.sweep_rule(beta, n, "heatbath")
    assert np.array_equal(nat(lat), ref.s)


TILED = [  # d, L, tile, hits, heatbath, beta, sweeps
    (2, 64, 32, 3, False, BETA_C, 4),
    (2, 128, 32, 5, False, 0.6, 3),
    (2, 256, 64, 2, False, BETA_C, 2),
    (2, 64, 32, 4, True, BETA_C, 4),
    (3, 64, 32, 2, False, 0.2216546, 2),
    (3, 64, 32, 1, True, 0.25, 2),
    (2, 64, 16, 3, False, BETA_C, 4),      # the paper's 16 x 16 tiles
    (2, 160, 16, 2, False, 0.6, 3),        # 50 tiles per colour: a partly filled workgroup
    (2, 64, 16, 2, True, BETA_C, 3),
    (3, 32, 16, 2, False, 0.2216546, 2),
    (3, 32, 16, 1, True, 0.25, 2),
]


def _tile_kernel_name(d, T, hb):
    # 2D tiles of 16, 64 or 128 and 3D tiles of 16 (either rule) take the
    # bit-packed tile kernels
    packed = T in (16, 64, 128) if d == 2 else T == 16
    return "ising_tiles_packed" if packed else "ising_tiles"


@pytest.mark.parametrize("d,L,T,k,hb,beta,n", TILED)
def test_tiled_schedule_matches_oracle(smc_gpu, oracle_mod, d, L, T, k, hb, beta, n):
    print(f"tiles d={d} L={L} T={T} k={k} hb={hb}", flush=True)
    lat = smc_gpu.Lattice(d, 1, L, seed=7, heatbath=hb, tile=T, hits=k)
    assert lat.kernel() == (_tile_kernel_name(d, T, hb), T)
    ref = oracle_mod.OracleLattice(d, 1, L, 7)
    lat.sweep(beta, n)
    ref.sweep_rule(beta, n, "heatbath" if hb else "metropolis", T, k)
    assert np.array_equal(nat(lat), ref.s)
    o, r = lat.measure(), ref.measure()
    assert (o.E_int, o.M_int) == (r.E_int, r.M_int)
    assert lat.t == n


PACKED_TILES = [  # L, tile, hits, J0, beta, sweeps
    (128, 64, 3, 1.0, BETA_C, 3),     # two tiles a colour: one workgroup, two of its four tiles idle
    (384, 64, 2, 1.0, 0.6, 2),        # 18 tiles a colour: the last workgroup half filled
    (128, 64, 4, 1.0, 2.0, 3),        # low temperature: mostly refusable moves, many exact ties
    (256, 128, 2, 1.0, BETA_C, 2),    # one 128-tile a workgroup, two words a tile row
    (128, 64, 3, -1.0, 0.5, 3),       # J0 < 0: the general bit-sliced decision
    (64, 16, 3, 1.0, BETA_C, 3),      # the paper's 16 x 16 tiles: 8 tiles a colour, one workgroup
    (1056, 16, 2, 1.0, 0.6, 2),       # 2178 tiles a colour: 35 workgroups, the last partly filled
    (96, 16, 4, 1.0, 2.0, 3),         # low temperature: many exact ties
    (64, 16, 3, -1.0, 0.5, 3),        # J0 < 0
]


@pytest.mark.parametrize("ties", ["group", "lane"])
@pytest.mark.parametrize("L,T,k,J0,beta,n", PACKED_TILES)
def test_packed_tiles_match_oracle(smc_gpu, oracle_mod, monkeypatch, L, T, k, J0, beta, n, ties):
    """The bit-packed tile kernels (2D, Metropolis, T = 16, 64 or 128) against
    the oracle's tiled schedule, bit for bit, with the measurement after it;
    exact ties resolved by the workgroup, or (its fallback) each lane drawing
    its own."""
    monkeypatch.setenv("SMC_PACKED_TIES", ties)
    print(f"packed tiles L={L} T={T} k={k} J0={J0} beta={beta} ties={ties}", flush=True)
    lat = smc_gpu.Lattice(2, 1, L, seed=13, J0=J0, tile=T, hits=k)
    assert lat.kernel() == ("ising_tiles_packed", T)
    ref = oracle_mod.OracleLattice(2, 1, L, 13, J0=J0)
    lat.sweep(beta, n)
    ref.sweep_rule(beta, n, "metropolis", T, k)
    assert np.array_equal(nat(lat), ref.s)
    o, r = lat.measure(), ref.measure()
    assert (o.E_int, o.M_int) == (r.E_int, r.M_int)


@pytest.mark.parametrize("hb", [False, True])
@pytest.mark.parametrize("T", [16, 64, 128])
def test_packed_and_byte_tiles_run_the_same_chain(smc_gpu, monkeypatch, T, hb):
    """Both tile kernels on a 2D L=1024 lattice, k = 5 hits, either rule: the
    same states."""
    import torch
    states = {}
    for kernel in ("byte", "packed"):
        if kernel == "byte":
            monkeypatch.setenv("SMC_TILE_KERNEL", "byte")
        else:
            monkeypatch.delenv("SMC_TILE_KERNEL", raising=False)
        lat = smc_gpu.Lattice(2, 1, 1024, seed=17, tile=T, hits=5, heatbath=hb)
        assert lat.kernel()[0] == ("ising_tiles" if kernel == "byte" else "ising_tiles_packed")
        lat.sweep(BETA_C, 3)
        states[kernel] = lat.spins.clone()
    assert torch.equal(states["byte"], states["packed"])


PACKED_HB_TILES = [  # L, tile, hits, J0, beta, sweeps
    (128, 64, 3, 1.0, BETA_C, 3),
    (256, 128, 2, 1.0, 0.6, 2),
    (128, 64, 2, -1.0, 0.5, 2),        # J0 < 0
    (96, 16, 3, 1.0, BETA_C, 3),       # the paper's 16 x 16 tiles
    (64, 16, 2, 1.0, 2.0, 3),          # low temperature
    (128, 64, 2, 1.0, float("inf"), 2),  # thresholds 0, 2^31 and 2^32
]


@pytest.mark.parametrize("L,T,k,J0,beta,n", PACKED_HB_TILES)
def test_packed_heatbath_tiles_match_oracle(smc_gpu, oracle_mod, L, T, k, J0, beta, n):
    """The bit-packed tile kernels under the heat-bath rule (the class of a
    site is its number of up neighbours) against the oracle's tiled schedule,
    bit for bit, with the measurement after it."""
    print(f"packed heat-bath tiles L={L} T={T} k={k} J0={J0} beta={beta}", flush=True)
    lat = smc_gpu.Lattice(2, 1, L, seed=19, J0=J0, tile=T, hits=k, heatbath=True)
    assert lat.kernel() == ("ising_tiles_packed", T)
    ref = oracle_mod.OracleLattice(2, 1, L, 19, J0=J0)
    lat.sweep(beta, n)
    ref.sweep_rule(beta, n, "heatbath", T, k)
    assert np.array_equal(nat(lat), ref.s)
    o, r = lat.measure(), ref.measure()
    assert (o.E_int, o.M_int) == (r.E_int, r.M_int)


PACKED_3D_TILES = [  # L, hits, J0, heatbath, beta, sweeps
    (32, 3, 1.0, False, 0.2216546, 2),    # 4 tiles a colour: one workgroup
    (64, 2, 1.0, False, 0.3, 2),          # 32 tiles a colour: 8 workgroups
    (96, 2, 1.0, False, 0.2216546, 1),    # 108 tiles a colour: the last workgroup fully used
    (32, 3, 1.0, False, 1.0, 2),          # low temperature: many exact ties
    (32, 2, -1.0, False, 0.3, 2),         # J0 < 0: the general decision
    (32, 2, 1.0, True, 0.25, 2),          # heat bath
    (64, 2, 1.0, True, 1.0, 2),           # heat bath, low temperature
]


@pytest.mark.parametrize("ties", ["group", "lane"])
@pytest.mark.parametrize("L,k,J0,hb,beta,n", PACKED_3D_TILES)
def test_packed_3d_tiles_match_oracle(smc_gpu, oracle_mod, monkeypatch, L, k, J0, hb, beta, n, ties):
    """The bit-packed 16^3 tile kernel (either rule) against the oracle's tiled
    schedule, bit for bit, with the measurement after it."""
    monkeypatch.setenv("SMC_PACKED_TIES", ties)
    print(f"packed 3D tiles L={L} k={k} J0={J0} hb={hb} beta={beta} ties={ties}", flush=True)
    lat = smc_gpu.Lattice(3, 1, L, seed=23, J0=J0, tile=16, hits=k, heatbath=hb)
    assert lat.kernel() == ("ising_tiles_packed", 16)
    ref = oracle_mod.OracleLattice(3, 1, L, 23, J0=J0)
    lat.sweep(beta, n)
    ref.sweep_rule(beta, n, "heatbath" if hb else "metropolis", 16, k)
    assert np.array_equal(nat(lat), ref.s)
    o, r = lat.measure(), ref.measure()
    assert (o.E_int, o.M_int) == (r.E_int, r.M_int)


@pytest.mark.parametrize("hb", [False, True])
def test_packed_and_byte_3d_tiles_run_the_same_chain(smc_gpu, monkeypatch, hb):
    """Both 16^3 tile kernels on a 3D L=128 lattice, k = 3 hits: the same states."""
    import torch
    states = {}
    for kernel in ("byte", "packed"):
        if kernel == "byte":
            monkeypatch.setenv("SMC_TILE_KERNEL", "byte")
        else:
            monkeypatch.delenv("SMC_TILE_KERNEL", raising=False)
        lat = smc_gpu.Lattice(3, 1, 128, seed=29, tile=16, hits=3, heatbath=hb)
        assert lat.kernel()[0] == ("ising_tiles" if kernel == "byte" else "ising_tiles_packed")
        lat.sweep(0.2216546, 2)
        states[kernel] = lat.spins.clone()
    assert torch.equal(states["byte"], states["packed"])


def test_tiled_sweep_measure(smc_gpu, oracle_mod):
    import torch
    lat = smc_gpu.Lattice(2, 1, 64, seed=11, tile=32, hits=3)
    ref = oracle_mod.OracleLattice(2, 1, 64, 11)
    slot = torch.zeros(8, dtype=torch.int64, device=lat.device)
    lat.sweep_measure(0.5, 3, slot)
    ref.sweep_rule(0.5, 3, "metropolis", 32, 3)
    o = smc_gpu.Lattice.decode_obs(slot)[0]
    r = ref.measure()
    assert (o.E_int, o.M_int, o.sweep) == (r.E_int, r.M_int, 3)


def test_tiled_half_sweep_is_refused(smc_gpu):
    lat = smc_gpu.Lattice(2, 1, 64, seed=1, tile=32, hits=2)
    with pytest.raises(smc_gpu.SmcError):
        lat.half_sweep(0.4, 0)


def test_tile_lds_limit_survives_a_smaller_handle(smc_gpu, oracle_mod):
    """A lattice with 256 x 256 tiles needs more than 64 KiB of LDS per
    workgroup; creating a lattice with small tiles afterwards must not lower
    the kernels' LDS limit under it."""
    print("tiles: T=256 lattice after a T=16 one", flush=True)
    big = smc_gpu.Lattice(2, 1, 512, seed=5, tile=256, hits=2)
    small = smc_gpu.Lattice(2, 1, 64, seed=6, tile=16, hits=2)
    small.sweep(0.5, 1)
    big.sweep(0.5, 1)
    ref = oracle_mod.OracleLattice(2, 1, 512, 5)
    ref.sweep_rule(0.5, 1, "metropolis", 256, 2)
    assert np.array_equal(nat(big), ref.s)
