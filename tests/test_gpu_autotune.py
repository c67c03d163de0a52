"""The schedule autotuner: band heights of the single-lattice kernels and the
batch's workgroup size, lattice order and path.

* Every band height the tuner can pick gives the same chain: the Ising
  kernels against the oracle bit for bit, the continuous streaming kernel
  bit-identical across heights (the arithmetic per site does not depend on
  the band).
* Tuning leaves the state and the sweep counter as they were, picks one of
  the candidate heights, and the tuned lattice continues the same chain.
* The cache named by SMC_AUTOTUNE_CACHE stores the choice and a stored
  choice is taken without timing."""
import numpy as np
import pytest

import layout

pytestmark = pytest.mark.gpu

# (name, lattice keyword arguments, environment override, candidate heights)
KERNELS = [
    ("ising_stream", dict(d=2, n=1, L=256), "SMC_STREAM_ROWS", [4, 8, 16, 32, 64]),
    ("ising_stream", dict(d=3, n=1, L=64), "SMC_STREAM_ROWS", [4, 8, 16, 32, 64]),
    ("ising_packed", dict(d=2, n=1, L=256, packed=True), "SMC_PACKED_ROWS", [1, 2, 4, 8, 16, 32, 64]),
    ("ising_packed", dict(d=3, n=1, L=64, packed=True), "SMC_PACKED_ROWS", [1, 2, 4, 8, 16, 32, 64]),
    ("xy_stream", dict(d=2, n=2, L=256, delta=1.63), "SMC_CONT_ROWS", [4, 8, 16, 32, 64]),
    ("heisenberg_stream", dict(d=3, n=3, L=64, delta=2.058), "SMC_CONT_ROWS", [4, 8, 16, 32, 64]),
    ("ising_fused", dict(d=2, n=1, L=2048, fused=True), "SMC_FUSED_ROWS", [4, 8, 16, 32, 64]),
]
BETA = {1: 0.44, 2: 1.12, 3: 0.693}


def _make(smc_gpu, kw, seed=12):
    kw = dict(kw)
    d, n, L = kw.pop("d"), kw.pop("n"), kw.pop("L")
    return smc_gpu.Lattice(d, n, L, seed=seed, **kw)


def _state(lat):
    if lat.packed:
        import paper_1107_5463_amd as smc
        return smc.unpack_spins(lat.spins.view(-1)).cpu().numpy()
    return lat.spins.cpu().numpy()


@pytest.mark.parametrize("name,kw,env,heights", KERNELS)
def test_every_band_height_gives_the_same_chain(smc_gpu, oracle_mod, monkeypatch, name, kw, env,
                                                heights):
    print(f"band heights {name} {kw}", flush=True)
    d, n, L = kw["d"], kw["n"], kw["L"]
    sweeps = 3
    states = []
    for H in heights:
        monkeypatch.setenv(env, str(H))
        lat = _make(smc_gpu, kw)
        assert lat.kernel() == (name, H), (lat.kernel(), H)
        lat.sweep(BETA[n], sweeps)
        states.append(_state(lat))
    for H, s in zip(heights[1:], states[1:]):
        assert np.array_equal(s, states[0]), (name, H)
    if n == 1:
        ref = oracle_mod.OracleLattice(d, 1, L, 12)
        ref.sweep(BETA[1], sweeps)
        assert np.array_equal(layout.to_natural(states[0].reshape(2, -1), d, L), ref.s)


@pytest.mark.parametrize("name,kw,env,heights", KERNELS)
def test_autotune_keeps_the_chain(smc_gpu, monkeypatch, tmp_path, name, kw, env, heights):
    import torch
    monkeypatch.delenv(env, raising=False)
    monkeypatch.setenv("SMC_AUTOTUNE_CACHE", str(tmp_path / "tune.txt"))
    n = kw["n"]
    lat = _make(smc_gpu, kw)
    lat.sweep(BETA[n], 2)
    before, t0 = lat.spins.clone(), lat.t
    H = lat.autotune(BETA[n])
    print(f"autotune {name} {kw}: rows {H}", flush=True)
    assert H in heights and lat.kernel() == (name, H)
    assert torch.equal(lat.spins, before) and lat.t == t0
    lat.sweep(BETA[n], 2)
    ref = _make(smc_gpu, kw)
    ref.sweep(BETA[n], 4)
    assert torch.equal(lat.spins, ref.spins)
    prefix = {"ising_stream": "ising_stream:", "ising_packed": "packed:", "xy_stream": "xy_stream:",
              "heisenberg_stream": "heisenberg_stream:", "ising_fused": "fused:"}[name]
    lines = (tmp_path / "tune.txt").read_text().strip().split("\n")
    assert len(lines) == 1 and lines[0].startswith(prefix) and lines[0].endswith(f" {H}"), lines


def test_autotune_takes_a_cached_choice(smc_gpu, monkeypatch, tmp_path):
    cache = tmp_path / "tune.txt"
    monkeypatch.setenv("SMC_AUTOTUNE_CACHE", str(cache))
    kw = dict(d=2, n=1, L=256, packed=True)
    lat = _make(smc_gpu, kw)
    lat.autotune(0.44)
    (key, val), = [line.split(" ") for line in cache.read_text().strip().split("\n")]
    other = 2 if int(val) != 2 else 4
    cache.write_text(f"{key} {other}\n")
    lat2 = _make(smc_gpu, kw)
    assert lat2.autotune(0.44) == other
    assert lat2.kernel() == ("ising_packed", other)


def test_batch_autotune_cache(smc_gpu, monkeypatch, tmp_path):
    import torch
    cache = tmp_path / "tune.txt"
    monkeypatch.setenv("SMC_AUTOTUNE_CACHE", str(cache))
    L = [[8, 12, 16, 24, 32][r % 5] for r in range(20)]
    beta = [0.5 + 0.1 * r for r in range(20)]
    ref = smc_gpu.Batch(3, L, beta, seed=3)
    ref.sweep(4)
    b = smc_gpu.Batch(3, L, beta, seed=3)
    th, lf = b.autotune()
    text = cache.read_text()
    assert text.startswith("batch:d3:J1:n20:") and f" {th},{int(lf)}," in text, text
    # a stored choice is taken as it stands
    key = text.split(" ")[0]
    cache.write_text(f"{key} 128,0,0\n")
    b2 = smc_gpu.Batch(3, L, beta, seed=3)
    assert b2.autotune() == (128, False)
    assert not any(b2.packed(r) for r in range(20))
    b2.sweep(4)
    b.sweep(4)
    assert torch.equal(b.spins, ref.spins) and torch.equal(b2.spins, ref.spins)
