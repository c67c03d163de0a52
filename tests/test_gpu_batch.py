"""GPU parity of batched sweeps: every lattice of a mixed batch (uneven L, its
own beta and disorder realisation) equals the oracle's single-lattice chain
with replica r, bit for bit, whatever the workgroup size, lattice order or
graph replay."""
import numpy as np
import pytest

import layout

pytestmark = pytest.mark.gpu


def _batch_params(d, n):
    Ls = [8, 12, 16, 24, 32] if d == 3 else [8, 12, 16, 32, 64, 6]
    L = [Ls[r % len(Ls)] for r in range(n)]
    beta = [0.5 + 2.5 * (r % 32) / 31 for r in range(n)]
    return L, beta


def _check(smc_gpu, oracle_mod, b, d, L, beta, kind, sweeps, seed, obs=None):
    for r in range(len(L)):
        ref = oracle_mod.OracleLattice(d, 1, L[r], seed, J_kind=kind, replica=r)
        if kind == 1:
            assert np.array_equal(layout.to_natural(b.couplings_of(r).cpu().numpy(), d, L[r]), ref.J)
        ref.sweep(beta[r], sweeps)
        got = layout.to_natural(b.spins_of(r).cpu().numpy(), d, L[r])
        assert np.array_equal(got, ref.s), (r, L[r], beta[r])
        if obs is not None:
            o = ref.measure()
            assert (obs[r].E_int, obs[r].M_int) == (o.E_int, o.M_int), r
            assert obs[r].sweep == sweeps


@pytest.mark.parametrize("d,kind,n", [(3, 1, 15), (2, 1, 12), (3, 0, 10), (2, 0, 7)])
def test_batch_matches_oracle(smc_gpu, oracle_mod, d, kind, n):
    import torch
    print(f"batch d={d} kind={kind} n={n}", flush=True)
    L, beta = _batch_params(d, n)
    b = smc_gpu.Batch(d, L, beta, seed=33, J_kind=kind)
    obs = torch.zeros((n, 8), dtype=torch.int64, device=b.device)
    b.sweep(7, obs)
    _check(smc_gpu, oracle_mod, b, d, L, beta, kind, 7, 33, smc_gpu.Lattice.decode_obs(obs))
    assert b.t == 7


def test_batch_schedules_and_graph_are_bit_identical(smc_gpu):
    import torch
    L, beta = _batch_params(3, 20)
    ref = smc_gpu.Batch(3, L, beta, seed=5)
    ref.sweep(6)
    tuned = smc_gpu.Batch(3, L, beta, seed=5)
    threads, largest = tuned.autotune()
    assert threads in (64, 128, 256, 512, 1024)
    tuned.sweep(2)
    tuned.use_graph(True)
    tuned.sweep(2)
    tuned.sweep(2)  # replay with an updated counter
    assert tuned.t == 6
    assert torch.equal(ref.spins, tuned.spins)


def test_batch_matches_single_lattice_path(smc_gpu):
    L, beta = _batch_params(3, 6)
    b = smc_gpu.Batch(3, L, beta, seed=9)
    b.sweep(5)
    for r in range(6):
        lat = smc_gpu.Lattice(3, 1, L[r], seed=9, J_kind=1, replica=r)
        lat.sweep(beta[r], 5)
        assert np.array_equal(lat.spins.cpu().numpy(), b.spins_of(r).cpu().numpy())


def test_batch_rejects_bad_shapes(smc_gpu):
    with pytest.raises(smc_gpu.SmcError):
        smc_gpu.Batch(3, [8, 42], [0.5, 0.5], seed=1)   # 42^3 > 65536 sites
    with pytest.raises(smc_gpu.SmcError):
        smc_gpu.Batch(3, [8, 9], [0.5, 0.5], seed=1)    # odd edge


@pytest.mark.parametrize("d,kind,n,graph", [(3, 1, 10, False), (2, 0, 12, True), (3, 0, 5, True)])
def test_batch_measurement_series_matches_oracle(smc_gpu, oracle_mod, d, kind, n, graph):
    """E and M recorded inside one launch every `every` sweeps equal the
    oracle's measurements of each lattice's chain at those sweeps."""
    import torch
    print(f"batch series d={d} kind={kind} n={n} graph={graph}", flush=True)
    L, beta = _batch_params(d, n)
    b = smc_gpu.Batch(d, L, beta, seed=41, J_kind=kind)
    b.use_graph(graph)
    every, sweeps = 3, 12
    series = torch.zeros((sweeps // every, n, 8), dtype=torch.int64, device=b.device)
    b.sweep(2)                                   # a counter offset before the series
    b.sweep(sweeps, series, every=every)
    assert b.t == 2 + sweeps
    recs = [smc_gpu.Lattice.decode_obs(series[m]) for m in range(sweeps // every)]
    for r in range(n):
        ref = oracle_mod.OracleLattice(d, 1, L[r], 41, J_kind=kind, replica=r)
        ref.sweep(beta[r], 2)
        for m in range(sweeps // every):
            ref.sweep(beta[r], every)
            o = ref.measure()
            got = recs[m][r]
            assert (got.E_int, got.M_int, got.sweep) == (o.E_int, o.M_int, 2 + every * (m + 1)), (r, m)
    _check(smc_gpu, oracle_mod, b, d, L, beta, kind, 2 + sweeps, 41)


def test_batch_series_rejects_bad_every(smc_gpu):
    import torch
    L, beta = _batch_params(3, 3)
    b = smc_gpu.Batch(3, L, beta, seed=1)
    obs = torch.zeros((4, 3, 8), dtype=torch.int64, device=b.device)
    with pytest.raises(smc_gpu.SmcError):
        b.sweep(10, obs, every=3)   # 3 does not divide 10
    with pytest.raises(smc_gpu.SmcError):
        b.sweep(10, obs, every=0)
    assert b.t == 0


@pytest.mark.parametrize("d,Ls,kind", [(3, [4, 20, 12, 28, 6], 1), (2, [4, 20, 28, 44, 10, 36], 0)])
def test_batch_pair_and_site_paths_match_oracle(smc_gpu, oracle_mod, d, Ls, kind):
    """Lattices whose plane rows are whole 2-site pairs (L/2 = 2, 6, 10, 14,
    ...), odd half-rows (one-site path) and whole words, side by side."""
    import torch
    n = len(Ls)
    beta = [0.3 + 0.4 * r for r in range(n)]
    b = smc_gpu.Batch(d, Ls, beta, seed=17, J_kind=kind)
    obs = torch.zeros((3, n, 8), dtype=torch.int64, device=b.device)
    b.sweep(9, obs, every=3)
    _check(smc_gpu, oracle_mod, b, d, Ls, beta, kind, 9, 17,
           smc_gpu.Lattice.decode_obs(obs[2]))


@pytest.mark.parametrize("kind,beta,sweeps", [(0, 0.4406868, 1), (0, 0.4406868, 3), (1, 0.8, 2)])
def test_batch_ensemble_matches_exact_propagation(smc_gpu, oracle_mod, kind, beta, sweeps):
    """2^17 copies of one 4 x 4 lattice (the same start state and couplings,
    replica = lattice index, so independent random streams) after a few sweeps
    are distributed as the exact propagation of Eq. (2) over all 2^16 states
    (chi^2 at p = 1e-4).  This pins the GPU chain to the dynamics without going
    through the oracle's chain (the oracle only supplies the start state)."""
    import torch
    from scipy.stats import chi2

    import oracle.exact as ex
    from test_oracle_ising import _chi2_states

    d, L, n = 2, 4, 1 << 17
    N = L ** d
    print(f"batch ensemble kind={kind} beta={beta} sweeps={sweeps}", flush=True)
    ref = oracle_mod.OracleLattice(d, 1, L, 11, J_kind=kind)
    b = smc_gpu.Batch(d, [L] * n, [beta] * n, seed=11, J_kind=kind, init="cold")
    assert b.spin_offsets == [N * r for r in range(n)]
    s0 = torch.from_numpy(layout.to_split(ref.s, d, L).reshape(-1).copy())
    b.spins.view(n, N).copy_(s0.to(b.device).expand(n, N))
    if kind == 1:
        assert b.coupling_offsets == [d * N * r for r in range(n)]
        J0 = torch.from_numpy(layout.to_split(ref.J, d, L).reshape(-1).copy())
        b.J.view(n, d * N).copy_(J0.to(b.device).expand(n, d * N))
    b.sweep(sweeps)
    got = layout.to_natural(b.spins.view(n, 2, N // 2).cpu().numpy(), d, L)
    chain = ex.SmallLatticeChain(d, L, beta, J=None if kind == 0 else ref.J)
    pi = np.zeros(1 << N)
    pi[ex.state_index(ref.s)] = 1.0
    for _ in range(sweeps):
        pi = chain.sweep(pi)
    stat, dof = _chi2_states(ex.state_index(got), pi)
    assert stat < chi2.ppf(1 - 1e-4, dof), (stat, dof)


@pytest.mark.parametrize("d,Ls,kind", [(2, [128, 96, 64, 32], 1), (3, [32, 24, 16], 0)])
def test_batch_index_paths_match_oracle(smc_gpu, oracle_mod, d, Ls, kind):
    """With 256 lanes per lattice: lattices of at most 256 groups of 16 sites
    (indices formed once per call), longer ones whose plane rows hold whole
    groups (L/2 % 16 == 0: formed once per group) and the rest (per word)."""
    import torch
    n = len(Ls)
    beta = [0.35 + 0.3 * r for r in range(n)]
    b = smc_gpu.Batch(d, Ls, beta, seed=23, J_kind=kind)
    obs = torch.zeros((n, 8), dtype=torch.int64, device=b.device)
    b.sweep(6, obs)
    _check(smc_gpu, oracle_mod, b, d, Ls, beta, kind, 6, 23, smc_gpu.Lattice.decode_obs(obs))


def test_batch_lds_limit_survives_a_smaller_batch(smc_gpu, oracle_mod):
    """A batch holding a 65536-site lattice needs more than 64 KiB of LDS per
    workgroup; a smaller batch created afterwards must not lower the limit."""
    big = smc_gpu.Batch(2, [256, 8], [0.45, 0.7], seed=31, J_kind=1)
    small = smc_gpu.Batch(2, [8, 12], [0.5, 0.6], seed=32, J_kind=1)
    small.sweep(2)
    big.sweep(2)
    _check(smc_gpu, oracle_mod, big, 2, [256, 8], [0.45, 0.7], 1, 2, 31)


def _c3_like(n):
    L = [[8, 12, 16, 24, 32][r % 5] for r in range(n)]
    beta = [0.5 + 2.5 * (r % 32) / 31 for r in range(n)]
    return L, beta


@pytest.mark.parametrize("threads", [64, 256, 1024])
def test_packed_and_byte_paths_run_the_same_chains(smc_gpu, monkeypatch, threads):
    """The spin-glass workload's mix (3D +-J, L in {8, 12, 16, 24, 32}, 32
    temperatures): lattices take the packed path where a lane holds at most
    two 32-site words of a colour (z-planes of whole words for L % 8 == 0,
    split words for L = 12), else the byte path; with the packed path
    switched off every lattice takes the byte path.  Final states and the E/M
    series inside the launch are equal."""
    import torch
    n = 45
    L, beta = _c3_like(n)
    out = {}
    for packed in (True, False):
        if packed:
            monkeypatch.delenv("SMC_BATCH_PACKED", raising=False)
        else:
            monkeypatch.setenv("SMC_BATCH_PACKED", "0")
        b = smc_gpu.Batch(3, L, beta, seed=61)
        b.threads = threads
        obs = torch.zeros((5, n, 8), dtype=torch.int64, device=b.device)
        b.sweep(25, obs, every=5)
        want = [(Lr % 4 == 0 and (Lr ** 3 // 64) <= 2 * threads) if packed else False for Lr in L]
        assert [b.packed(r) for r in range(n)] == want
        out[packed] = (b.spins.clone(), obs.clone())
    assert torch.equal(out[True][0], out[False][0])
    assert torch.equal(out[True][1], out[False][1])


@pytest.mark.parametrize("J0,betas", [(1.0, [0.0, float("inf"), 0.7, 2.9]),
                                      (-1.0, [0.3, 1.1, 2.2, float("inf")])])
def test_packed_batch_matches_oracle(smc_gpu, oracle_mod, J0, betas):
    """The packed path against the oracle, lattice by lattice, at the special
    temperatures and with J0 < 0 (classes with more than d unsatisfied bonds
    refusable: the general bit-sliced decision)."""
    import torch
    L = [8, 16, 24, 32, 4, 12, 20, 28]
    beta = [betas[r % len(betas)] for r in range(len(L))]
    b = smc_gpu.Batch(3, L, beta, seed=71, J0=J0)
    assert all(b.packed(r) for r in range(len(L)))
    obs = torch.zeros((len(L), 8), dtype=torch.int64, device=b.device)
    b.sweep(6, obs)
    recs = smc_gpu.Lattice.decode_obs(obs)
    for r in range(len(L)):
        ref = oracle_mod.OracleLattice(3, 1, L[r], 71, J_kind=1, J0=J0, replica=r)
        ref.sweep(beta[r], 6)
        got = layout.to_natural(b.spins_of(r).cpu().numpy(), 3, L[r])
        assert np.array_equal(got, ref.s), (r, L[r], beta[r])
        o = ref.measure()
        assert (recs[r].E_int, recs[r].M_int) == (o.E_int, o.M_int), r


@pytest.mark.parametrize("threads", [512, 1024])
def test_packed_batch_largest_lattices(smc_gpu, oracle_mod, threads):
    """The largest lattices the packed path takes, L = 36 (split z-plane
    words) and L = 40 (1000 words a colour: two per lane at 512 lanes, the
    last lane's second word past the plane), beside one L = 4, against the
    oracle at beta_c-like and low temperatures."""
    import torch
    L = [40, 36, 4]
    beta = [0.25, 0.9, 0.4]
    b = smc_gpu.Batch(3, L, beta, seed=83)
    b.threads = threads
    assert all(b.packed(r) for r in range(len(L)))
    obs = torch.zeros((len(L), 8), dtype=torch.int64, device=b.device)
    b.sweep(4, obs)
    recs = smc_gpu.Lattice.decode_obs(obs)
    for r in range(len(L)):
        ref = oracle_mod.OracleLattice(3, 1, L[r], 83, J_kind=1, replica=r)
        ref.sweep(beta[r], 4)
        got = layout.to_natural(b.spins_of(r).cpu().numpy(), 3, L[r])
        assert np.array_equal(got, ref.s), (r, L[r], beta[r])
        o = ref.measure()
        assert (recs[r].E_int, recs[r].M_int) == (o.E_int, o.M_int), r
