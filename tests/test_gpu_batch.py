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
    assert threads in (64, 128, 256, 512)
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
