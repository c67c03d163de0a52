"""smc_measure_noalloc -- the measurement for callers that cannot allocate
device memory -- against smc_measure_async on the same states.

Both run the same measurement kernels; the allocation-free entry point takes
its reduction partials from the library's static per-GPU scratch instead of a
handle's workspace, so the 64-byte observable records must be equal bit for
bit.  Each sequence measures a lattice and then a smaller one (the scratch
keeps the first call's partials; the second must not read them), and then
the first again.  The packed 2D L = 16384 case fills the scratch's whole
capacity (16384 partials)."""
import pytest

pytestmark = pytest.mark.gpu

SEQUENCES = [
    [dict(d=3, n=1, L=64, J_kind=1, seed=3), dict(d=2, n=1, L=32, seed=4)],
    [dict(d=2, n=1, L=16384, packed=True, seed=2), dict(d=2, n=1, L=128, packed=True, J_kind=1, seed=6)],
    [dict(d=3, n=3, L=32, seed=7, delta=1.0), dict(d=2, n=2, L=16, seed=8, delta=1.0)],
    [dict(d=2, n=1, L=256, J_kind=2, J_sigma=0.3, seed=9), dict(d=3, n=1, L=8, seed=10)],
]

BETA = {1: 0.44, 2: 1.12, 3: 0.693}


def _lattice(smc_gpu, kw):
    kw = dict(kw)
    d, n, L = kw.pop("d"), kw.pop("n"), kw.pop("L")
    lat = smc_gpu.Lattice(d, n, L, **kw)
    lat.sweep(BETA[n], 3)
    return lat


@pytest.mark.parametrize("seq", range(len(SEQUENCES)))
def test_noalloc_measure_matches_workspace_measure(smc_gpu, seq):
    import torch
    lats = [_lattice(smc_gpu, kw) for kw in SEQUENCES[seq]]
    for k in (0, 1, 0):
        lat = lats[k]
        print(f"noalloc measure: sequence {seq}, lattice {SEQUENCES[seq][k]}", flush=True)
        want = torch.zeros(8, dtype=torch.int64, device=lat.device)
        got = torch.full((8,), -1, dtype=torch.int64, device=lat.device)
        lat.measure_async(want)
        lat.measure_noalloc(got)
        torch.cuda.synchronize()
        assert torch.equal(got.cpu(), want.cpu()), (seq, k, got.cpu(), want.cpu())
        o = smc_gpu.Lattice.decode_obs(got.view(1, 8))[0]
        assert o.sweep == 3
        if lat.n == 1 and not lat.params.J_kind == smc_gpu.J_FP32:
            assert o.E_int != 0 and o.E == o.E_int * lat.params.J0
