"""Precision of the FP32 continuous-spin path against the FP64 oracle, per
observable (printed, and bounded):

* measurement of one and the same FP32 state (E, M in FP64 on both sides:
  products of FP32 numbers are exact in FP64, only the summation order
  differs);
* one sweep from the same FP32 state: spin components (FP32 update against
  FP64), then E and M of the two resulting states;
* bond correlations of the resulting state.
"""
import numpy as np
import pytest

import layout

pytestmark = pytest.mark.gpu


def nat(lat):
    return layout.to_natural(lat.spins.cpu().numpy().astype(np.float64), lat.d, lat.L)


@pytest.mark.parametrize("kernel", ["stream", "row"])
@pytest.mark.parametrize("d,n,L,beta,delta", [(2, 2, 64, 1.12, 1.63), (3, 3, 16, 0.693, 2.058)])
def test_precision_per_observable(smc_gpu, oracle_mod, d, n, L, beta, delta, kernel, monkeypatch):
    import torch
    monkeypatch.setenv("SMC_CONT_KERNEL", kernel)
    monkeypatch.delenv("SMC_CONT_ROWS", raising=False)
    N = L ** d
    ref = oracle_mod.OracleLattice(d, n, L, 23, delta=delta, renorm_every=0)
    ref.s = ref.s.astype(np.float32).astype(np.float64)
    sp = torch.from_numpy(layout.to_split(ref.s.astype(np.float32), d, L))
    lat = smc_gpu.Lattice(d, n, L, seed=23, delta=delta, renorm_every=0, spins=sp)
    # the same FP32 state
    o, r = lat.measure(), ref.measure()
    e_meas = abs(o.E - r.E) / N
    m_meas = max(abs(a - b) for a, b in zip(o.M[:n], r.M[:n])) / N
    # one sweep from it
    lat.sweep(beta, 1)
    ref.sweep(beta, 1)
    g = nat(lat)
    diff = np.abs(g - ref.s).max(axis=0)
    moved_apart = int(np.sum(diff > 1e-3))  # a decision taken differently
    comp = float(diff[diff <= 1e-3].max(initial=0.0))
    o2, r2 = lat.measure(), ref.measure()
    e_sweep = abs(o2.E - r2.E) / N
    m_sweep = max(abs(a - b) for a, b in zip(o2.M[:n], r2.M[:n])) / N
    lat.bond_reset()
    lat.bond_accumulate()
    acc = np.zeros((d, N))
    ref.s = g  # the GPU's state: bond products of the same numbers
    ref.bond_accumulate(acc)
    got = layout.to_natural(lat.bond_accumulator().cpu().numpy(), d, L)
    bond = float(np.abs(got - acc).max())
    print(f"precision d={d} n={n} L={L} kernel={kernel}: same-state E/N {e_meas:.2e} M/N {m_meas:.2e};"
          f" one sweep: component max {comp:.2e}, sites decided apart {moved_apart},"
          f" E/N {e_sweep:.2e}, M/N {m_sweep:.2e}; bond products max {bond:.2e}", flush=True)
    assert e_meas <= 1e-14 and m_meas <= 1e-14
    assert comp <= 1e-5
    assert moved_apart == 0
    assert e_sweep <= 1e-5 and m_sweep <= 1e-5
    assert bond <= 1e-15
