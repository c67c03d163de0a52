"""Host checks of the benchmark configuration: the proposal widths give about
half acceptance at the benchmark temperatures (measured with the oracle), and
the multi-GPU request is refused."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


@pytest.mark.parametrize("name,L", [("xy", 32), ("heisenberg", 8)])
def test_proposal_width_gives_half_acceptance(oracle_mod, name, L):
    wl = bench.WORKLOADS[name]
    ref = oracle_mod.OracleLattice(wl["d"], wl["n"], L, 21, delta=wl["delta"], renorm_every=100)
    ref.sweep(wl["beta"], 200)
    _, st = ref.sweep(wl["beta"], 200)
    rate = st.n_accept / st.n_attempt
    assert 0.45 <= rate <= 0.55, rate


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=60)
    assert r.returncode == 2
    assert "one GPU" in r.stdout


def test_batched_workload_matches_the_spin_glass_configuration():
    wl = bench.WORKLOADS["batched"]
    Ls = [wl["Ls"][r % 5] for r in range(wl["lattices"])]
    assert abs(sum(L ** 3 for L in Ls) - 2.17e7) < 0.01e7
