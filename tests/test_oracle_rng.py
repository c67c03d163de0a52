"""Pins for the oracle's random numbers (CPU only).

* Philox4x32-10 against PyTorch's independently written engine (header source
  ATen/core/PhiloxRNGEngine.h, compiled here by a test-only harness), on random
  raw (counter, key) pairs and on edge patterns.
* Statistical sanity of the counter -> bytes mapping: byte frequencies,
  hot-start magnetisation and +-J fraction within 3 sigma.
"""
import os
import shutil
import subprocess

import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))


def _torch_include():
    try:
        import torch
    except Exception:
        return None
    inc = os.path.join(os.path.dirname(torch.__file__), "include")
    return inc if os.path.exists(os.path.join(inc, "ATen", "core", "PhiloxRNGEngine.h")) else None


@pytest.fixture(scope="module")
def torch_philox(tmp_path_factory):
    inc = _torch_include()
    if inc is None or shutil.which("g++") is None:
        pytest.skip("PyTorch headers or g++ not available")
    exe = str(tmp_path_factory.mktemp("philox") / "tph")
    subprocess.run(["g++", "-std=c++17", "-O1", "-I", inc, "-o", exe,
                    os.path.join(HERE, "pins", "torch_philox_harness.cpp")], check=True)

    def run(rows):
        inp = "\n".join(" ".join(str(int(v)) for v in r) for r in rows) + "\n"
        out = subprocess.run([exe], input=inp, capture_output=True, text=True, check=True).stdout
        return [tuple(int(v) for v in line.split()) for line in out.strip().splitlines()]

    return run


def test_philox_matches_pytorch_engine(oracle_mod, torch_philox):
    rng = np.random.default_rng(1234)
    rows = [tuple(int(v) for v in r) for r in rng.integers(0, 2 ** 32, size=(4000, 6),
                                                          dtype=np.uint64)]
    M = 0xFFFFFFFF
    rows += [(0, 0, 0, 0, 0, 0), (M, M, M, M, M, M), (1, 0, 0, 0, 0, 0), (0, 0, 0, 1, 0, 0),
             (0, 0, 0, 0, 0, 1), (0x243F6A88, 0x85A308D3, 0x13198A2E, 0x03707344,
                                  0xA4093822, 0x299F31D0)]
    ref = torch_philox(rows)
    for r, want in zip(rows, ref):
        got = tuple(oracle_mod.philox4x32_10(r[:4], r[4:]))
        assert got == want, (r, got, want)


def test_philox_counter_map_is_injective_on_sample(oracle_mod):
    # a bijection of the 128-bit counter for fixed key: distinct counters in a
    # sample must give distinct blocks
    seen = set()
    for b in range(2000):
        out = tuple(oracle_mod.philox4x32_10([b, 7, 3, 2], [11, 13]))
        assert out not in seen
        seen.add(out)


def test_philox_byte_frequencies_chi2(oracle_mod):
    from scipy.stats import chi2
    counts = np.zeros(256, dtype=np.int64)
    for b in range(4096):
        for w in oracle_mod.philox4x32_10([b, 5, 0, 0], [1, 0]):
            for k in range(4):
                counts[(w >> (8 * k)) & 0xFF] += 1
    expected = counts.sum() / 256
    stat = ((counts - expected) ** 2 / expected).sum()
    assert stat < chi2.ppf(0.9999, 255)


def test_u01_exact_and_symmetric(oracle_mod):
    # u01 takes (2k+1)/2^24, exactly representable in float32, symmetric about 1/2
    for w in (0, 1, 511, 512, 0xFFFFFFFF, 0x80000000, 0x7FFFFFFF, 12345678):
        u = oracle_mod.u01(w)
        assert 0.0 < u < 1.0
        assert float(np.float32(u)) == u
        assert u == ((w >> 9) * 2 + 1) / 2 ** 24
    assert oracle_mod.u01(0) + oracle_mod.u01(0xFFFFFFFF) == 1.0


@pytest.mark.parametrize("d,L", [(2, 64), (3, 16)])
def test_hot_start_is_balanced(oracle_mod, d, L):
    lat = oracle_mod.OracleLattice(d, 1, L, seed=99)
    N = L ** d
    m = int(lat.s.astype(np.int64).sum())
    assert abs(m) < 3 * np.sqrt(N)
    assert set(np.unique(lat.s)) <= {-1, 1}


def test_pm_couplings_are_balanced(oracle_mod):
    lat = oracle_mod.OracleLattice(3, 1, 16, seed=5, J_kind=oracle_mod.J_PM)
    n = lat.J.size
    plus = int((lat.J == 1).sum())
    assert set(np.unique(lat.J)) <= {-1, 1}
    assert abs(plus - n / 2) < 3 * np.sqrt(n / 4)


def test_gaussian_couplings_moments(oracle_mod):
    lat = oracle_mod.OracleLattice(2, 1, 64, seed=5, J_kind=oracle_mod.J_FP32, J0=1.0,
                                   J_sigma=0.1)
    J = lat.J.astype(np.float64).ravel()
    n = J.size
    assert abs(J.mean() - 1.0) < 3 * 0.1 / np.sqrt(n)
    assert abs(J.std() - 0.1) < 3 * 0.1 / np.sqrt(2 * n)


def test_continuous_hot_start_unit_and_isotropic(oracle_mod):
    for n, d, L in ((2, 2, 64), (3, 3, 16)):
        lat = oracle_mod.OracleLattice(d, n, L, seed=3)
        norms = np.sqrt((lat.s ** 2).sum(axis=0))
        assert np.all(np.abs(norms - 1.0) < 1e-6)
        N = L ** d
        for k in range(n):
            assert abs(lat.s[k].mean()) < 3 * np.sqrt(1.0 / n / N)
