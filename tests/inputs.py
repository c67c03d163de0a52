"""Seeded synthetic inputs shared by the oracle and the GPU side of the tests.

Holds none of the method's arithmetic: only random configurations to upload
into both (natural site order, numpy)."""
import numpy as np


def random_ising(N: int, seed: int) -> np.ndarray:
    """int8 +-1 spins, independent and equiprobable."""
    rng = np.random.default_rng(seed)
    return rng.choice(np.array([-1, 1], dtype=np.int8), size=N)


def random_unit_vectors(n: int, N: int, seed: int) -> np.ndarray:
    """[n, N] float64 holding FP32-representable unit vectors (isotropic)."""
    rng = np.random.default_rng(seed)
    v = rng.standard_normal((n, N))
    v /= np.sqrt((v ** 2).sum(axis=0))
    return v.astype(np.float32).astype(np.float64)


def random_pm_couplings(d: int, N: int, seed: int) -> np.ndarray:
    rng = np.random.default_rng(seed)
    return rng.choice(np.array([-1, 1], dtype=np.int8), size=(d, N))
