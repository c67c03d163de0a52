"""Test-side index maps between the oracle's natural site order and the GPU's
colour-split layout (pure index permutations; no model arithmetic).

Site i = x + L*y + L*L*z has colour c = (x+y+z) % 2 and in-colour index
j = i // 2; the GPU stores plane c at offset c*N/2 + j."""
import functools

import numpy as np


@functools.lru_cache(maxsize=4)
def split_index(d: int, L: int) -> np.ndarray:
    """perm[i] = position of natural site i in the flattened [2, N/2] layout."""
    N = L ** d
    i = np.arange(N, dtype=np.int64)
    x = i % L
    y = (i // L) % L
    z = i // (L * L) if d == 3 else np.zeros_like(i)
    c = (x + y + z) & 1
    return c * (N // 2) + (i >> 1)


def to_split(a: np.ndarray, d: int, L: int) -> np.ndarray:
    """Natural order [..., N] -> colour-split [..., 2, N/2]."""
    a = np.asarray(a)
    N = L ** d
    out = np.empty_like(a)
    out[..., split_index(d, L)] = a
    return out.reshape(a.shape[:-1] + (2, N // 2))


def to_natural(a: np.ndarray, d: int, L: int) -> np.ndarray:
    """Colour-split [..., 2, N/2] -> natural order [..., N]."""
    a = np.asarray(a)
    N = L ** d
    flat = a.reshape(a.shape[:-2] + (N,))
    return flat[..., split_index(d, L)]
