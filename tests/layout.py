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


@functools.lru_cache(maxsize=8)
def natural_neighbours(d: int, L: int) -> np.ndarray:
    """[N, 2d] natural indices of the +x, -x, +y, -y(, +z, -z) neighbours
    (periodic)."""
    N = L ** d
    i = np.arange(N, dtype=np.int64)
    co = [i % L, (i // L) % L] + ([i // (L * L)] if d == 3 else [])
    out = np.empty((N, 2 * d), dtype=np.int64)
    for mu in range(d):
        for k, step in enumerate((1, -1)):
            c2 = list(co)
            c2[mu] = (co[mu] + step) % L
            out[:, 2 * mu + k] = sum(c2[a] * L ** a for a in range(d))
    return out


def natural_colours(d: int, L: int) -> np.ndarray:
    """Colour (x + y + z) % 2 of each natural site."""
    N = L ** d
    i = np.arange(N, dtype=np.int64)
    s = i % L + (i // L) % L + (i // (L * L) if d == 3 else 0)
    return (s & 1).astype(np.int8)
