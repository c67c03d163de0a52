"""Exact results used to pin the oracle -- TEST INFRASTRUCTURE.

Nothing here calls the C oracle or the HIP path; these are independent
computations from the mathematics of the model:

* brute-force enumeration of small periodic Ising lattices (Eq. (1) of the
  paper with J = 1), giving the density of states, ln Z and canonical means;
* Kaufman's exact partition function of the finite m x n torus (B. Kaufman,
  Phys. Rev. 76, 1232 (1949); in the form used by A. E. Ferdinand and
  M. E. Fisher, Phys. Rev. 185, 832 (1969)), evaluated in mpmath;
* Onsager's critical coupling and infinite-lattice energy;
* exact propagation of the probability distribution over all 2^16 states of
  the 4 x 4 torus under the checkerboard Metropolis half-sweeps, built site by
  site from p_acc = min[1, exp(-beta dE)] (Eq. (2)) with exact exponentials;
* single-spin averages in a frozen local field (Ising tanh, XY Bessel ratio,
  Heisenberg Langevin function).
"""
from __future__ import annotations

import math

import mpmath as mp
import numpy as np

# --------------------------------------------------------------------------
# Enumeration of a periodic L x L Ising torus (J = 1)
# --------------------------------------------------------------------------


def enumerate_torus(L: int):
    """All 2^(L*L) states of the L x L torus; returns (E, M) int arrays.

    Bit i of the state index is site i = x + L*y; bit 1 means spin -1.
    Each nearest-neighbour bond is counted once (forward bonds)."""
    N = L * L
    assert N <= 20
    states = np.arange(1 << N, dtype=np.int64)
    spins = 1 - 2 * ((states[:, None] >> np.arange(N)[None, :]) & 1)  # [S, N]
    E = np.zeros(len(states), dtype=np.int64)
    for y in range(L):
        for x in range(L):
            i = x + L * y
            right = (x + 1) % L + L * y
            down = x + L * ((y + 1) % L)
            E -= spins[:, i] * spins[:, right]
            E -= spins[:, i] * spins[:, down]
    M = spins.sum(axis=1)
    return E, M


def canonical_means(E: np.ndarray, M: np.ndarray, beta: float, N: int):
    """<e>, <|m|>, <m^2>, ln Z from enumerated energies/magnetisations (mpmath)."""
    mp.mp.dps = 40
    Es, counts = np.unique(np.stack([E, np.abs(M)]), axis=1, return_counts=True)
    Z = mp.mpf(0)
    sE = mp.mpf(0)
    sM = mp.mpf(0)
    sM2 = mp.mpf(0)
    for (e, m), g in zip(Es.T, counts):
        w = g * mp.e ** (-beta * int(e))
        Z += w
        sE += w * int(e)
        sM += w * int(m)
        sM2 += w * int(m) ** 2
    return (float(sE / Z / N), float(sM / Z / N), float(sM2 / Z / N ** 2), float(mp.log(Z)))


# --------------------------------------------------------------------------
# Kaufman's finite torus partition function
# --------------------------------------------------------------------------


def kaufman_lnZ(m: int, n: int, K, dps: int = 50):
    """ln Z of the m x n periodic Ising torus at coupling K = beta J.

    Z = 1/2 (2 sinh 2K)^{mn/2} (Z1 + Z2 + Z3 + Z4) with
    Z1 = prod_r 2 cosh(m g_{2r+1}/2), Z2 = prod_r 2 sinh(m g_{2r+1}/2),
    Z3 = prod_r 2 cosh(m g_{2r}/2),   Z4 = prod_r 2 sinh(m g_{2r}/2),
    r = 0..n-1, cosh g_l = cosh 2K coth 2K - cos(pi l / n) for l >= 1 and the
    signed g_0 = 2K + ln tanh K."""
    with mp.workdps(dps):
        K = mp.mpf(K)
        c = mp.cosh(2 * K) * mp.coth(2 * K)

        def gamma(l):
            if l == 0:
                return 2 * K + mp.log(mp.tanh(K))
            return mp.acosh(c - mp.cos(mp.pi * l / n))

        Z1 = Z2 = Z3 = Z4 = mp.mpf(1)
        for r in range(n):
            go = gamma(2 * r + 1)
            ge = gamma(2 * r)
            Z1 *= 2 * mp.cosh(m * go / 2)
            Z2 *= 2 * mp.sinh(m * go / 2)
            Z3 *= 2 * mp.cosh(m * ge / 2)
            Z4 *= 2 * mp.sinh(m * ge / 2)
        Z = mp.mpf(1) / 2 * (2 * mp.sinh(2 * K)) ** (mp.mpf(m * n) / 2) * (Z1 + Z2 + Z3 + Z4)
        return mp.log(Z)


def kaufman_energy(L: int, beta: float, dps: int = 60) -> float:
    """Exact energy per site -d lnZ/d beta / N of the L x L torus (J = 1), by a
    central difference with step 1e-20 at dps digits (truncation error ~1e-40)."""
    with mp.workdps(dps):
        b = mp.mpf(beta)
        h = mp.mpf(10) ** -20
        d = (kaufman_lnZ(L, L, b + h, dps) - kaufman_lnZ(L, L, b - h, dps)) / (2 * h)
        return float(-d / (L * L))


# --------------------------------------------------------------------------
# Onsager
# --------------------------------------------------------------------------


def onsager_beta_c() -> float:
    """beta_c = ln(1 + sqrt 2) / 2 for the square-lattice Ising model, J = 1."""
    return 0.5 * math.log(1.0 + math.sqrt(2.0))


def onsager_energy(beta: float) -> float:
    """Infinite-lattice energy per site,
    e = -coth 2K [1 + (2/pi)(2 tanh^2 2K - 1) K(q^2)], q = 2 sinh 2K / cosh^2 2K."""
    with mp.workdps(40):
        K = mp.mpf(beta)
        q = 2 * mp.sinh(2 * K) / mp.cosh(2 * K) ** 2
        e = -mp.coth(2 * K) * (1 + 2 / mp.pi * (2 * mp.tanh(2 * K) ** 2 - 1) * mp.ellipk(q * q))
        return float(e)


# --------------------------------------------------------------------------
# Exact propagation on small lattices (4 x 4 torus, 2 x 2 x 2 cube)
# --------------------------------------------------------------------------


class SmallLatticeChain:
    """Distribution over all 2^N states of a small periodic Ising lattice
    (d = 2 or 3, N = L^d <= 16, couplings J (+-1, natural order [d][N]) or 1)
    under the checkerboard Metropolis dynamics of Eq. (2).

    One half-sweep of colour c flips every colour-c site independently with
    probability min(1, exp(-beta dE_i)), dE_i = 2 s_i h_i depending only on s_i
    and its (other-colour) neighbours; it is applied here as the product of the
    single-site kernels of the colour-c sites, which commute.  For L = 2 the
    +mu and -mu neighbours coincide and both bonds count."""

    def __init__(self, d: int, L: int, beta: float, J=None):
        self.d, self.L, self.N, self.beta = d, L, L ** d, beta
        N = self.N
        assert N <= 16
        S = 1 << N
        states = np.arange(S, dtype=np.int64)
        self.spins = 1 - 2 * ((states[:, None] >> np.arange(N)[None, :]) & 1)
        Jb = np.ones((d, N), dtype=np.int64) if J is None else np.asarray(J, dtype=np.int64)

        def coord(i):
            return [(i // L ** a) % L for a in range(d)]

        def site(x):
            return sum(int(x[a]) * L ** a for a in range(d))

        def step(i, mu, s):
            x = coord(i)
            x[mu] = (x[mu] + s) % L
            return site(x)

        self.E = np.zeros(S, dtype=np.int64)
        for i in range(N):
            for mu in range(d):
                self.E -= Jb[mu, i] * self.spins[:, i] * self.spins[:, step(i, mu, 1)]
        self.M = self.spins.sum(axis=1)
        self.col = [sum(coord(i)) & 1 for i in range(N)]
        self.flip_prob = {}
        for i in range(N):
            h = np.zeros(S, dtype=np.int64)
            for mu in range(d):
                ip, im = step(i, mu, 1), step(i, mu, -1)
                h += Jb[mu, i] * self.spins[:, ip] + Jb[mu, im] * self.spins[:, im]
            dE = 2 * self.spins[:, i] * h
            with np.errstate(over="ignore"):
                self.flip_prob[i] = np.minimum(1.0, np.exp(-beta * dE.astype(np.float64)))

    def half_sweep(self, pi: np.ndarray, c: int) -> np.ndarray:
        idx = np.arange(len(pi), dtype=np.int64)
        for i in range(self.N):
            if self.col[i] != c:
                continue
            a = self.flip_prob[i]
            partner = idx ^ (1 << i)
            pi = pi * (1.0 - a) + pi[partner] * a[partner]
        return pi

    def sweep(self, pi: np.ndarray) -> np.ndarray:
        return self.half_sweep(self.half_sweep(pi, 0), 1)

    def boltzmann(self) -> np.ndarray:
        w = np.exp(-self.beta * (self.E - self.E.min()).astype(np.float64))
        return w / w.sum()


def TorusChain(L: int, beta: float) -> SmallLatticeChain:
    """The L x L torus with J = 1."""
    return SmallLatticeChain(2, L, beta)


def state_index(spins_natural: np.ndarray) -> np.ndarray:
    """Map int8 +-1 spin arrays [..., N] to state indices (bit i set = spin -1)."""
    bits = (np.asarray(spins_natural) < 0).astype(np.int64)
    return (bits << np.arange(bits.shape[-1])).sum(axis=-1)


# --------------------------------------------------------------------------
# Single spin in a frozen field
# --------------------------------------------------------------------------


def ising_single_spin_mean(beta_h: float) -> float:
    """<s> of an Ising spin in field h: tanh(beta h)."""
    return math.tanh(beta_h)


def xy_single_spin_mean(beta_h: float) -> float:
    """<cos theta> of a planar rotor in field h: I1(beta h) / I0(beta h)."""
    from scipy.special import ive
    return float(ive(1, beta_h) / ive(0, beta_h))


def heisenberg_single_spin_mean(beta_h: float) -> float:
    """<s . h_hat> of a classical 3-vector in field h: coth(beta h) - 1/(beta h)."""
    return 1.0 / math.tanh(beta_h) - 1.0 / beta_h


# --------------------------------------------------------------------------
# Real couplings: bond moments of the L x L torus by enumeration
# --------------------------------------------------------------------------

def torus_bond_products(L: int) -> np.ndarray:
    """x_b = s_i s_{i+mu} for every state of the L x L torus and every bond
    b = (mu, i) (site i = x + L y to its +x (mu = 0) or +y (mu = 1)
    neighbour): int8 [2^N, 2, N], state index bits as in enumerate_torus."""
    N = L * L
    assert N <= 20
    states = np.arange(1 << N, dtype=np.int64)
    spins = (1 - 2 * ((states[:, None] >> np.arange(N)[None, :]) & 1)).astype(np.int8)
    x = np.empty((len(states), 2, N), dtype=np.int8)
    for i in range(N):
        cx, cy = i % L, i // L
        x[:, 0, i] = spins[:, i] * spins[:, (cx + 1) % L + L * cy]
        x[:, 1, i] = spins[:, i] * spins[:, cx + L * ((cy + 1) % L)]
    return x


def exact_bond_moments(L: int, J: np.ndarray, beta: float, x: np.ndarray | None = None):
    """Boltzmann moments of the bond products on the L x L torus with per-bond
    couplings J[mu][i]: weights exp(beta sum_b J_b x_b) (Eq. (1)).  Returns
    (<x> [2, N], Cov(x_a, x_b) [2N, 2N], ln Z), in float64 with the weights
    shifted by their maximum before exponentiation."""
    if x is None:
        x = torus_bond_products(L)
    X = x.reshape(len(x), -1).astype(np.float64)
    a = beta * (X @ np.asarray(J, dtype=np.float64).reshape(-1))
    amax = a.max()
    w = np.exp(a - amax)
    Zs = w.sum()
    p = w / Zs
    mean = p @ X
    cov = (X * p[:, None]).T @ X - np.outer(mean, mean)
    return mean.reshape(2, L * L), cov, float(np.log(Zs) + amax)
