"""FP64 CPU oracle for the checkerboard Metropolis chain -- TEST INFRASTRUCTURE.

Only the test suite, the smoke check and the benchmark's CPU-baseline leg may
import this package.  The product library (paper_1107_5463_amd) never imports,
links or calls it, and it shares no code with the HIP path.

The arithmetic lives in smc_oracle.c (plain C, double precision, natural site
order i = x + L*y + L*L*z); this module only marshals numpy arrays through
ctypes.  Spins: int8 [N] for Ising, float64 [n, N] for XY / Heisenberg.
Couplings: int8 [d, N] (+-1, scaled by J0) or float32 [d, N] (bond (i, i+mu)).
"""
from __future__ import annotations

import ctypes as C
import dataclasses
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
# SMC_ORACLE_LIB: another build of the same source (the sanitizer leg of the
# tests loads an AddressSanitizer / UBSan build this way)
LIB_PATH = os.environ.get("SMC_ORACLE_LIB") or os.path.join(HERE, "liboracle.so")

J_UNIFORM, J_PM, J_FP32 = 0, 1, 2


class _Params(C.Structure):
    _fields_ = [("d", C.c_int32), ("n", C.c_int32), ("L", C.c_int32), ("J_kind", C.c_int32),
                ("seed", C.c_uint64), ("replica", C.c_uint32), ("renorm_every", C.c_int32),
                ("J0", C.c_double), ("J_sigma", C.c_double), ("delta", C.c_double)]


class _Stats(C.Structure):
    _fields_ = [("n_attempt", C.c_int64), ("n_accept", C.c_int64), ("dE_units", C.c_int64),
                ("dE", C.c_double), ("n_near", C.c_int64)]


class _Obs(C.Structure):
    _fields_ = [("E_int", C.c_int64), ("M_int", C.c_int64), ("E", C.c_double),
                ("M", C.c_double * 3), ("absM", C.c_double)]


def _load():
    if not os.path.exists(LIB_PATH):
        from . import build as _b  # noqa: F401  (build on first use)
        _b.build()
    lib = C.CDLL(LIB_PATH)
    P = C.POINTER(_Params)
    vp = C.c_void_p
    lib.oracle_philox4x32_10.argtypes = [C.POINTER(C.c_uint32), C.POINTER(C.c_uint32),
                                         C.POINTER(C.c_uint32)]
    lib.oracle_philox4x32_10.restype = None
    lib.oracle_u01.argtypes = [C.c_uint32]
    lib.oracle_u01.restype = C.c_double
    lib.oracle_threshold.argtypes = [C.c_double, C.c_double]
    lib.oracle_threshold.restype = C.c_uint64
    lib.oracle_init_ising.argtypes = [P, C.c_int, vp]
    lib.oracle_init_continuous.argtypes = [P, C.c_int, vp]
    lib.oracle_init_couplings.argtypes = [P, vp]
    lib.oracle_half_sweep.argtypes = [P, vp, vp, C.c_double, C.c_uint64, C.c_int,
                                      C.POINTER(_Stats), vp]
    lib.oracle_renormalize.argtypes = [P, vp]
    lib.oracle_renormalize.restype = None
    lib.oracle_measure.argtypes = [P, vp, vp, C.POINTER(_Obs)]
    lib.oracle_measure.restype = None
    lib.oracle_bond_accumulate.argtypes = [P, vp, vp]
    lib.oracle_bond_accumulate.restype = None
    lib.oracle_sweeps.argtypes = [P, vp, vp, C.c_double, C.c_uint64, C.c_int64, C.c_int64,
                                  C.POINTER(_Obs), C.POINTER(_Stats)]
    lib.oracle_ensemble_ising.argtypes = [P, vp, vp, C.c_double, C.c_uint64, C.c_int64,
                                          C.c_int64, vp]
    lib.oracle_num_threads.restype = C.c_int
    for f in ("oracle_init_ising", "oracle_init_continuous", "oracle_init_couplings",
              "oracle_half_sweep", "oracle_sweeps", "oracle_ensemble_ising"):
        getattr(lib, f).restype = C.c_int
    return lib


_LIB = None


def lib():
    global _LIB
    if _LIB is None:
        _LIB = _load()
    return _LIB


def philox4x32_10(counter, key):
    """Raw Philox4x32-10 block: counter (4 x u32), key (2 x u32) -> 4 x u32."""
    c = (C.c_uint32 * 4)(*[int(v) & 0xFFFFFFFF for v in counter])
    k = (C.c_uint32 * 2)(*[int(v) & 0xFFFFFFFF for v in key])
    o = (C.c_uint32 * 4)()
    lib().oracle_philox4x32_10(c, k, o)
    return [int(v) for v in o]


def u01(w: int) -> float:
    return float(lib().oracle_u01(int(w) & 0xFFFFFFFF))


def threshold(beta: float, dE: float) -> int:
    """ceil(2^32 exp(-beta dE)) for dE > 0 (2^32 means always accept)."""
    return int(lib().oracle_threshold(float(beta), float(dE)))


def threshold_hb(beta: float, h: float) -> int:
    f = lib().oracle_threshold_hb
    f.argtypes = [C.c_double, C.c_double]
    f.restype = C.c_uint64
    return int(f(float(beta), float(h)))


def num_threads() -> int:
    return int(lib().oracle_num_threads())


def set_num_threads(n: int) -> None:
    """Threads of the oracle's OpenMP loops (n <= 0: one per processor)."""
    f = lib().oracle_set_num_threads
    f.argtypes = [C.c_int]
    f.restype = None
    f(int(n))


@dataclasses.dataclass
class Obs:
    E_int: int
    M_int: int
    E: float
    M: tuple
    absM: float


def _obs(o: _Obs) -> Obs:
    return Obs(int(o.E_int), int(o.M_int), float(o.E), tuple(float(v) for v in o.M),
               float(o.absM))


@dataclasses.dataclass
class Stats:
    n_attempt: int = 0
    n_accept: int = 0
    dE_units: int = 0
    dE: float = 0.0
    n_near: int = 0


class OracleLattice:
    """A lattice held by the oracle, in natural site order."""

    def __init__(self, d: int, n: int, L: int, seed: int, *, J_kind: int = J_UNIFORM,
                 J0: float = 1.0, J_sigma: float = 0.0, delta: float = 0.0,
                 renorm_every: int = 100, replica: int = 0, init: str = "hot",
                 spins=None, J=None):
        self.p = _Params(d, n, L, J_kind, seed & 0xFFFFFFFFFFFFFFFF, replica, renorm_every,
                         J0, J_sigma, delta)
        self.d, self.n, self.L = d, n, L
        self.N = L ** d
        self.t = 0
        if J_kind == J_UNIFORM:
            self.J = None
        elif J is not None:
            self.J = np.ascontiguousarray(J, dtype=np.int8 if J_kind == J_PM else np.float32)
            assert self.J.shape == (d, self.N)
        else:
            self.J = np.zeros((d, self.N), dtype=np.int8 if J_kind == J_PM else np.float32)
            rc = lib().oracle_init_couplings(C.byref(self.p), self.J.ctypes.data)
            assert rc == 0
        if spins is not None:
            self.s = np.ascontiguousarray(spins, dtype=np.int8 if n == 1 else np.float64).copy()
        elif n == 1:
            self.s = np.zeros(self.N, dtype=np.int8)
            rc = lib().oracle_init_ising(C.byref(self.p), 1 if init == "hot" else 0,
                                         self.s.ctypes.data)
            assert rc == 0
        else:
            self.s = np.zeros((n, self.N), dtype=np.float64)
            rc = lib().oracle_init_continuous(C.byref(self.p), 1 if init == "hot" else 0,
                                              self.s.ctypes.data)
            assert rc == 0

    @property
    def s(self):
        return self._s

    @s.setter
    def s(self, value):
        # the C routines take the array's buffer: keep it C-contiguous, in
        # the dtype they read
        self._s = np.ascontiguousarray(value, dtype=np.int8 if self.n == 1 else np.float64)

    @property
    def _Jp(self):
        return None if self.J is None else self.J.ctypes.data

    def half_sweep(self, beta: float, colour: int, t: int | None = None, want_margin=False):
        t = self.t if t is None else t
        st = _Stats()
        margin = np.full(self.N, np.nan) if want_margin else None
        rc = lib().oracle_half_sweep(C.byref(self.p), self.s.ctypes.data, self._Jp, float(beta),
                                     int(t), int(colour), C.byref(st),
                                     None if margin is None else margin.ctypes.data)
        if rc != 0:
            raise ValueError(f"oracle_half_sweep rejected its arguments (rc={rc})")
        out = Stats(st.n_attempt, st.n_accept, st.dE_units, st.dE, st.n_near)
        return (out, margin) if want_margin else out

    def sweep(self, beta: float, n_sweeps: int = 1, measure_every: int = 0):
        nser = n_sweeps // measure_every if measure_every > 0 else 0
        series = (_Obs * max(nser, 1))()
        st = _Stats()
        rc = lib().oracle_sweeps(C.byref(self.p), self.s.ctypes.data, self._Jp, float(beta),
                                 int(self.t), int(n_sweeps), int(measure_every), series,
                                 C.byref(st))
        if rc != 0:
            raise ValueError(f"oracle_sweeps rejected its arguments (rc={rc})")
        self.t += n_sweeps
        return [_obs(series[k]) for k in range(nser)], Stats(st.n_attempt, st.n_accept,
                                                             st.dE_units, st.dE, st.n_near)

    def sweep_rule(self, beta: float, n_sweeps: int = 1, rule: str = "metropolis", tile: int = 0,
                   hits: int = 1):
        """Ising sweeps under the Metropolis or heat-bath rule, plain (tile 0)
        or tiled k-hit (tile edge T, k = hits)."""
        f = lib().oracle_sweeps_rule
        f.argtypes = [C.POINTER(_Params), C.c_void_p, C.c_void_p, C.c_double, C.c_uint64, C.c_int64,
                      C.c_int, C.c_int, C.c_int]
        f.restype = C.c_int
        r = {"metropolis": 0, "heatbath": 1}[rule]
        rc = f(C.byref(self.p), self.s.ctypes.data, self._Jp, float(beta), int(self.t),
               int(n_sweeps), r, int(tile), int(hits))
        if rc != 0:
            raise ValueError(f"oracle_sweeps_rule rejected its arguments (rc={rc})")
        self.t += n_sweeps

    def tile_pass(self, beta: float, tile: int, hits: int, tile_colour: int,
                  rule: str = "metropolis", t: int | None = None):
        """One half of a tiled k-hit sweep: the pass over tile colour
        `tile_colour` alone, with sweep counter t (default self.t, which is
        not advanced)."""
        f = lib().oracle_tile_pass
        f.argtypes = [C.POINTER(_Params), C.c_void_p, C.c_void_p, C.c_double, C.c_uint64, C.c_int,
                      C.c_int, C.c_int, C.c_int]
        f.restype = C.c_int
        r = {"metropolis": 0, "heatbath": 1}[rule]
        rc = f(C.byref(self.p), self.s.ctypes.data, self._Jp, float(beta),
               int(self.t if t is None else t), r, int(tile), int(hits), int(tile_colour))
        if rc != 0:
            raise ValueError(f"oracle_tile_pass rejected its arguments (rc={rc})")

    def renormalize(self):
        lib().oracle_renormalize(C.byref(self.p), self.s.ctypes.data)

    def measure(self) -> Obs:
        o = _Obs()
        lib().oracle_measure(C.byref(self.p), self.s.ctypes.data, self._Jp, C.byref(o))
        return _obs(o)

    def bond_accumulate(self, acc: np.ndarray):
        assert acc.dtype == (np.int64 if self.n == 1 else np.float64)
        assert acc.shape == (self.d, self.N) and acc.flags.c_contiguous
        lib().oracle_bond_accumulate(C.byref(self.p), self.s.ctypes.data, acc.ctypes.data)

    def ensemble(self, beta: float, n_sweeps: int, n_chains: int, t0: int = 0) -> np.ndarray:
        """n_chains independent copies (replica = replica0 + k) of n_sweeps from self.s."""
        assert self.n == 1
        out = np.zeros((n_chains, self.N), dtype=np.int8)
        rc = lib().oracle_ensemble_ising(C.byref(self.p), self.s.ctypes.data, self._Jp,
                                         float(beta), int(t0), int(n_sweeps), int(n_chains),
                                         out.ctypes.data)
        assert rc == 0
        return out


def chains_ising(d: int, L: int, seed: int, J: np.ndarray, beta: float, s0: np.ndarray,
                 n_sweeps: int, t0: int = 0, replica0: int = 0, want_samples: bool = False):
    """Independent Ising chains with shared FP32 couplings J[mu][i] (natural
    order); chain k uses replica replica0 + k and starts from s0[k].

    Returns (final states [n, N], bond-product sums over chains and sweeps
    [d, N] int64, per-sweep bond products [n, n_sweeps, d, N] int8 or None,
    smallest decision margin)."""
    s0 = np.ascontiguousarray(s0, dtype=np.int8)
    n_chains, N = s0.shape
    assert N == L ** d
    Jf = np.ascontiguousarray(J, dtype=np.float32)
    assert Jf.shape == (d, N)
    p = _Params(d, 1, L, J_FP32, seed & 0xFFFFFFFFFFFFFFFF, replica0, 0, 1.0, 0.0, 0.0)
    out = np.zeros((n_chains, N), dtype=np.int8)
    bond_sum = np.zeros((d, N), dtype=np.int64)
    samples = np.zeros((n_chains, n_sweeps, d, N), dtype=np.int8) if want_samples else None
    mm = C.c_double(0.0)
    f = lib().oracle_chains_ising
    f.argtypes = [C.POINTER(_Params), C.c_void_p, C.c_void_p, C.c_double, C.c_uint64, C.c_int64,
                  C.c_int64, C.c_void_p, C.c_void_p, C.c_void_p, C.POINTER(C.c_double)]
    f.restype = C.c_int
    rc = f(C.byref(p), s0.ctypes.data, Jf.ctypes.data, float(beta), int(t0), int(n_sweeps),
           int(n_chains), out.ctypes.data, bond_sum.ctypes.data,
           None if samples is None else samples.ctypes.data, C.byref(mm))
    assert rc == 0, rc
    return out, bond_sum, samples, float(mm.value)


def init_ising(d: int, L: int, seed: int, replica: int = 0, hot: bool = True) -> np.ndarray:
    """Start state of one Ising lattice (natural order) from (seed, replica)."""
    p = _Params(d, 1, L, J_UNIFORM, seed & 0xFFFFFFFFFFFFFFFF, replica, 0, 1.0, 0.0, 0.0)
    s = np.zeros(L ** d, dtype=np.int8)
    assert lib().oracle_init_ising(C.byref(p), 1 if hot else 0, s.ctypes.data) == 0
    return s


def bond_covariance(samples: np.ndarray, g: np.ndarray):
    """Sample covariance Cov(G, x_b) over all chains and sweeps, with x the
    per-sweep bond products and G = sum_b g_b x_b: the definition, written out
    (mean of G x_b minus the product of the means)."""
    x = samples.reshape(-1, samples.shape[-2] * samples.shape[-1]).astype(np.float64)
    G = x @ np.asarray(g, dtype=np.float64).reshape(-1)
    cov = (G[:, None] * x).mean(axis=0) - G.mean() * x.mean(axis=0)
    return cov.reshape(samples.shape[-2], samples.shape[-1])


def ising_sweep_sites(lat: "OracleLattice", beta: float, t: int, sites) -> np.ndarray:
    """Spins of the given natural sites after one sweep with counter t, from
    lat.s as the state before the sweep (lat is not modified)."""
    import numpy as _np
    sites = _np.ascontiguousarray(sites, dtype=_np.int64)
    out = _np.zeros(len(sites), dtype=_np.int8)
    f = lib().oracle_ising_sweep_sites
    f.argtypes = [C.POINTER(_Params), C.c_void_p, C.c_void_p, C.c_double, C.c_uint64, C.c_int64,
                  C.c_void_p, C.c_void_p]
    f.restype = C.c_int
    rc = f(C.byref(lat.p), lat.s.ctypes.data, lat._Jp, float(beta), int(t), len(sites),
           sites.ctypes.data, out.ctypes.data)
    assert rc == 0
    return out
