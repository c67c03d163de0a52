"""Python binding of libsmc: checkerboard Metropolis sweeps of O(n) lattice spin
models on MI355X.

Argument marshalling only: buffers are torch tensors on the GPU, their
pointers and the current torch stream are handed to the C ABI of
include/smc.h, and every step of the update runs in the HIP kernels of
libsmc.so.  There is no CPU fallback: without the built library (python -m
paper_1107_5463_amd.build) every call raises.

Layouts (see include/smc.h): site i = x + L*y + L*L*z has colour
c = (x+y+z) % 2 and index j = i // 2 within its colour.
  Ising spins        int8    [2, N/2]          (+1 / -1)
  XY / Heisenberg    float32 [n, 2, N/2]
  couplings          int8 / float32 [d, 2, N/2] (bond from (c, j) to its +mu neighbour)
  bond accumulators  int64 / float64 [d, 2, N/2]
"""
from __future__ import annotations

import ctypes as C
import dataclasses
import math
import os

__all__ = ["Lattice", "Batch", "Chains", "SmcError", "load_library", "lib_path", "Obs", "J_UNIFORM", "J_PM",
           "J_FP32", "EXPORTS"]

_HERE = os.path.dirname(os.path.abspath(__file__))
# SMC_LIBRARY: another build of the same sources (the tests' sanitizer leg
# loads one whose host code is built with AddressSanitizer and UBSan)
_LIB_PATH = os.environ.get("SMC_LIBRARY") or os.path.join(_HERE, "libsmc.so")

J_UNIFORM, J_PM, J_FP32 = 0, 1, 2
INIT_HOT, INIT_COLD, INIT_KEEP = 0, 1, 2
FLAG_FAST_MATH, FLAG_SCHEDULE_FUSED, FLAG_GENERIC_KERNEL, FLAG_COUPLINGS_KEEP = 1, 2, 4, 8
FLAG_PACKED = 16
FLAG_HEATBATH = 32
BOND_RESET, BOND_ACCUMULATE, BOND_READ = 0, 1, 2
SMC_OK, SMC_EINVAL, SMC_ERANGE, SMC_EDEVICE, SMC_ESTATE = 0, -1, -2, -3, -4

# every symbol declared in include/smc.h
EXPORTS = ["smc_spin_bytes", "smc_coupling_bytes", "smc_workspace_bytes", "smc_bond_bytes",
           "smc_init_lattice", "smc_set_stream", "smc_sweep", "smc_sweep_measure", "smc_half_sweep",
           "smc_measure",
           "smc_measure_async", "smc_measure_noalloc", "smc_bond_correlations", "smc_get_samples", "smc_set_samples",
           "smc_renormalize", "smc_validate", "smc_get_sweep_index", "smc_set_sweep_index",
           "smc_kernel_name", "smc_autotune", "smc_destroy", "smc_last_error", "smc_version",
           "smc_batch_spin_bytes", "smc_batch_coupling_bytes", "smc_batch_workspace_bytes",
           "smc_batch_offsets", "smc_batch_init", "smc_batch_sweep", "smc_batch_sweep_series",
           "smc_batch_autotune", "smc_batch_lattice_packed", "smc_batch_set_schedule",
           "smc_batch_get_schedule",
           "smc_batch_use_graph", "smc_batch_get_sweep_index", "smc_batch_set_sweep_index",
           "smc_batch_destroy",
           "smc_chains_spin_bytes", "smc_chains_coupling_bytes", "smc_chains_bond_bytes",
           "smc_chains_workspace_bytes", "smc_chains_init", "smc_chains_sample",
           "smc_chains_covariance", "smc_chains_half_sweep", "smc_chains_kernel_name",
           "smc_chains_mean", "smc_chains_dot", "smc_chains_vjp", "smc_chains_lnz_grad",
           "smc_chains_fit_step",
           "smc_chains_get_sweep_index", "smc_chains_set_sweep_index",
           "smc_chains_destroy", "smc_pack_spins", "smc_unpack_spins", "smc_probe"]


class SmcError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"smc error {code}: {msg}")
        self.code = code
        self.msg = msg


class Params(C.Structure):
    _fields_ = [("d", C.c_int32), ("n", C.c_int32), ("L", C.c_int32), ("J_kind", C.c_int32),
                ("seed", C.c_uint64), ("replica", C.c_uint32), ("init", C.c_int32),
                ("J0", C.c_double), ("J_sigma", C.c_double), ("delta", C.c_double),
                ("renorm_every", C.c_int32), ("flags", C.c_int32), ("tile", C.c_int32),
                ("hits", C.c_int32)]


class _ObsC(C.Structure):
    _fields_ = [("E_int", C.c_int64), ("M_int", C.c_int64), ("E", C.c_double),
                ("M", C.c_double * 3), ("absM", C.c_double), ("sweep", C.c_int64)]


@dataclasses.dataclass
class Obs:
    E_int: int
    M_int: int
    E: float
    M: tuple
    absM: float
    sweep: int = -1  # sweep counter of the measured state


_LIB = None


def lib_path() -> str:
    return _LIB_PATH


def load_library():
    """Load libsmc.so (built in-tree); raises if it has not been built."""
    global _LIB
    if _LIB is not None:
        return _LIB
    if not os.path.exists(_LIB_PATH):
        raise ImportError(f"libsmc.so not built at {_LIB_PATH}; run python -m paper_1107_5463_amd.build")
    lib = C.CDLL(_LIB_PATH)
    P = C.POINTER(Params)
    vp = C.c_void_p
    sz = C.c_size_t
    for f in ("smc_spin_bytes", "smc_coupling_bytes", "smc_workspace_bytes", "smc_bond_bytes"):
        getattr(lib, f).argtypes = [P]
        getattr(lib, f).restype = sz
    lib.smc_init_lattice.argtypes = [C.POINTER(vp), P, vp, vp, vp, sz, vp]
    lib.smc_set_stream.argtypes = [vp, vp]
    lib.smc_sweep.argtypes = [vp, C.c_double, C.c_int64]
    lib.smc_sweep_measure.argtypes = [vp, C.c_double, C.c_int64, vp]
    lib.smc_half_sweep.argtypes = [vp, C.c_double, C.c_int]
    lib.smc_measure.argtypes = [vp, C.POINTER(_ObsC)]
    lib.smc_measure_async.argtypes = [vp, vp]
    lib.smc_measure_noalloc.argtypes = [P, vp, vp, C.c_int64, vp, vp]
    lib.smc_bond_correlations.argtypes = [vp, C.c_int, vp, vp]
    lib.smc_get_samples.argtypes = [vp, C.POINTER(C.c_int64)]
    lib.smc_set_samples.argtypes = [vp, C.c_int64]
    lib.smc_renormalize.argtypes = [vp]
    lib.smc_validate.argtypes = [vp]
    lib.smc_get_sweep_index.argtypes = [vp, C.POINTER(C.c_uint64)]
    lib.smc_set_sweep_index.argtypes = [vp, C.c_uint64]
    lib.smc_autotune.argtypes = [vp, C.c_double, vp, sz, C.POINTER(C.c_uint32)]
    lib.smc_kernel_name.argtypes = [vp, C.POINTER(C.c_uint32)]
    lib.smc_kernel_name.restype = C.c_char_p
    lib.smc_destroy.argtypes = [vp]
    i32p = C.POINTER(C.c_int32)
    for f in ("smc_batch_spin_bytes", "smc_batch_coupling_bytes", "smc_batch_workspace_bytes"):
        getattr(lib, f).argtypes = [C.c_int32, C.c_int32, i32p]
        getattr(lib, f).restype = sz
    lib.smc_batch_offsets.argtypes = [C.c_int32, C.c_int32, i32p, C.POINTER(C.c_int64),
                                      C.POINTER(C.c_int64)]
    lib.smc_batch_init.argtypes = [C.POINTER(vp), C.c_int32, C.c_int32, C.c_uint64, C.c_double,
                                   C.c_int32, C.c_int32, C.c_int32, i32p, C.POINTER(C.c_double),
                                   C.POINTER(C.c_uint32), vp, vp, vp, sz, vp]
    lib.smc_batch_sweep.argtypes = [vp, C.c_int64, vp]
    lib.smc_batch_sweep_series.argtypes = [vp, C.c_int64, C.c_int64, vp]
    lib.smc_batch_autotune.argtypes = [vp, i32p, i32p]
    lib.smc_batch_use_graph.argtypes = [vp, C.c_int32]
    lib.smc_batch_lattice_packed.argtypes = [vp, C.c_int32]
    lib.smc_batch_set_schedule.argtypes = [vp, C.c_int32, C.c_int32]
    lib.smc_batch_get_schedule.argtypes = [vp, i32p, i32p]
    lib.smc_batch_get_sweep_index.argtypes = [vp, C.POINTER(C.c_uint64)]
    lib.smc_batch_set_sweep_index.argtypes = [vp, C.c_uint64]
    lib.smc_batch_destroy.argtypes = [vp]
    for f in ("smc_chains_spin_bytes", "smc_chains_workspace_bytes"):
        getattr(lib, f).argtypes = [C.c_int32, C.c_int32, C.c_int32]
        getattr(lib, f).restype = sz
    for f in ("smc_chains_coupling_bytes", "smc_chains_bond_bytes"):
        getattr(lib, f).argtypes = [C.c_int32, C.c_int32]
        getattr(lib, f).restype = sz
    lib.smc_chains_init.argtypes = [C.POINTER(vp), C.c_int32, C.c_int32, C.c_int32, C.c_uint64,
                                    C.c_uint32, C.c_int32, vp, vp, vp, sz, vp]
    lib.smc_chains_sample.argtypes = [vp, C.c_double, C.c_int64, vp]
    lib.smc_chains_covariance.argtypes = [vp, C.c_double, C.c_int64, vp, vp, vp, vp]
    lib.smc_chains_mean.argtypes = [vp, vp, C.c_int64, vp]
    lib.smc_chains_dot.argtypes = [vp, vp, vp, vp]
    lib.smc_chains_vjp.argtypes = [vp, C.c_double, C.c_int64, vp, vp, vp, vp, vp, vp]
    lib.smc_chains_lnz_grad.argtypes = [vp, C.c_double, vp, vp, vp, vp, vp, vp]
    lib.smc_chains_fit_step.argtypes = [vp, C.c_double, C.c_double, vp, vp, vp]
    lib.smc_chains_half_sweep.argtypes = [vp, C.c_double, C.c_int]
    lib.smc_chains_kernel_name.argtypes = [vp]
    lib.smc_chains_kernel_name.restype = C.c_char_p
    lib.smc_chains_get_sweep_index.argtypes = [vp, C.POINTER(C.c_uint64)]
    lib.smc_chains_set_sweep_index.argtypes = [vp, C.c_uint64]
    lib.smc_chains_destroy.argtypes = [vp]
    lib.smc_probe.argtypes = [C.c_int32, C.c_uint32, C.c_uint32, vp, vp]
    lib.smc_pack_spins.argtypes = [vp, vp, C.c_int64, vp]
    lib.smc_unpack_spins.argtypes = [vp, vp, C.c_int64, vp]
    lib.smc_last_error.restype = C.c_char_p
    lib.smc_version.restype = C.c_char_p
    for f in EXPORTS:
        if f not in ("smc_spin_bytes", "smc_coupling_bytes", "smc_workspace_bytes", "smc_bond_bytes",
                     "smc_last_error", "smc_version", "smc_kernel_name", "smc_chains_kernel_name",
                     "smc_batch_spin_bytes",
                     "smc_batch_coupling_bytes", "smc_batch_workspace_bytes"):
            getattr(lib, f).restype = C.c_int
    _LIB = lib
    return lib


def _check(rc: int):
    if rc != SMC_OK:
        raise SmcError(rc, load_library().smc_last_error().decode())


def _kind(J_kind) -> int:
    if isinstance(J_kind, str):
        return {"uniform": J_UNIFORM, "pm": J_PM, "fp32": J_FP32, "gaussian": J_FP32}[J_kind]
    return int(J_kind)


def make_params(d, n, L, seed=0, *, J_kind=J_UNIFORM, J0=1.0, J_sigma=0.0, init="hot",
                delta=None, renorm_every=100, replica=0, flags=0, tile=0, hits=0) -> Params:
    if delta is None:
        delta = 1.0 if n > 1 else 0.0
    init_k = {"hot": INIT_HOT, "cold": INIT_COLD, "keep": INIT_KEEP}[init] if isinstance(init, str) else init
    return Params(d, n, L, _kind(J_kind), seed & 0xFFFFFFFFFFFFFFFF, replica, init_k, float(J0),
                  float(J_sigma), float(delta), renorm_every, flags, tile, hits)


class Lattice:
    """One lattice on the current GPU, its state in torch tensors.

    All work is enqueued on the torch stream current at construction (or the
    one passed); nothing synchronises except measure() and validate()."""

    def __init__(self, d: int, n: int, L: int, seed: int = 0, *, J_kind=J_UNIFORM, J0: float = 1.0,
                 J_sigma: float = 0.0, init="hot", delta=None, renorm_every: int = 100,
                 replica: int = 0, fast_math: bool = False, fused: bool = False,
                 generic: bool = False, packed: bool = False, heatbath: bool = False,
                 tile: int = 0, hits: int = 0, spins=None, J=None, device=None, stream=None):
        """packed: Ising spins (and +-1 couplings) at one bit per site; then
        `spins` is int32 [2, N/64] and J int32 [d, 2, N/64] (bit k & 31 of word
        k >> 5 = site k of a plane, bit 1 = -1).  heatbath: the heat-bath rule;
        tile / hits: the tiled k-hit schedule (tile edge T, k hits per load)."""
        import torch
        lib = load_library()
        self.torch = torch
        self.device = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
        flags = (FLAG_FAST_MATH if fast_math else 0) | (FLAG_SCHEDULE_FUSED if fused else 0) | (
            FLAG_GENERIC_KERNEL if generic else 0) | (FLAG_PACKED if packed else 0) | (
            FLAG_HEATBATH if heatbath else 0)
        self.packed = packed
        if J is not None:
            flags |= FLAG_COUPLINGS_KEEP
        if spins is not None and init == "hot":
            init = "keep"
        self.params = make_params(d, n, L, seed, J_kind=J_kind, J0=J0, J_sigma=J_sigma, init=init,
                                  delta=delta, renorm_every=renorm_every, replica=replica,
                                  flags=flags, tile=tile, hits=hits)
        p = self.params
        self.d, self.n, self.L = d, n, L
        self.N = L ** d
        if lib.smc_spin_bytes(C.byref(p)) == 0:
            # let the library produce the error message
            h = C.c_void_p()
            _check(lib.smc_init_lattice(C.byref(h), C.byref(p), None, None, None, 0, None))
        shape = (2, self.N // 2) if n == 1 else (n, 2, self.N // 2)
        dt = torch.int8 if n == 1 else torch.float32
        if packed:
            shape, dt = (2, self.N // 64), torch.int32
        if spins is not None:
            spins = spins.to(self.device, dt).contiguous().view(shape)
            self.spins = spins.clone()
        else:
            self.spins = torch.empty(shape, dtype=dt, device=self.device)
        kind = p.J_kind
        if kind == J_UNIFORM:
            self.J = None
        else:
            jdt = torch.int8 if kind == J_PM else torch.float32
            jshape = (d, 2, self.N // 2)
            if packed:
                jdt, jshape = torch.int32, (d, 2, self.N // 64)
            if J is not None:
                self.J = J.to(self.device, jdt).contiguous().view(jshape).clone()
            else:
                self.J = torch.empty(jshape, dtype=jdt, device=self.device)
        wsb = lib.smc_workspace_bytes(C.byref(p))
        self.workspace = torch.empty(wsb + 256, dtype=torch.uint8, device=self.device)
        off = (-self.workspace.data_ptr()) % 256
        self._ws_ptr = self.workspace.data_ptr() + off
        self._ws_bytes = wsb
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self._h = C.c_void_p()
        _check(lib.smc_init_lattice(C.byref(self._h), C.byref(p), C.c_void_p(self.spins.data_ptr()),
                                    None if self.J is None else C.c_void_p(self.J.data_ptr()),
                                    C.c_void_p(self._ws_ptr), wsb, C.c_void_p(self.stream.cuda_stream)))
        self._acc = None

    # ------------------------------------------------------------------
    def _lib(self):
        return load_library()

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            self._lib().smc_destroy(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def t(self) -> int:
        v = C.c_uint64()
        _check(self._lib().smc_get_sweep_index(self._h, C.byref(v)))
        return int(v.value)

    @t.setter
    def t(self, value: int):
        _check(self._lib().smc_set_sweep_index(self._h, int(value)))

    def kernel(self):
        """(name, rows_per_band) of the half-sweep kernel this lattice launches."""
        rows = C.c_uint32()
        name = self._lib().smc_kernel_name(self._h, C.byref(rows)).decode()
        return name, int(rows.value)

    def autotune(self, beta: float) -> int:
        """Time the band heights of this lattice's kernel on a scratch copy of
        the spins and keep the fastest (smc_autotune); returns the height (0:
        the kernel has no bands).  The state is left as it was."""
        scratch = self.torch.empty_like(self.spins)
        rows = C.c_uint32()
        _check(self._lib().smc_autotune(self._h, float(beta), C.c_void_p(scratch.data_ptr()),
                                        scratch.numel() * scratch.element_size(), C.byref(rows)))
        return int(rows.value)

    def set_stream(self, stream):
        self.stream = stream
        _check(self._lib().smc_set_stream(self._h, C.c_void_p(stream.cuda_stream)))

    def sweep(self, beta: float, n_sweeps: int = 1):
        _check(self._lib().smc_sweep(self._h, float(beta), int(n_sweeps)))

    def sweep_measure(self, beta: float, n_sweeps: int, dev_slot):
        """n_sweeps sweeps, then the observables of the final state written to
        dev_slot (device tensor of >= 64 bytes) without synchronising."""
        assert dev_slot.is_cuda and dev_slot.numel() * dev_slot.element_size() >= 64
        _check(self._lib().smc_sweep_measure(self._h, float(beta), int(n_sweeps),
                                             C.c_void_p(dev_slot.data_ptr())))

    def half_sweep(self, beta: float, colour: int):
        _check(self._lib().smc_half_sweep(self._h, float(beta), int(colour)))

    def measure(self) -> Obs:
        o = _ObsC()
        _check(self._lib().smc_measure(self._h, C.byref(o)))
        return Obs(int(o.E_int), int(o.M_int), float(o.E), tuple(float(v) for v in o.M),
                   float(o.absM), int(o.sweep))

    def measure_async(self, dev_slot):
        """Write the observables (8 x 8-byte smc_obs layout) into a device tensor
        slot (>= 64 bytes) without synchronising."""
        assert dev_slot.is_cuda and dev_slot.numel() * dev_slot.element_size() >= 64
        _check(self._lib().smc_measure_async(self._h, C.c_void_p(dev_slot.data_ptr())))

    def measure_noalloc(self, dev_slot, stream=None):
        """smc_measure_noalloc on this lattice's parameters and buffers: the
        observables of the current state into dev_slot (>= 64 bytes) through
        the library's static scratch instead of the handle's workspace."""
        assert dev_slot.is_cuda and dev_slot.numel() * dev_slot.element_size() >= 64
        st = stream if stream is not None else self.stream
        _check(self._lib().smc_measure_noalloc(
            C.byref(self.params), C.c_void_p(self.spins.data_ptr()),
            None if self.J is None else C.c_void_p(self.J.data_ptr()), self.t,
            C.c_void_p(dev_slot.data_ptr()), C.c_void_p(st.cuda_stream)))

    @staticmethod
    def decode_obs(buf) -> list:
        """Decode a [k, 8] int64 CPU tensor of smc_obs records."""
        import numpy as np
        a = buf.cpu().numpy()
        out = []
        for row in a.reshape(-1, 8):
            f = row.view(np.float64)
            out.append(Obs(int(row[0]), int(row[1]), float(f[2]), (float(f[3]), float(f[4]),
                                                                    float(f[5])), float(f[6]), int(row[7])))
        return out

    # ------------------------------------------------------------------
    def bond_accumulator(self):
        if self._acc is None:
            t = self.torch
            self._acc = t.zeros((self.d, 2, self.N // 2),
                                dtype=t.int64 if self.n == 1 else t.float64, device=self.device)
        return self._acc

    def bond_reset(self):
        acc = self.bond_accumulator()
        _check(self._lib().smc_bond_correlations(self._h, BOND_RESET, C.c_void_p(acc.data_ptr()), None))

    def bond_accumulate(self):
        acc = self.bond_accumulator()
        _check(self._lib().smc_bond_correlations(self._h, BOND_ACCUMULATE,
                                                 C.c_void_p(acc.data_ptr()), None))

    def bond_mean(self):
        acc = self.bond_accumulator()
        out = self.torch.empty((self.d, 2, self.N // 2), dtype=self.torch.float64, device=self.device)
        _check(self._lib().smc_bond_correlations(self._h, BOND_READ, C.c_void_p(acc.data_ptr()),
                                                 C.c_void_p(out.data_ptr())))
        return out

    @property
    def samples(self) -> int:
        v = C.c_int64()
        _check(self._lib().smc_get_samples(self._h, C.byref(v)))
        return int(v.value)

    @samples.setter
    def samples(self, value: int):
        _check(self._lib().smc_set_samples(self._h, int(value)))

    def renormalize(self):
        _check(self._lib().smc_renormalize(self._h))

    def validate(self):
        _check(self._lib().smc_validate(self._h))

    # ------------------------------------------------------------------
    def state_dict(self) -> dict:
        """Everything needed to resume bit-identically (the RNG is stateless)."""
        d = {"t": self.t, "spins": self.spins.clone(), "samples": self.samples}
        if self.J is not None:
            d["J"] = self.J.clone()
        if self._acc is not None:
            d["acc"] = self._acc.clone()
        return d

    def load_state_dict(self, sd: dict):
        self.spins.copy_(sd["spins"])
        if "J" in sd and self.J is not None:
            self.J.copy_(sd["J"])
        if "acc" in sd:
            self.bond_accumulator().copy_(sd["acc"])
        self.t = sd["t"]
        self.samples = sd.get("samples", 0)


class Batch:
    """Many independent Ising lattices (edges L[r], inverse temperatures
    beta[r], replicas replica[r] or r) swept together by one persistent
    launch; lattice r follows the single-lattice chain with those parameters.
    Spins and couplings live in two flat int8 tensors; lattice views are
    available through spins_of(r) / couplings_of(r)."""

    def __init__(self, d: int, L, beta, seed: int = 0, *, J_kind=J_PM, J0: float = 1.0,
                 init="hot", replica=None, spins=None, J=None, device=None, stream=None):
        import numpy as np
        import torch
        lib = load_library()
        self.torch = torch
        self.d = d
        self.L = [int(v) for v in L]
        self.n = len(self.L)
        self.beta = [float(v) for v in beta]
        assert len(self.beta) == self.n
        self.device = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
        Larr = (C.c_int32 * self.n)(*self.L)
        self._Larr = Larr
        sb = lib.smc_batch_spin_bytes(d, self.n, Larr)
        if sb == 0:
            h = C.c_void_p()
            _check(lib.smc_batch_init(C.byref(h), d, 0, 0, 1.0, 0, 0, self.n, Larr, None, None,
                                      None, None, None, 0, None))
        jb = lib.smc_batch_coupling_bytes(d, self.n, Larr)
        wb = lib.smc_batch_workspace_bytes(d, self.n, Larr)
        so = (C.c_int64 * self.n)()
        jo = (C.c_int64 * self.n)()
        _check(lib.smc_batch_offsets(d, self.n, Larr, so, jo))
        self.spin_offsets = [int(v) for v in so]
        self.coupling_offsets = [int(v) for v in jo]
        kind = _kind(J_kind)
        self.J_kind = kind
        self.spins = torch.zeros(sb, dtype=torch.int8, device=self.device)
        if spins is not None:
            self.spins.copy_(spins.to(self.device, torch.int8).view(-1))
            init = "keep"
        self.J = torch.zeros(jb, dtype=torch.int8, device=self.device) if kind == J_PM else None
        keep_J = 0
        if J is not None and self.J is not None:
            self.J.copy_(J.to(self.device, torch.int8).view(-1))
            keep_J = 1
        self.workspace = torch.empty(wb + 256, dtype=torch.uint8, device=self.device)
        ws = self.workspace.data_ptr() + (-self.workspace.data_ptr()) % 256
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        init_k = {"hot": INIT_HOT, "cold": INIT_COLD, "keep": INIT_KEEP}[init]
        betas = (C.c_double * self.n)(*self.beta)
        reps = None if replica is None else (C.c_uint32 * self.n)(*[int(v) for v in replica])
        self._h = C.c_void_p()
        _check(lib.smc_batch_init(C.byref(self._h), d, kind, seed & 0xFFFFFFFFFFFFFFFF, float(J0),
                                  init_k, keep_J, self.n, Larr, betas, reps,
                                  C.c_void_p(self.spins.data_ptr()),
                                  None if self.J is None else C.c_void_p(self.J.data_ptr()),
                                  C.c_void_p(ws), wb, C.c_void_p(self.stream.cuda_stream)))

    def schedule(self):
        """(lanes per workgroup, largest lattice first)."""
        th, lf = C.c_int32(), C.c_int32()
        _check(load_library().smc_batch_get_schedule(self._h, C.byref(th), C.byref(lf)))
        return int(th.value), bool(lf.value)

    def set_schedule(self, threads: int, largest_first: bool = True):
        _check(load_library().smc_batch_set_schedule(self._h, int(threads), 1 if largest_first else 0))

    @property
    def threads(self) -> int:
        return self.schedule()[0]

    @threads.setter
    def threads(self, value: int):
        self.set_schedule(value, self.schedule()[1])

    def packed(self, r: int) -> bool:
        """Whether lattice r takes the packed (one bit per site) path."""
        rc = load_library().smc_batch_lattice_packed(self._h, int(r))
        if rc < 0:
            _check(rc)
        return rc == 1

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            load_library().smc_batch_destroy(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def spins_of(self, r: int):
        N = self.L[r] ** self.d
        o = self.spin_offsets[r]
        return self.spins[o:o + N].view(2, N // 2)

    def couplings_of(self, r: int):
        N = self.L[r] ** self.d
        o = self.coupling_offsets[r]
        return self.J[o:o + self.d * N].view(self.d, 2, N // 2)

    def sweep(self, n_sweeps: int, obs=None, every: int | None = None):
        """n_sweeps sweeps of every lattice in one launch.  With obs (device
        int64 tensor) the observables are written: the final state's
        ([n_lattices, 8]) or, with `every`, those after every `every` sweeps
        ([n_sweeps / every, n_lattices, 8]), recorded inside the launch."""
        ptr = None
        if obs is not None:
            recs = 1 if every is None or n_sweeps == 0 or every <= 0 else n_sweeps // every
            assert obs.is_cuda and obs.numel() >= 8 * self.n * recs
            ptr = C.c_void_p(obs.data_ptr())
        if every is None:
            _check(load_library().smc_batch_sweep(self._h, int(n_sweeps), ptr))
        else:
            _check(load_library().smc_batch_sweep_series(self._h, int(n_sweeps), int(every), ptr))

    def autotune(self):
        th = C.c_int32()
        lf = C.c_int32()
        _check(load_library().smc_batch_autotune(self._h, C.byref(th), C.byref(lf)))
        return int(th.value), bool(lf.value)

    def use_graph(self, enable: bool = True):
        _check(load_library().smc_batch_use_graph(self._h, 1 if enable else 0))

    @property
    def t(self) -> int:
        v = C.c_uint64()
        _check(load_library().smc_batch_get_sweep_index(self._h, C.byref(v)))
        return int(v.value)

    @t.setter
    def t(self, value: int):
        _check(load_library().smc_batch_set_sweep_index(self._h, int(value)))


class Chains:
    """n_chains independent Metropolis chains of one small d-dimensional Ising
    lattice with shared FP32 couplings J[mu][c][j] (bond from site (c, j) to
    its +mu neighbour), for derivatives of ln Z.  Chain k uses replica
    replica0 + k.  spins: int8 [n_chains, 2, N/2] (colour planes)."""

    def __init__(self, d: int, L: int, n_chains: int, seed: int = 0, *, J=None,
                 replica0: int = 0, init="hot", spins=None, device=None, stream=None):
        import torch
        lib = load_library()
        self.torch = torch
        self.d, self.L, self.n_chains = d, L, n_chains
        self.N = L ** d
        self.device = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
        sb = lib.smc_chains_spin_bytes(d, L, n_chains)
        if sb == 0:
            h = C.c_void_p()
            _check(lib.smc_chains_init(C.byref(h), d, L, n_chains, 0, 0, 0, None, None, None, 0,
                                       None))
        self.J = torch.ones((d, 2, self.N // 2), dtype=torch.float32, device=self.device)
        if J is not None:
            self.J.copy_(J)
        self.spins = torch.zeros((n_chains, 2, self.N // 2), dtype=torch.int8, device=self.device)
        init_k = INIT_KEEP if spins is not None else {"hot": INIT_HOT, "cold": INIT_COLD}[init]
        if spins is not None:
            self.spins.copy_(spins.view(n_chains, 2, self.N // 2))
        wb = lib.smc_chains_workspace_bytes(d, L, n_chains)
        self.workspace = torch.empty(wb + 256, dtype=torch.uint8, device=self.device)
        ws = self.workspace.data_ptr() + (-self.workspace.data_ptr()) % 256
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self._h = C.c_void_p()
        _check(lib.smc_chains_init(C.byref(self._h), d, L, n_chains, seed & 0xFFFFFFFFFFFFFFFF,
                                   replica0, init_k, C.c_void_p(self.J.data_ptr()),
                                   C.c_void_p(self.spins.data_ptr()), C.c_void_p(ws), wb,
                                   C.c_void_p(self.stream.cuda_stream)))

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            load_library().smc_chains_destroy(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def bond_zeros(self, dtype=None):
        t = self.torch
        return t.zeros((self.d, 2, self.N // 2), dtype=dtype or t.int64, device=self.device)

    def set_couplings(self, J):
        self.J.copy_(J)

    def sample(self, beta: float, n_sweeps: int, bond_sum=None):
        """n_sweeps sweeps of every chain; with bond_sum (int64 [d, 2, N/2]
        device tensor) the bond products after every sweep are added to it."""
        ptr = None
        if bond_sum is not None:
            assert bond_sum.dtype == self.torch.int64 and bond_sum.is_contiguous()
            assert bond_sum.numel() == self.d * self.N
            ptr = C.c_void_p(bond_sum.data_ptr())
        _check(load_library().smc_chains_sample(self._h, float(beta), int(n_sweeps), ptr))

    def half_sweep(self, beta: float, colour: int):
        """One colour's half of sweep t of every chain (t is not advanced)."""
        _check(load_library().smc_chains_half_sweep(self._h, float(beta), int(colour)))

    def kernel(self) -> str:
        return load_library().smc_chains_kernel_name(self._h).decode()

    def covariance(self, beta: float, n_sweeps: int, g, g_center, cov_acc, G_acc):
        """Replay of n_sweeps sampling sweeps accumulating (G - g_center) x_b
        into cov_acc and G - g_center, (G - g_center)^2 into G_acc (float64
        device tensors [d, 2, N/2] and [2]), G = sum_b g_b x_b; g_center: a
        float64 device tensor of one element (e.g. from dot), or None (0)."""
        t = self.torch
        for a in (g, cov_acc, G_acc):
            self._bonds_f64(a, full=a is not G_acc)
        assert G_acc.numel() >= 2
        gc = None
        if g_center is not None:
            self._bonds_f64(g_center, full=False)
            gc = C.c_void_p(g_center.data_ptr())
        _check(load_library().smc_chains_covariance(self._h, float(beta), int(n_sweeps),
                                                    C.c_void_p(g.data_ptr()), gc,
                                                    C.c_void_p(cov_acc.data_ptr()),
                                                    C.c_void_p(G_acc.data_ptr())))

    # -- finishing the estimates (the library's FP64 kernels) ---------------
    def _bonds_f64(self, a, full=True):
        t = self.torch
        assert a.dtype == t.float64 and a.is_contiguous() and a.is_cuda
        if full:
            assert a.numel() == self.d * self.N

    def _bonds_f32(self, a):
        t = self.torch
        assert a.dtype == t.float32 and a.is_contiguous() and a.is_cuda
        assert a.numel() == self.d * self.N

    def mean(self, bond_sum, n_samples: int):
        """<x_b> = bond_sum / n_samples (float64 [d, 2, N/2])."""
        t = self.torch
        assert bond_sum.dtype == t.int64 and bond_sum.is_contiguous() and bond_sum.is_cuda
        out = t.empty((self.d, 2, self.N // 2), dtype=t.float64, device=self.device)
        _check(load_library().smc_chains_mean(self._h, C.c_void_p(bond_sum.data_ptr()),
                                              int(n_samples), C.c_void_p(out.data_ptr())))
        return out

    def dot(self, a, w):
        """sum_b a_b w_b as a one-element float64 device tensor."""
        t = self.torch
        self._bonds_f64(a)
        self._bonds_f64(w)
        out = t.empty(1, dtype=t.float64, device=self.device)
        _check(load_library().smc_chains_dot(self._h, C.c_void_p(a.data_ptr()),
                                             C.c_void_p(w.data_ptr()), C.c_void_p(out.data_ptr())))
        return out

    def vjp(self, beta: float, n_samples: int, cov_acc, G_acc, mean, J):
        """(beta Cov(G, x_b) as float32, sum_b J_b Cov(G, x_b) as a one-element
        float64 tensor) from a covariance replay's sums."""
        t = self.torch
        for a in (cov_acc, mean):
            self._bonds_f64(a)
        self._bonds_f64(G_acc, full=False)
        self._bonds_f32(J)
        gJ = t.empty((self.d, 2, self.N // 2), dtype=t.float32, device=self.device)
        gb = t.empty(1, dtype=t.float64, device=self.device)
        _check(load_library().smc_chains_vjp(self._h, float(beta), int(n_samples),
                                             C.c_void_p(cov_acc.data_ptr()), C.c_void_p(G_acc.data_ptr()),
                                             C.c_void_p(mean.data_ptr()), C.c_void_p(J.data_ptr()),
                                             C.c_void_p(gJ.data_ptr()), C.c_void_p(gb.data_ptr())))
        return gJ, gb

    def lnz_grad(self, beta: float, mean, J, scale=None, dtype=None):
        """(scale beta <x_b>, scale sum_b J_b <x_b>): the gradients of ln Z in J
        (float32 or float64 per dtype) and beta (one-element float64);
        scale: a one-element float64 device tensor or None (1)."""
        t = self.torch
        self._bonds_f64(mean)
        self._bonds_f32(J)
        dt = dtype or t.float32
        gJ = t.empty((self.d, 2, self.N // 2), dtype=dt, device=self.device)
        gb = t.empty(1, dtype=t.float64, device=self.device)
        sp = None
        if scale is not None:
            self._bonds_f64(scale, full=False)
            sp = C.c_void_p(scale.data_ptr())
        f32 = C.c_void_p(gJ.data_ptr()) if dt == t.float32 else None
        f64 = C.c_void_p(gJ.data_ptr()) if dt == t.float64 else None
        _check(load_library().smc_chains_lnz_grad(self._h, float(beta), C.c_void_p(mean.data_ptr()),
                                                  C.c_void_p(J.data_ptr()), sp, f32, f64,
                                                  C.c_void_p(gb.data_ptr())))
        return gJ, gb

    def fit_step(self, beta: float, lr: float, target, mean, J):
        """Moment matching, in place: J += lr beta (target - <x>)."""
        self._bonds_f64(target)
        self._bonds_f64(mean)
        self._bonds_f32(J)
        _check(load_library().smc_chains_fit_step(self._h, float(beta), float(lr),
                                                  C.c_void_p(target.data_ptr()),
                                                  C.c_void_p(mean.data_ptr()), C.c_void_p(J.data_ptr())))

    @property
    def t(self) -> int:
        v = C.c_uint64()
        _check(load_library().smc_chains_get_sweep_index(self._h, C.byref(v)))
        return int(v.value)

    @t.setter
    def t(self, value: int):
        _check(load_library().smc_chains_set_sweep_index(self._h, int(value)))


def pack_spins(src, stream=None):
    """int8 +-1 sites (any shape, total a multiple of 32) -> int32 words, one
    bit per site (bit 1 = -1), in the library's kernels."""
    import torch
    assert src.dtype == torch.int8 and src.is_cuda and src.is_contiguous()
    n = src.numel()
    out = torch.empty(n // 32, dtype=torch.int32, device=src.device)
    st = stream if stream is not None else torch.cuda.current_stream(src.device)
    _check(load_library().smc_pack_spins(C.c_void_p(src.data_ptr()), C.c_void_p(out.data_ptr()), n,
                                         C.c_void_p(st.cuda_stream)))
    return out


def unpack_spins(src, stream=None):
    """Inverse of pack_spins: int32 words -> int8 +-1 sites (flat)."""
    import torch
    assert src.dtype == torch.int32 and src.is_cuda and src.is_contiguous()
    n = src.numel() * 32
    out = torch.empty(n, dtype=torch.int8, device=src.device)
    st = stream if stream is not None else torch.cuda.current_stream(src.device)
    _check(load_library().smc_unpack_spins(C.c_void_p(src.data_ptr()), C.c_void_p(out.data_ptr()),
                                           n, C.c_void_p(st.cuda_stream)))
    return out


def probe(kind: str, n_lanes: int, reps: int, out, stream=None):
    """Launch a measurement probe ("philox" or "valu"); out: int32 device
    tensor of n_lanes elements."""
    import torch
    assert out.dtype == torch.int32 and out.is_cuda and out.numel() >= n_lanes
    st = stream if stream is not None else torch.cuda.current_stream(out.device)
    _check(load_library().smc_probe({"philox": 0, "valu": 1}[kind], int(n_lanes), int(reps),
                                    C.c_void_p(out.data_ptr()), C.c_void_p(st.cuda_stream)))


def version() -> str:
    return load_library().smc_version().decode()


def beta_c_2d() -> float:
    """Onsager's critical coupling of the square-lattice Ising model."""
    return 0.5 * math.log(1.0 + math.sqrt(2.0))
