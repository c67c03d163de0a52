"""Host-side checks of the C-ABI library (no GPU compute): it loads, exports
every function include/smc.h declares, sizes buffers and rejects invalid
parameters before touching any device."""
import ctypes as C
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def smc_host():
    import paper_1107_5463_amd as smc
    if not os.path.exists(smc.lib_path()):
        from paper_1107_5463_amd import build
        build.build()
    try:
        smc.load_library()
    except OSError as e:  # pragma: no cover - HIP runtime missing on this host
        pytest.skip(f"cannot load libsmc.so: {e}")
    return smc


def declared_functions():
    src = open(os.path.join(ROOT, "include", "smc.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(smc_[a-z_]+)\s*\(", src)))


def test_header_declares_the_binding_exports(smc_host):
    assert declared_functions() == sorted(smc_host.EXPORTS)


def test_library_exports_every_declared_symbol(smc_host):
    out = subprocess.run(["nm", "-D", "--defined-only", smc_host.lib_path()], capture_output=True,
                         text=True, check=True).stdout
    exported = set(re.findall(r"\bT (smc_\w+)", out))
    missing = set(declared_functions()) - exported
    assert not missing, missing
    lib = smc_host.load_library()
    for f in declared_functions():
        assert hasattr(lib, f)


def test_library_does_not_link_the_oracle(smc_host):
    out = subprocess.run(["nm", "-D", smc_host.lib_path()], capture_output=True, text=True).stdout
    assert "oracle_" not in out
    ldd = subprocess.run(["ldd", smc_host.lib_path()], capture_output=True, text=True).stdout
    assert "liboracle" not in ldd


def test_buffer_sizes(smc_host):
    lib = smc_host.load_library()
    p = smc_host.make_params(2, 1, 16384, 1)
    assert lib.smc_spin_bytes(C.byref(p)) == 16384 ** 2
    assert lib.smc_coupling_bytes(C.byref(p)) == 0
    assert lib.smc_bond_bytes(C.byref(p)) == 2 * 16384 ** 2 * 8
    assert lib.smc_workspace_bytes(C.byref(p)) > 0
    q = smc_host.make_params(3, 3, 256, 1, J_kind=smc_host.J_FP32)
    assert lib.smc_spin_bytes(C.byref(q)) == 3 * 4 * 256 ** 3
    assert lib.smc_coupling_bytes(C.byref(q)) == 3 * 4 * 256 ** 3
    q2 = smc_host.make_params(2, 1, 64, 1, J_kind=smc_host.J_PM)
    assert lib.smc_coupling_bytes(C.byref(q2)) == 2 * 64 * 64


@pytest.mark.parametrize("kw,msg", [
    (dict(d=4), b"d must be"),
    (dict(n=4), b"n must be"),
    (dict(L=31), b"L must be even"),
    (dict(L=2), b"L must be even"),
    (dict(L=65536, d=3), b"too large"),
    (dict(J_kind=7), b"J_kind"),
    (dict(n=2, delta=0.0), b"delta"),
    (dict(n=3, delta=4.0), b"cap"),
    (dict(J0=float("inf")), b"J0"),
    (dict(renorm_every=-1), b"renorm"),
])
def test_invalid_params_rejected(smc_host, kw, msg):
    lib = smc_host.load_library()
    args = dict(d=2, n=1, L=32)
    args.update({k: v for k, v in kw.items() if k in ("d", "n", "L")})
    p = smc_host.make_params(args["d"], args["n"], args["L"], 1,
                             **{k: v for k, v in kw.items() if k not in ("d", "n", "L")})
    assert lib.smc_workspace_bytes(C.byref(p)) == 0
    h = C.c_void_p()
    rc = lib.smc_init_lattice(C.byref(h), C.byref(p), None, None, None, 0, None)
    assert rc == smc_host.SMC_EINVAL
    assert msg in lib.smc_last_error()
    assert not h.value


def test_null_handle_calls_fail_cleanly(smc_host):
    lib = smc_host.load_library()
    assert lib.smc_sweep(None, 0.4, 1) == smc_host.SMC_EINVAL
    assert lib.smc_half_sweep(None, 0.4, 0) == smc_host.SMC_EINVAL
    assert lib.smc_destroy(None) == smc_host.SMC_OK
    assert b"handle" in lib.smc_last_error() or lib.smc_last_error() == b""
    assert lib.smc_version().startswith(b"libsmc")


def test_binding_fails_loudly_without_library(tmp_path, monkeypatch):
    import paper_1107_5463_amd as smc
    monkeypatch.setattr(smc, "_LIB", None)
    monkeypatch.setattr(smc, "_LIB_PATH", str(tmp_path / "missing.so"))
    with pytest.raises(ImportError):
        smc.load_library()


def test_obs_record_layout_matches_header(smc_host):
    """smc_obs is eight 8-byte fields (records packed back to back in a batch),
    in the order the header declares them."""
    src = open(os.path.join(ROOT, "include", "smc.h")).read()
    body = re.search(r"typedef struct smc_obs \{(.*?)\} smc_obs;", src, re.S).group(1)
    body = re.sub(r"/\*.*?\*/", "", body, flags=re.S)
    names = re.findall(r"\b([A-Za-z_]+)(?:\[\d+\])?\s*;", body)
    fields = [f[0] for f in smc_host._ObsC._fields_]
    assert names == fields
    assert C.sizeof(smc_host._ObsC) == 64


def test_chain_buffer_sizes_and_shapes(smc_host):
    lib = smc_host.load_library()
    assert lib.smc_chains_spin_bytes(2, 64, 256) == 256 * 64 * 64
    assert lib.smc_chains_coupling_bytes(2, 64) == 2 * 64 * 64 * 4
    assert lib.smc_chains_bond_bytes(3, 16) == 3 * 16 ** 3 * 8
    assert lib.smc_chains_workspace_bytes(2, 64, 256) >= 256 * 2 * 64 * 64 * 8 + 256 * 16
    # 2D needs L % 4 == 0, 3D even L; one chain must fit a workgroup's LDS
    for d, L in ((2, 6), (2, 2), (3, 5), (2, 100), (3, 20), (4, 8)):
        assert lib.smc_chains_spin_bytes(d, L, 1) == 0, (d, L)
    assert lib.smc_chains_spin_bytes(2, 96, 1) == 96 * 96
    assert lib.smc_chains_spin_bytes(3, 18, 1) == 18 ** 3
    assert lib.smc_chains_spin_bytes(2, 64, 0) == 0


def test_chain_init_rejects_bad_arguments(smc_host):
    lib = smc_host.load_library()
    h = C.c_void_p()
    assert lib.smc_chains_init(C.byref(h), 2, 6, 4, 0, 0, 0, None, None, None, 0, None) == smc_host.SMC_EINVAL
    assert b"multiple of 4" in lib.smc_last_error()
    assert lib.smc_chains_init(C.byref(h), 2, 8, 4, 0, 0, 0, None, None, None, 0, None) == smc_host.SMC_EINVAL
    assert b"J must be" in lib.smc_last_error()
    assert lib.smc_chains_sample(None, 0.4, 1, None) == smc_host.SMC_EINVAL
    assert lib.smc_chains_covariance(None, 0.4, 1, None, None, None, None) == smc_host.SMC_EINVAL
    assert lib.smc_chains_half_sweep(None, 0.4, 0) == smc_host.SMC_EINVAL
    assert lib.smc_chains_mean(None, None, 1, None) == smc_host.SMC_EINVAL
    assert lib.smc_chains_dot(None, None, None, None) == smc_host.SMC_EINVAL
    assert lib.smc_chains_vjp(None, 0.4, 1, None, None, None, None, None, None) == smc_host.SMC_EINVAL
    assert lib.smc_chains_lnz_grad(None, 0.4, None, None, None, None, None, None) == smc_host.SMC_EINVAL
    assert lib.smc_chains_fit_step(None, 0.4, 1.0, None, None, None) == smc_host.SMC_EINVAL
    assert lib.smc_chains_kernel_name(None) == b""


@pytest.mark.parametrize("kw,msg", [
    (dict(tile=33, hits=2, L=66), b"tile must be"),
    (dict(tile=48, hits=2, L=96), b"tile must be"),         # neither 16 nor a multiple of 32
    (dict(tile=32, hits=2, L=96), b"tile must be"),         # L / T odd
    (dict(tile=32, hits=0, L=64), b"hits must be"),
    (dict(tile=0, hits=5, L=64), b"hits must be 0 or 1"),
    (dict(tile=32, hits=1, L=64, J_kind=1), b"uniform couplings"),
    (dict(tile=32, hits=1, L=64, d=3, n=3), b"int8 Ising"),
    (dict(flags=32, n=2, L=64), b"heat-bath rule is Ising only"),
    (dict(flags=32, J_kind=2, L=64), b"heat-bath rule takes"),
    (dict(flags=16, L=96), b"L % 64"),
    (dict(flags=16 | 32, L=64), b"packed spins run the Metropolis"),
])
def test_rule_schedule_and_packing_params_rejected(smc_host, kw, msg):
    lib = smc_host.load_library()
    base = dict(d=2, n=1, L=64, J_kind=0, flags=0, tile=0, hits=0)
    base.update(kw)
    p = smc_host.make_params(base["d"], base["n"], base["L"], 1, J_kind=base["J_kind"],
                             flags=base["flags"], tile=base["tile"], hits=base["hits"])
    assert lib.smc_spin_bytes(C.byref(p)) == 0
    h = C.c_void_p()
    assert lib.smc_init_lattice(C.byref(h), C.byref(p), None, None, None, 0, None) == smc_host.SMC_EINVAL
    assert msg in lib.smc_last_error(), lib.smc_last_error()


def test_packed_buffer_sizes(smc_host):
    lib = smc_host.load_library()
    p = smc_host.make_params(2, 1, 16384, 1, flags=smc_host.FLAG_PACKED)
    assert lib.smc_spin_bytes(C.byref(p)) == 16384 ** 2 // 8
    q = smc_host.make_params(3, 1, 128, 1, J_kind=smc_host.J_PM, flags=smc_host.FLAG_PACKED)
    assert lib.smc_coupling_bytes(C.byref(q)) == 3 * 128 ** 3 // 8
    assert lib.smc_bond_bytes(C.byref(q)) == 0


@pytest.mark.parametrize("d,L,T", [(2, 64, 16), (3, 32, 16), (2, 64, 32), (2, 512, 256)])
def test_tile_sizes_accepted(smc_host, d, L, T):
    """The paper's 16 x 16 tiles and multiples of 32 pass validation."""
    lib = smc_host.load_library()
    p = smc_host.make_params(d, 1, L, 1, tile=T, hits=3)
    assert lib.smc_spin_bytes(C.byref(p)) == L ** d


def test_noalloc_measure_rejects_before_touching_the_device(smc_host):
    """smc_measure_noalloc validates its arguments on the host: bad parameters,
    misaligned pointers, and a packed lattice whose reduction needs more
    partials than the library's static scratch holds (N/2 > 2^27) fail with
    SMC_EINVAL and a message before any HIP call (the pointers here are never
    dereferenced)."""
    lib = smc_host.load_library()
    dev = C.c_void_p(1 << 20)  # aligned, never used
    big = smc_host.make_params(2, 1, 32768, 1, flags=smc_host.FLAG_PACKED)
    assert lib.smc_measure_noalloc(C.byref(big), dev, None, 0, dev, None) == smc_host.SMC_EINVAL
    msg = lib.smc_last_error()
    assert b"too large for the allocation-free measurement" in msg and b"16384" in msg, msg
    ok = smc_host.make_params(2, 1, 64, 1)
    assert lib.smc_measure_noalloc(C.byref(ok), C.c_void_p((1 << 20) + 4), None, 0, dev,
                                   None) == smc_host.SMC_EINVAL
    assert b"16-byte aligned" in lib.smc_last_error()
    assert lib.smc_measure_noalloc(C.byref(ok), dev, None, 0, C.c_void_p((1 << 20) + 4),
                                   None) == smc_host.SMC_EINVAL
    assert b"dev_obs" in lib.smc_last_error()
    pm = smc_host.make_params(2, 1, 64, 1, J_kind=smc_host.J_PM)
    assert lib.smc_measure_noalloc(C.byref(pm), dev, None, 0, dev, None) == smc_host.SMC_EINVAL
    assert b"J must be" in lib.smc_last_error()
    bad = smc_host.make_params(2, 1, 31, 1)
    assert lib.smc_measure_noalloc(C.byref(bad), dev, None, 0, dev, None) == smc_host.SMC_EINVAL
    assert lib.smc_measure_noalloc(None, dev, None, 0, dev, None) == smc_host.SMC_EINVAL
