"""GPU parity tests for Ising spins: the HIP path through the C ABI against the
FP64 CPU oracle on the same seeded inputs.  Integer work, so every comparison
is bit-exact."""
import numpy as np
import pytest

import inputs
import layout

pytestmark = pytest.mark.gpu

BETA_C = 0.4406868


def nat(lat):
    return layout.to_natural(lat.spins.cpu().numpy(), lat.d, lat.L)


def nat_J(lat):
    return layout.to_natural(lat.J.cpu().numpy(), lat.d, lat.L)


SHAPES = [(2, 32, 0), (2, 64, 1), (2, 6, 0), (2, 4, 1), (3, 16, 0), (3, 8, 1), (3, 32, 1),
          (2, 96, 0), (2, 10, 2), (3, 6, 2), (3, 64, 0), (2, 128, 1)]


@pytest.mark.parametrize("d,L,kind", SHAPES)
def test_init_parity(smc_gpu, oracle_mod, d, L, kind):
    print(f"init parity d={d} L={L} kind={kind}", flush=True)
    lat = smc_gpu.Lattice(d, 1, L, seed=1234, J_kind=kind, J0=1.0, J_sigma=0.3)
    ref = oracle_mod.OracleLattice(d, 1, L, 1234, J_kind=kind, J0=1.0, J_sigma=0.3)
    assert np.array_equal(nat(lat), ref.s)
    if kind == 1:
        assert np.array_equal(nat_J(lat), ref.J)
    if kind == 2:
        gj, oj = nat_J(lat), ref.J
        # both round the same double-precision Gaussian to FP32; allow 1 ulp
        assert np.all(np.abs(gj.view(np.int32).astype(np.int64) - oj.view(np.int32).astype(np.int64)) <= 1)
    lat.validate()


@pytest.mark.parametrize("generic", [False, True])
def test_c1_trajectory_bit_exact(smc_gpu, oracle_mod, generic):
    """2D Ising 32 x 32, J = 1, hot start seed 1, beta_c, 1000 sweeps, E and
    |M| after every sweep: the whole series and the final state match."""
    import torch
    print(f"C1 trajectory generic={generic}", flush=True)
    lat = smc_gpu.Lattice(2, 1, 32, seed=1, generic=generic)
    ref = oracle_mod.OracleLattice(2, 1, 32, 1)
    o0 = lat.measure()
    r0 = ref.measure()
    assert (o0.E_int, o0.M_int) == (r0.E_int, r0.M_int)
    slots = torch.zeros((1000, 8), dtype=torch.int64, device=lat.device)
    for k in range(1000):
        lat.sweep(BETA_C, 1)
        lat.measure_async(slots[k])
    series = smc_gpu.Lattice.decode_obs(slots)
    rser, _ = ref.sweep(BETA_C, 1000, 1)
    got = np.array([(o.E_int, o.M_int, o.absM) for o in series])
    want = np.array([(o.E_int, o.M_int, o.absM) for o in rser])
    assert np.array_equal(got, want)
    assert [o.sweep for o in series] == list(range(1, 1001))
    assert np.array_equal(nat(lat), ref.s)
    assert lat.t == 1000


def upload(smc_gpu, ref, **kw):
    """A GPU lattice holding the oracle's current state and couplings."""
    import torch
    d, L = ref.d, ref.L
    Jt = None if ref.J is None else torch.from_numpy(layout.to_split(ref.J, d, L))
    return smc_gpu.Lattice(d, 1, L, seed=int(ref.p.seed), J_kind=int(ref.p.J_kind),
                           J0=ref.p.J0, J_sigma=ref.p.J_sigma, replica=int(ref.p.replica),
                           spins=torch.from_numpy(layout.to_split(ref.s, d, L)), J=Jt, **kw)


@pytest.mark.parametrize("d,L,kind", SHAPES)
def test_sweeps_match_oracle(smc_gpu, oracle_mod, d, L, kind):
    print(f"sweep parity d={d} L={L} kind={kind}", flush=True)
    import torch
    beta = {2: 0.44, 3: 0.23}[d] if kind == 0 else 0.9
    sweeps = 12
    ref = oracle_mod.OracleLattice(d, 1, L, 77, J_kind=kind, J_sigma=0.2)
    if kind == 2:
        # FP32 couplings: the decision compares a float probability.  One
        # half-sweep at a time from the oracle's state: every site whose
        # margin |u - p| >= 1e-6 makes the oracle's decision.
        lat = upload(smc_gpu, ref)
        near = 0
        for t in range(sweeps):
            for c in (0, 1):
                lat.spins.copy_(torch.from_numpy(layout.to_split(ref.s, d, L)))
                lat.t = t
                lat.half_sweep(0.9, c)
                _, margin = ref.half_sweep(0.9, c, t, want_margin=True)
                diff = np.nonzero(nat(lat) != ref.s)[0]
                assert np.all(np.abs(margin[diff]) < 1e-6), (t, c, margin[diff])
                near += int(np.sum(np.abs(margin) < 1e-6))
        print(f"near-threshold sites: {near}")
        return
    lat = smc_gpu.Lattice(d, 1, L, seed=77, J_kind=kind, J_sigma=0.2)
    lat.sweep(beta, sweeps)
    ref.sweep(beta, sweeps)
    assert np.array_equal(nat(lat), ref.s)
    # generic one-site-per-thread kernel gives the same bits
    lat2 = smc_gpu.Lattice(d, 1, L, seed=77, J_kind=kind, generic=True)
    lat2.sweep(beta, sweeps)
    assert np.array_equal(lat2.spins.cpu().numpy(), lat.spins.cpu().numpy())


@pytest.mark.parametrize("beta", [0.0, float("inf"), 0.05, 3.0])
def test_special_temperatures(smc_gpu, oracle_mod, beta):
    for d, L in ((2, 64), (3, 32)):
        lat = smc_gpu.Lattice(d, 1, L, seed=5)
        ref = oracle_mod.OracleLattice(d, 1, L, 5)
        s0 = nat(lat)
        lat.sweep(beta, 3)
        ref.sweep(beta, 3)
        assert np.array_equal(nat(lat), ref.s)
        if beta == 0.0:
            assert np.array_equal(nat(lat), -s0)


def _sampled_sites(d, L, rng, n_random):
    N = L ** d
    sites = [rng.integers(0, N, size=n_random)]
    R = L // 2
    # chunk edges (in-colour index 0, 15, 16 of rows), lattice faces, corners
    xs = np.array([0, 1, 2, 30, 31, 32, 33, L - 2, L - 1])
    for y in (0, 1, L // 2, L - 1):
        zs = (0, 1, L - 1) if d == 3 else (0,)
        for z in zs:
            sites.append(xs + L * y + L * L * z)
    return np.unique(np.concatenate(sites))


@pytest.mark.parametrize("d,L,seed,beta", [(2, 16384, 2, BETA_C), (3, 512, 3, 0.2216546)])
def test_full_size_parity(smc_gpu, oracle_mod, d, L, seed, beta):
    """Workload sizes (2D L = 16384, 3D L = 512): the initial state, the state
    after two sweeps and E, M equal the oracle's, bit for bit."""
    print(f"full-size parity d={d} L={L}", flush=True)
    lat = smc_gpu.Lattice(d, 1, L, seed=seed)
    ref = oracle_mod.OracleLattice(d, 1, L, seed)
    assert np.array_equal(nat(lat), ref.s)
    lat.sweep(beta, 2)
    ref.sweep(beta, 2)
    assert np.array_equal(nat(lat), ref.s)
    o, r = lat.measure(), ref.measure()
    assert (o.E_int, o.M_int) == (r.E_int, r.M_int)


@pytest.mark.parametrize("d,L,seed,beta", [(2, 16384, 2, BETA_C), (3, 512, 3, 0.2216546)])
def test_full_size_sampled_late_counter(smc_gpu, oracle_mod, d, L, seed, beta):
    """One sweep from the initial state with a late sweep counter (t = 123456):
    sampled sites (random plus chunk edges, faces, corners) equal the oracle's
    site-by-site update of its own initial state."""
    print(f"full-size sampled d={d} L={L}", flush=True)
    t = 123456
    lat = smc_gpu.Lattice(d, 1, L, seed=seed)
    lat.t = t
    lat.sweep(beta, 1)
    ref = oracle_mod.OracleLattice(d, 1, L, seed)
    sites = _sampled_sites(d, L, np.random.default_rng(seed), 200_000)
    want = oracle_mod.ising_sweep_sites(ref, beta, t, sites)
    assert np.array_equal(nat(lat)[sites], want)


@pytest.mark.parametrize("d,L,kind", [(2, 32, 0), (2, 64, 1), (3, 8, 0), (3, 32, 1), (2, 12, 2),
                                      (2, 6, 0)])
def test_measure_matches_oracle(smc_gpu, oracle_mod, d, L, kind):
    import torch
    for trial in range(3):
        s = inputs.random_ising(L ** d, seed=d * 100 + L + trial)
        ref = oracle_mod.OracleLattice(d, 1, L, 9, J_kind=kind, J_sigma=0.5, spins=s)
        lat = upload(smc_gpu, ref)
        o, r = lat.measure(), ref.measure()
        assert o.M_int == r.M_int
        if kind == 2:
            assert abs(o.E - r.E) <= 1e-12 * max(1.0, abs(r.E))
        else:
            assert o.E_int == r.E_int and o.E == r.E


@pytest.mark.parametrize("d,L,kind", [(2, 32, 0), (3, 8, 1), (2, 6, 0)])
def test_bond_correlations_match_oracle(smc_gpu, oracle_mod, d, L, kind):
    lat = smc_gpu.Lattice(d, 1, L, seed=21, J_kind=kind)
    ref = oracle_mod.OracleLattice(d, 1, L, 21, J_kind=kind)
    acc = np.zeros((d, L ** d), dtype=np.int64)
    lat.bond_reset()
    for k in range(5):
        lat.sweep(0.5, 2)
        lat.bond_accumulate()
        ref.sweep(0.5, 2)
        ref.bond_accumulate(acc)
    assert lat.samples == 5
    got = layout.to_natural(lat.bond_accumulator().cpu().numpy(), d, L)
    assert np.array_equal(got, acc)
    mean = layout.to_natural(lat.bond_mean().cpu().numpy(), d, L)
    assert np.array_equal(mean, acc / 5.0)


def test_checkpoint_resume_bit_identical(smc_gpu):
    a = smc_gpu.Lattice(2, 1, 64, seed=31)
    a.sweep(BETA_C, 10)
    sd = a.state_dict()
    a.sweep(BETA_C, 10)
    b = smc_gpu.Lattice(2, 1, 64, seed=31, init="cold")
    b.load_state_dict(sd)
    assert b.t == 10
    b.sweep(BETA_C, 10)
    assert np.array_equal(a.spins.cpu().numpy(), b.spins.cpu().numpy())


def test_non_default_stream(smc_gpu):
    import torch
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        a = smc_gpu.Lattice(2, 1, 64, seed=41)
        a.sweep(BETA_C, 20)
    s.synchronize()
    b = smc_gpu.Lattice(2, 1, 64, seed=41)
    b.sweep(BETA_C, 20)
    torch.cuda.synchronize()
    assert np.array_equal(a.spins.cpu().numpy(), b.spins.cpu().numpy())


def test_abi_errors_on_device(smc_gpu):
    import torch
    lib = smc_gpu.load_library()
    import ctypes as C
    p = smc_gpu.make_params(2, 1, 32, 1)
    spins = torch.empty((2, 512), dtype=torch.int8, device="cuda")
    ws = torch.empty(lib.smc_workspace_bytes(C.byref(p)) + 512, dtype=torch.uint8, device="cuda")
    base = ws.data_ptr() + (-ws.data_ptr()) % 256
    h = C.c_void_p()
    # workspace too small
    assert lib.smc_init_lattice(C.byref(h), C.byref(p), C.c_void_p(spins.data_ptr()), None,
                                C.c_void_p(base), 16, None) == smc_gpu.SMC_EINVAL
    assert b"workspace" in lib.smc_last_error()
    # misaligned spins
    assert lib.smc_init_lattice(C.byref(h), C.byref(p), C.c_void_p(spins.data_ptr() + 1), None,
                                C.c_void_p(base), lib.smc_workspace_bytes(C.byref(p)), None) == smc_gpu.SMC_EINVAL
    lat = smc_gpu.Lattice(2, 1, 32, seed=1)
    with pytest.raises(smc_gpu.SmcError) as e:
        lat.sweep(float("nan"), 1)
    assert e.value.code == smc_gpu.SMC_EINVAL
    with pytest.raises(smc_gpu.SmcError) as e:
        lat.sweep(-1.0, 1)
    with pytest.raises(smc_gpu.SmcError) as e:
        lat.half_sweep(0.4, 2)
    lat.t = 2 ** 32 - 1
    with pytest.raises(smc_gpu.SmcError) as e:
        lat.sweep(0.4, 2)
    assert e.value.code == smc_gpu.SMC_ERANGE
    lat.sweep(0.4, 1)  # exactly reaches 2^32
    # validate flags a corrupted spin
    lat2 = smc_gpu.Lattice(2, 1, 32, seed=1)
    lat2.spins[0, 7] = 0
    with pytest.raises(smc_gpu.SmcError) as e:
        lat2.validate()
    assert e.value.code == smc_gpu.SMC_ESTATE


@pytest.mark.parametrize("d,L", [(2, 64), (2, 96), (3, 32), (2, 512), (3, 64)])
def test_kernel_variants_bit_identical(smc_gpu, oracle_mod, d, L, monkeypatch):
    """Every half-sweep kernel (one site per thread, one chunk per lane,
    streaming bands of every height) produces the oracle's chain: the same
    bits whatever the launch geometry -- this doubles as the race check."""
    ref = oracle_mod.OracleLattice(d, 1, L, 88)
    ref.sweep(0.3, 4)
    seen = set()
    for variant, rows in [("site", None), ("chunk", None), ("stream", "4"), ("stream", "8"),
                          ("stream", "16"), ("stream", "32"), ("stream", None)]:
        monkeypatch.setenv("SMC_ISING_KERNEL", variant)
        if rows is None:
            monkeypatch.delenv("SMC_STREAM_ROWS", raising=False)
        else:
            monkeypatch.setenv("SMC_STREAM_ROWS", rows)
        lat = smc_gpu.Lattice(d, 1, L, seed=88)
        seen.add(lat.kernel())
        lat.sweep(0.3, 4)
        assert np.array_equal(nat(lat), ref.s), (variant, rows, lat.kernel())
    assert {name for name, _ in seen} == {"ising_site", "ising_chunk", "ising_stream"}


@pytest.mark.parametrize("L,n,rows,kernel", [(2048, 4, None, None), (2048, 5, "4", None),
                                             (4096, 3, "8", None), (2048, 2, "64", None),
                                             (4096, 1, None, None), (2048, 4, "16", "fused_wave"),
                                             (4096, 3, None, "fused_wave"), (16384, 2, "32", "fused_wave"),
                                             (16384, 2, None, None)])
def test_fused_schedule_matches_oracle(smc_gpu, oracle_mod, L, n, rows, kernel, monkeypatch):
    """The one-kernel-per-sweep schedule (ping-pong buffers, redundant
    band-edge rows; wave segments with recomputed halo chunks, or whole-row
    workgroups with LDS edge exchange) gives the oracle's chain bit for bit,
    for odd and even sweep counts and any band height; the energy and
    magnetisation reduced inside the last fused sweep equal the oracle's."""
    import torch
    if kernel is not None:
        monkeypatch.setenv("SMC_ISING_KERNEL", kernel)
    if rows is None:
        monkeypatch.delenv("SMC_FUSED_ROWS", raising=False)
    else:
        monkeypatch.setenv("SMC_FUSED_ROWS", rows)
    lat = smc_gpu.Lattice(2, 1, L, seed=12, fused=True)
    assert lat.kernel()[0] == "ising_fused"
    ref = oracle_mod.OracleLattice(2, 1, L, 12)
    lat.sweep(BETA_C, n)
    ref.sweep(BETA_C, n)
    assert np.array_equal(nat(lat), ref.s)
    slot = torch.zeros(8, dtype=torch.int64, device=lat.device)
    lat.sweep_measure(BETA_C, n, slot)
    ref.sweep(BETA_C, n)
    o = smc_gpu.Lattice.decode_obs(slot)[0]
    r = ref.measure()
    assert (o.E_int, o.M_int) == (r.E_int, r.M_int)
    assert o.sweep == 2 * n
    assert np.array_equal(nat(lat), ref.s)
    assert lat.t == 2 * n


@pytest.mark.parametrize("d,L,variant", [(2, 64, "stream"), (2, 64, "chunk"), (2, 64, "site"),
                                         (3, 32, "stream"), (3, 32, "chunk"), (2, 10, "site"),
                                         (3, 16, "stream")])
def test_sweep_measure_matches_oracle(smc_gpu, oracle_mod, d, L, variant, monkeypatch):
    import torch
    monkeypatch.setenv("SMC_ISING_KERNEL", variant)
    lat = smc_gpu.Lattice(d, 1, L, seed=14)
    ref = oracle_mod.OracleLattice(d, 1, L, 14)
    slots = torch.zeros((3, 8), dtype=torch.int64, device=lat.device)
    for k, n in enumerate((1, 3, 0)):
        lat.sweep_measure(0.35, n, slots[k])
    got = smc_gpu.Lattice.decode_obs(slots)
    for k, n in enumerate((1, 3, 0)):
        ref.sweep(0.35, n)
        r = ref.measure()
        assert (got[k].E_int, got[k].M_int) == (r.E_int, r.M_int), (k, variant)
    assert [o.sweep for o in got] == [1, 4, 4]
