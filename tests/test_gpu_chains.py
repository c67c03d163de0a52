"""GPU parity of the real-coupling chains (derivatives of ln Z).

* The counted near-threshold protocol of FP32 couplings: from the oracle's
  state, one half-sweep at a time, every decision whose margin |u - p| is at
  least 1e-6 equals the oracle's; the others are counted and printed.  One
  whole sweep from the same state with its bond products: states differ only
  at those sites (and at colour-1 sites next to a colour-0 site that
  differs), and the bond sums equal the oracle's on every bond whose two
  ends agree.  Seed 7's case has such a decision (margin 4.6e-7).
* Chains against the oracle's chains over many sweeps on seeds with no
  decision within 1e-6 of its threshold (the oracle reports the smallest
  margin; there the chain is unique): start states, final states and the
  summed bond products bit-exact.
* Both chain kernels (the register-resident pair kernel and the LDS kernel)
  run every case.
* Chain k equals the single-lattice chain with FP32 couplings and replica k.
* The covariance replay equals the oracle's sample covariance over the same
  samples.
* At L = 4, the estimates of <x_b>, of the gradient of the correlations and
  of ln Z's gradients agree with exact enumeration within their statistical
  errors, common-random-number finite differences agree with beta Cov, and
  moment matching recovers hidden couplings.
"""
import numpy as np
import pytest

import layout

import oracle.exact as ex

pytestmark = pytest.mark.gpu


def split(a, d, L):
    return layout.to_split(np.ascontiguousarray(a), d, L)


def natural(a, d, L):
    return layout.to_natural(np.ascontiguousarray(a), d, L)


@pytest.fixture(params=["pair", "lds"])
def chains_kernel(request, monkeypatch):
    """Run the case on the pair kernel (where the lattice has at most 1024
    site pairs per colour) or force the LDS kernel."""
    if request.param == "lds":
        monkeypatch.setenv("SMC_CHAINS_KERNEL", "lds")
    else:
        monkeypatch.delenv("SMC_CHAINS_KERNEL", raising=False)
    return request.param


def make(smc_gpu, oracle_mod, d, L, nch, seed, replica0, J_nat):
    import torch
    Jt = torch.from_numpy(split(J_nat, d, L)).cuda()
    ch = smc_gpu.Chains(d, L, nch, seed, J=Jt, replica0=replica0)
    s0 = np.stack([oracle_mod.init_ising(d, L, seed, replica=replica0 + k) for k in range(nch)])
    return ch, s0


def expected_kernel(kernel, d, L):
    return "chains_pair" if kernel == "pair" and L ** d // 4 <= 1024 else "chains_lds"


def upload(ch, states, d, L):
    import torch
    ch.spins.copy_(torch.from_numpy(split(states, d, L)).view_as(ch.spins))


REPLAY = [  # d, L, chains, sweeps, beta, seed, sigma of J ~ N(1, sigma^2)
    (2, 4, 9, 50, 0.5, 7, 0.2),   # chain 4, sweep 40, colour 0, site 2: margin 4.6e-7
    (2, 4, 9, 50, 0.5, 8, 0.2),
    (2, 8, 6, 20, 0.45, 3, 0.2),
    (3, 4, 5, 15, 0.25, 4, 0.2),
    (2, 64, 2, 6, 0.4, 5, 0.2),
    (3, 6, 3, 10, 0.3, 6, 0.2),
    (2, 84, 2, 3, 0.4, 9, 0.2),   # 1764 pairs: the LDS kernel either way
    (2, 64, 256, 3, 0.4, 21, 0.1),  # the derivative workload's shape and launch: 256 chains
]


@pytest.mark.parametrize("d,L,nch,nsw,beta,seed,sigma", REPLAY)
def test_chains_half_sweeps_match_oracle(smc_gpu, oracle_mod, chains_kernel, d, L, nch, nsw,
                                          beta, seed, sigma):
    """Eq. (2) with FP32 couplings, the counted protocol (see the module
    docstring), sweep by sweep from the oracle's own states."""
    print(f"chains replay d={d} L={L} chains={nch} sweeps={nsw} seed={seed} {chains_kernel}",
          flush=True)
    rng = np.random.default_rng(seed)
    J = rng.normal(1.0, sigma, size=(d, L ** d)).astype(np.float32)
    ch, s0 = make(smc_gpu, oracle_mod, d, L, nch, seed, 100, J)
    assert ch.kernel() == expected_kernel(chains_kernel, d, L)
    refs = [oracle_mod.OracleLattice(d, 1, L, seed, J_kind=oracle_mod.J_FP32, J=J, replica=100 + k,
                                     spins=s0[k]) for k in range(nch)]
    nbr = layout.natural_neighbours(d, L)
    col = layout.natural_colours(d, L)
    near, excluded = 0, 0
    for t in range(nsw):
        start = np.stack([r.s.copy() for r in refs])
        near_mask = np.zeros((nch, L ** d), dtype=bool)
        for c in (0, 1):
            upload(ch, np.stack([r.s for r in refs]), d, L)
            ch.t = t
            ch.half_sweep(beta, c)
            got = np.stack([natural(ch.spins[k].cpu().numpy(), d, L) for k in range(nch)])
            for k, r in enumerate(refs):
                _, margin = r.half_sweep(beta, c, t, want_margin=True)
                close = np.abs(margin) < 1e-6
                diff = np.nonzero(got[k] != r.s)[0]
                assert np.all(close[diff]), (t, c, k, diff, margin[diff])
                near_mask[k] |= close
        near += int(near_mask.sum())
        # the whole sweep with its bond products, from the same start
        upload(ch, start, d, L)
        ch.t = t
        acc = ch.bond_zeros()
        ch.sample(beta, 1, acc)
        assert ch.t == t + 1
        got = np.stack([natural(ch.spins[k].cpu().numpy(), d, L) for k in range(nch)])
        want = np.stack([r.s for r in refs])
        mism = got != want
        knock = (col == 1)[None, :] & (mism & (col == 0)[None, :])[:, nbr].any(axis=2)
        assert not np.any(mism & ~(near_mask | knock)), (t, np.nonzero(mism & ~(near_mask | knock)))
        want_b = np.zeros((d, L ** d), dtype=np.int64)
        for r in refs:
            r.bond_accumulate(want_b)
        ok_site = ~mism.any(axis=0)
        agree = np.stack([ok_site & ok_site[nbr[:, 2 * mu]] for mu in range(d)])
        excluded += int((~agree).sum())
        assert np.array_equal(natural(acc.cpu().numpy(), d, L)[agree], want_b[agree]), t
    print(f"near-threshold decisions (|u - p| < 1e-6): {near}; bonds left out of the sum check: "
          f"{excluded}", flush=True)
    if seed == 7:
        assert near >= 1


CASES = [  # d, L, chains, sweeps, beta, seed (no decision within 1e-6 of its threshold)
    (2, 8, 6, 40, 0.45, 3),
    (3, 4, 5, 30, 0.25, 4),
    (2, 64, 2, 10, 0.4, 5),
    (3, 6, 3, 20, 0.3, 6),
    (2, 4, 9, 50, 0.5, 8),
]


@pytest.mark.parametrize("d,L,nch,nsw,beta,seed", CASES)
def test_chains_match_oracle(smc_gpu, oracle_mod, chains_kernel, d, L, nch, nsw, beta, seed):
    print(f"chains d={d} L={L} chains={nch} sweeps={nsw} {chains_kernel}", flush=True)
    rng = np.random.default_rng(seed)
    J = rng.normal(1.0, 0.2, size=(d, L ** d)).astype(np.float32)
    ch, s0 = make(smc_gpu, oracle_mod, d, L, nch, seed, 100, J)
    assert ch.kernel() == expected_kernel(chains_kernel, d, L)
    got0 = np.stack([natural(ch.spins[k].cpu().numpy(), d, L) for k in range(nch)])
    assert np.array_equal(got0, s0)
    # burn-in without accumulation, then accumulate
    ch.sample(beta, 3)
    st, _, _, m1 = oracle_mod.chains_ising(d, L, seed, J, beta, s0, 3, replica0=100)
    acc = ch.bond_zeros()
    ch.sample(beta, nsw, acc)
    out, bsum, _, m2 = oracle_mod.chains_ising(d, L, seed, J, beta, st, nsw, t0=3, replica0=100)
    # the precondition of a unique chain (a case with a near-threshold
    # decision belongs in the replay test above)
    assert min(m1, m2) > 1e-6, "a decision came within 1e-6 of its threshold"
    got = np.stack([natural(ch.spins[k].cpu().numpy(), d, L) for k in range(nch)])
    assert np.array_equal(got, out)
    assert np.array_equal(natural(acc.cpu().numpy(), d, L), bsum)
    assert ch.t == 3 + nsw


def test_chain_equals_single_lattice_chain(smc_gpu, oracle_mod, chains_kernel):
    import torch
    d, L, nch, seed, beta = 2, 16, 4, 9, 0.42
    rng = np.random.default_rng(1)
    J = rng.normal(1.0, 0.1, size=(d, L ** d)).astype(np.float32)
    ch, _ = make(smc_gpu, oracle_mod, d, L, nch, seed, 7, J)
    assert ch.kernel() == expected_kernel(chains_kernel, d, L)
    ch.sample(beta, 25)
    Jt = torch.from_numpy(split(J, d, L)).cuda()
    for k in range(nch):
        lat = smc_gpu.Lattice(d, 1, L, seed=seed, J_kind=smc_gpu.J_FP32, J=Jt, replica=7 + k)
        lat.sweep(beta, 25)
        assert torch.equal(lat.spins.view(-1).cpu(), ch.spins[k].view(-1).cpu()), k


# the last two: couplings too large to share LDS with the covariance
# accumulators, so the covariance pass reads them from global memory
@pytest.mark.parametrize("d,L,nch,nsw,beta,seed", [(2, 8, 6, 40, 0.45, 3), (3, 4, 5, 30, 0.25, 4),
                                                   (2, 64, 3, 6, 0.4, 12),
                                                   (2, 84, 2, 4, 0.4, 9), (3, 18, 2, 3, 0.25, 11)])
def test_covariance_replay_matches_oracle(smc_gpu, oracle_mod, chains_kernel, d, L, nch, nsw, beta,
                                          seed):
    import torch
    rng = np.random.default_rng(seed + 50)
    J = rng.normal(1.0, 0.2, size=(d, L ** d)).astype(np.float32)
    ch, s0 = make(smc_gpu, oracle_mod, d, L, nch, seed, 0, J)
    start = ch.spins.clone()
    acc = ch.bond_zeros()
    ch.sample(beta, nsw, acc)
    _, bsum, samples, mm = oracle_mod.chains_ising(d, L, seed, J, beta, s0, nsw,
                                                   want_samples=True)
    assert mm > 1e-6
    assert np.array_equal(natural(acc.cpu().numpy(), d, L), bsum)
    g_nat = rng.normal(size=(d, L ** d))
    S = nch * nsw
    mean_nat = bsum / S
    # the library's mean and centre
    mean = ch.mean(acc, S)
    assert np.array_equal(natural(mean.cpu().numpy(), d, L), mean_nat)
    g = torch.from_numpy(split(g_nat, d, L)).cuda()
    center = ch.dot(g, mean)
    gc = float((g_nat * mean_nat).sum())
    assert abs(float(center) - gc) <= 1e-12 * max(1.0, np.abs(g_nat * mean_nat).sum())
    end = ch.spins.clone()
    ch.spins.copy_(start)
    ch.t = 0
    cov_acc = ch.bond_zeros(torch.float64)
    G_acc = torch.zeros(2, dtype=torch.float64, device=ch.device)
    ch.covariance(beta, nsw, g, center, cov_acc, G_acc)
    assert torch.equal(ch.spins, end)
    gc = float(center)
    cov = natural((cov_acc / S).cpu().numpy(), d, L) - (float(G_acc[0]) / S) * mean_nat
    want = oracle_mod.bond_covariance(samples, g_nat)
    tol = 1e-11 * max(1.0, np.abs(want).max())
    assert np.abs(cov - want).max() <= tol
    # G moments: sum (G - c) and sum (G - c)^2 over the samples
    X = samples.reshape(S, -1).astype(np.float64)
    Gs = X @ g_nat.reshape(-1) - gc
    assert abs(float(G_acc[0]) - Gs.sum()) < 1e-9 * max(1.0, np.abs(Gs).sum())
    assert abs(float(G_acc[1]) - (Gs ** 2).sum()) < 1e-9 * (Gs ** 2).sum()
    # the library's vector-Jacobian product: beta Cov(G, x_b) (float32) and
    # sum_b J_b Cov(G, x_b)
    Jt = torch.from_numpy(split(J, d, L)).cuda()
    gJ, gb = ch.vjp(beta, S, cov_acc, G_acc, mean, Jt)
    gJn = natural(gJ.cpu().numpy().astype(np.float64), d, L)
    assert np.all(np.abs(gJn - beta * want) <= 2e-7 * np.abs(beta * want) + beta * tol + 1e-30)
    wb = float((J.astype(np.float64) * want).sum())
    assert abs(float(gb) - wb) <= 1e-10 * max(1.0, np.abs(J * want).sum())


@pytest.fixture(scope="module")
def x4():
    return ex.torus_bond_products(4)


def test_autograd_against_exact_enumeration(smc_gpu, x4):
    import torch
    from paper_1107_5463_amd import autodiff
    rng = np.random.default_rng(21)
    d, L, beta = 2, 4, 0.4
    J_nat = rng.normal(1.0, 0.2, size=(d, 16))
    mean, cov, _ = ex.exact_bond_moments(L, J_nat, beta, x4)
    nch, nsw = 256, 2000
    ch = smc_gpu.Chains(d, L, nch, 31)
    J = torch.from_numpy(split(J_nat.astype(np.float32), d, L)).cuda().requires_grad_(True)
    b = torch.tensor(beta, dtype=torch.float64, requires_grad=True)
    m = autodiff.bond_correlations(J, b, ch, nsw, n_burn=200)
    S = nch * nsw
    tau = 10.0  # generous integrated autocorrelation time (sweeps)
    var = np.diag(cov).reshape(d, 16)
    got = natural(m.detach().cpu().numpy().astype(np.float64), d, L)
    tol = 6 * np.sqrt(var * tau / S) + 1e-6
    assert np.all(np.abs(got - mean) < tol), np.max(np.abs(got - mean) / tol)
    g_nat = rng.normal(size=(d, 16))
    m.backward(torch.from_numpy(split(g_nat.astype(np.float32), d, L)).cuda())
    want = beta * (cov @ g_nat.reshape(-1)).reshape(d, 16)
    EG2 = g_nat.reshape(-1) @ (cov + np.outer(mean.reshape(-1), mean.reshape(-1))) @ g_nat.reshape(-1)
    gtol = 6 * beta * np.sqrt(EG2 * tau / S) + 1e-6
    gotJ = natural(J.grad.cpu().numpy().astype(np.float64), d, L)
    assert np.all(np.abs(gotJ - want) < gtol), np.max(np.abs(gotJ - want) / gtol)
    want_b = float((cov @ g_nat.reshape(-1)) @ J_nat.reshape(-1))
    Jv = J_nat.reshape(-1)
    EH2 = Jv @ (cov + np.outer(mean.reshape(-1), mean.reshape(-1))) @ Jv
    assert abs(float(b.grad) - want_b) < 6 * np.sqrt(EG2 * EH2 * tau / S)


def test_log_partition_gradients(smc_gpu, x4):
    import torch
    from paper_1107_5463_amd import autodiff
    rng = np.random.default_rng(4)
    J_nat = rng.normal(1.0, 0.1, size=(2, 16))
    beta = 0.35
    mean, _, _ = ex.exact_bond_moments(4, J_nat, beta, x4)
    J = torch.from_numpy(split(J_nat.astype(np.float32), 2, 4)).cuda().requires_grad_(True)
    b = torch.tensor(beta, dtype=torch.float64, requires_grad=True)
    ch = smc_gpu.Chains(2, 4, 128, 5)
    z = autodiff.log_partition(J, b, ch, 2000, n_burn=100)
    assert float(z) == 0.0
    z.backward()
    ch2 = smc_gpu.Chains(2, 4, 128, 5)
    gJ, gb = autodiff.log_partition_grad(J.detach(), beta, ch2, 2000, n_burn=100)
    assert torch.allclose(J.grad.double(), gJ.float().double(), rtol=0, atol=1e-6)
    assert abs(float(b.grad) - gb) < 1e-6 * max(1.0, abs(gb))
    got = natural(gJ.cpu().numpy(), 2, 4) / beta
    assert np.abs(got - mean).max() < 0.02


def test_moment_matching_recovers_hidden_couplings(smc_gpu, x4):
    import torch
    from paper_1107_5463_amd import autodiff
    rng = np.random.default_rng(7)
    J_star = rng.normal(1.0, 0.1, size=(2, 16))
    beta = 0.4
    target_nat, _, _ = ex.exact_bond_moments(4, J_star, beta, x4)
    target = torch.from_numpy(split(target_nat, 2, 4)).cuda()
    ch = smc_gpu.Chains(2, 4, 256, 13)
    hist = []
    autodiff.fit_couplings(target, beta, ch, steps=60, lr=2.5, n_sweeps=500, n_burn=20,
                           J_init=torch.ones((2, 2, 8), device="cuda"), history=hist)
    J_fit = torch.stack(hist[-15:]).mean(0)
    err = np.abs(natural(J_fit.cpu().numpy().astype(np.float64), 2, 4) - J_star)
    assert err.max() < 0.05, err.max()


def test_moment_matching_recovers_hidden_couplings_at_l64(smc_gpu):
    """The derivative workload: 2D L = 64, 256 chains, beta = 0.4, hidden
    couplings J* ~ N(1, 0.1^2) from a numpy seed.  The targets are bond
    correlations the library samples under J* (10^4 sweeps of the 256 chains
    after 500 sweeps of burn-in); the fit starts from J = 1 and ascends the
    log-likelihood by moment matching (Eq. (1): its gradient in J is
    beta (target - <x>_J)).  Two fits to two independently sampled targets:
    their difference measures the spread the sampling noise puts on one fit,
    and each fit's error against J* must stay within 3 times that spread (rms
    over the 8192 bonds) -- no bias beyond the sampling error -- and far
    below the spread of J* itself."""
    import torch
    from paper_1107_5463_amd import autodiff
    d, L, nch, beta = 2, 64, 256, 0.4
    rng = np.random.default_rng(2024)
    J_star_nat = rng.normal(1.0, 0.1, size=(d, L * L)).astype(np.float32)
    J_star = torch.from_numpy(split(J_star_nat, d, L)).cuda()

    def sampled_target(seed):
        ch = smc_gpu.Chains(d, L, nch, seed, J=J_star)
        ch.sample(beta, 500)
        acc = ch.bond_zeros()
        ch.sample(beta, 10000, acc)
        return ch.mean(acc, nch * 10000)

    errs = []
    for seed in (901, 902):
        print(f"C5 fit: targets from seed {seed}", flush=True)
        tgt = sampled_target(seed)
        ch = smc_gpu.Chains(d, L, nch, seed + 100)
        hist = []
        autodiff.fit_couplings(tgt, beta, ch, steps=50, lr=2.0, n_sweeps=1000, n_burn=100,
                               J_init=torch.ones((d, 2, L * L // 2), device="cuda"), history=hist)
        J_fit = torch.stack(hist[-10:]).double().mean(0)
        errs.append(natural(J_fit.cpu().numpy(), d, L) - J_star_nat.astype(np.float64))
    rms = [float(np.sqrt((e ** 2).mean())) for e in errs]
    spread = float(np.sqrt(((errs[0] - errs[1]) ** 2).mean() / 2))
    print(f"C5 fit: rms error {rms}, sampling spread {spread:.4g}", flush=True)
    for r in rms:
        assert r <= 3 * spread, (rms, spread)
        assert r < 0.025, rms


def test_common_random_number_finite_differences(smc_gpu, x4):
    """Central finite differences of the sampled bond correlations under
    common random numbers (the same seed, hence the same start states and
    random streams, at J + eps e_b and J - eps e_b) equal the derivative
    d<x_a>/dJ_b = beta Cov(x_a, x_b) -- that of exact enumeration and the
    backward pass's covariance estimate -- at L = 4 within their errors."""
    import torch
    from paper_1107_5463_amd import autodiff
    rng = np.random.default_rng(9)
    d, L, beta, eps = 2, 4, 0.4, 0.25  # curvature error of the central difference ~3e-4
    J_nat = rng.normal(1.0, 0.1, size=(d, 16))
    bond = (0, 5)  # J_b: the +x bond of site 5
    nch, nsw, burn = 256, 3000, 100
    bt = torch.tensor(beta, dtype=torch.float64)

    def means(Jn, seed):
        ch = smc_gpu.Chains(d, L, nch, seed)
        J = torch.from_numpy(split(Jn.astype(np.float32), d, L)).cuda()
        m = autodiff.bond_correlations(J, bt, ch, nsw, n_burn=burn)
        return natural(m.detach().cpu().numpy().astype(np.float64), d, L)

    Jp, Jm = J_nat.copy(), J_nat.copy()
    Jp[bond] += eps
    Jm[bond] -= eps
    fds = np.array([(means(Jp, s) - means(Jm, s)) / (2 * eps) for s in (41, 42, 43, 44)])
    fd, se = fds.mean(0), fds.std(0, ddof=1) / 2
    # exact: the central difference and the derivative differ by O(eps^2)
    _, cov, _ = ex.exact_bond_moments(L, J_nat, beta, x4)
    want = beta * cov[:, bond[0] * 16 + bond[1]].reshape(d, 16)
    fd_exact = (ex.exact_bond_moments(L, Jp, beta, x4)[0] -
                ex.exact_bond_moments(L, Jm, beta, x4)[0]) / (2 * eps)
    assert np.abs(fd_exact - want).max() < 2e-3
    assert np.all(np.abs(fd - fd_exact) < 6 * se + 5e-3), np.max(np.abs(fd - fd_exact) - 6 * se)
    # the backward pass at J: J.grad for the cotangent e_b is column b of beta Cov
    J = torch.from_numpy(split(J_nat.astype(np.float32), d, L)).cuda().requires_grad_(True)
    m = autodiff.bond_correlations(J, bt, smc_gpu.Chains(d, L, 4 * nch, 45), nsw, n_burn=burn)
    g = np.zeros((d, 16))
    g[bond] = 1.0
    m.backward(torch.from_numpy(split(g.astype(np.float32), d, L)).cuda())
    bw = natural(J.grad.cpu().numpy().astype(np.float64), d, L)
    assert np.abs(bw - want).max() < 0.02, np.abs(bw - want).max()
    assert np.all(np.abs(fd - bw) < 6 * se + 0.02)


def test_pair_and_lds_kernels_run_the_same_chains(smc_gpu, monkeypatch):
    """The derivative workload's shape (2D L = 64, 256 chains, J ~ N(1, 0.1^2),
    beta = 0.4), 300 sweeps with bond sums and a covariance replay: the pair
    kernel and the LDS kernel take the same decisions (same FP32 arithmetic),
    so states and bond sums are equal and the covariance sums agree to
    rounding (different reduction order)."""
    import torch
    d, L, nch, beta = 2, 64, 256, 0.4
    rng = np.random.default_rng(17)
    J = torch.from_numpy(split(rng.normal(1.0, 0.1, size=(d, L * L)).astype(np.float32), d, L)).cuda()
    g = torch.from_numpy(split(rng.normal(size=(d, L * L)), d, L)).cuda()
    out = {}
    for kern in ("pair", "lds"):
        if kern == "lds":
            monkeypatch.setenv("SMC_CHAINS_KERNEL", "lds")
        else:
            monkeypatch.delenv("SMC_CHAINS_KERNEL", raising=False)
        ch = smc_gpu.Chains(d, L, nch, 33, J=J)
        assert ch.kernel() == "chains_" + kern
        ch.sample(beta, 50)
        start = ch.spins.clone()
        acc = ch.bond_zeros()
        ch.sample(beta, 300, acc)
        end = ch.spins.clone()
        ch.spins.copy_(start)
        ch.t = 50
        cov = ch.bond_zeros(torch.float64)
        G = torch.zeros(2, dtype=torch.float64, device=ch.device)
        ch.covariance(beta, 300, g, torch.full((1,), 0.25, dtype=torch.float64, device=ch.device),
                      cov, G)
        assert torch.equal(ch.spins, end)
        out[kern] = (end.cpu(), acc.cpu(), cov.cpu(), G.cpu())
    assert torch.equal(out["pair"][0], out["lds"][0])
    assert torch.equal(out["pair"][1], out["lds"][1])
    for a, b in ((out["pair"][2], out["lds"][2]), (out["pair"][3], out["lds"][3])):
        assert float((a - b).abs().max()) <= 1e-11 * float(b.abs().max())
