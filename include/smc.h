/*
 * smc.h -- C ABI of libsmc: checkerboard single-spin-flip Metropolis sweeps of
 * nearest-neighbour O(n) spin models on one MI355X (gfx950) GPU.
 *
 * Model (Weigel & Yavors'kii, "GPU accelerated Monte Carlo simulations of
 * lattice spin models", Sec. 2, Eq. (1)): H = -sum_<ij> J_ij s_i . s_j with
 * n = 1 (Ising, s = +-1), n = 2 (XY) or n = 3 (Heisenberg) unit-vector spins
 * on a periodic square (d = 2) or simple-cubic (d = 3) lattice of edge L.
 * Update (Eq. (2)): single-spin Metropolis moves accepted with probability
 * min[1, exp(-beta dE)], all sites of one checkerboard colour at once, then
 * the other colour (Sec. 2, checkerboard decomposition).  One sweep = colour
 * 0 then colour 1 = N attempts.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * Sites.  i = x + L*y + L*L*z, colour c = (x + y + z) mod 2, and the index of
 *   site i within its colour is j = i >> 1 (L even), 0 <= j < N/2.
 * Device buffers (all caller-owned, all on the device of `stream`; the
 *   library never allocates, frees or reallocates device memory -- its one
 *   device array of its own is smc_measure_noalloc's static scratch):
 *   spins  Ising: int8 [2][N/2], plane c holds the spins +1/-1 of colour c.
 *          XY / Heisenberg: float [n][2][N/2], component k of site (c, j) at
 *          k*N + c*N/2 + j.  Aligned to 16 bytes.
 *   J      SMC_J_UNIFORM: NULL (every bond has J0).
 *          SMC_J_PM: int8 [d][2][N/2], J[mu][c][j] = +-1 scales J0 on the bond
 *          from site (c, j) to its +mu neighbour.
 *          SMC_J_FP32: float [d][2][N/2], the coupling of that bond.
 *   workspace  at least smc_workspace_bytes(p) bytes, 256-byte aligned:
 *          reduction partials, an observable slot and, for the fused schedule,
 *          the second spin buffer.
 * Random numbers.  Philox4x32-10 (Salmon et al., SC'11), key = seed, counter
 *   = (block, sweep t, replica, colour | purpose << 1); the same (seed,
 *   replica) gives the same chain whatever the launch geometry or schedule.
 * Streams.  Every call enqueues its work on the handle's stream and returns
 *   without synchronising, except smc_measure, smc_validate and
 *   smc_get_samples-free reads noted below.
 * Errors.  0 = SMC_OK, negative codes otherwise; no exception or abort
 *   crosses the ABI; smc_last_error() gives the calling thread's last message.
 *   Calls are re-entrant per handle but a handle must not be used from two
 *   threads at once.
 */
#ifndef SMC_H
#define SMC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum smc_status {
  SMC_OK = 0,
  SMC_EINVAL = -1,  /* bad d/n/L/beta/delta, NULL or misaligned pointer, small workspace */
  SMC_ERANGE = -2,  /* sweep counter would pass 2^32 - 1 */
  SMC_EDEVICE = -3, /* a HIP call failed (its message is in smc_last_error) */
  SMC_ESTATE = -4   /* smc_validate found a spin or coupling out of range */
};

enum smc_J_kind { SMC_J_UNIFORM = 0, SMC_J_PM = 1, SMC_J_FP32 = 2 };
enum smc_init_kind { SMC_INIT_HOT = 0, SMC_INIT_COLD = 1, SMC_INIT_KEEP = 2 };

enum smc_flags {
  SMC_FLAG_FAST_MATH = 1,        /* hardware transcendentals for continuous spins */
  SMC_FLAG_SCHEDULE_FUSED = 2,   /* 2D Ising, uniform J, L % 2048 == 0, L <= 16384: one kernel per sweep,
                                    ping-ponging through the workspace (bit-identical
                                    results; other shapes keep the two-pass schedule) */
  SMC_FLAG_GENERIC_KERNEL = 4,   /* force the one-site-per-thread kernels (testing) */
  SMC_FLAG_COUPLINGS_KEEP = 8,   /* do not generate J at init; use the caller's values */
  SMC_FLAG_HEATBATH = 32,        /* Ising, uniform or +-1 J: heat-bath rule (Sec. 2): new spin
                                    +1 iff u32 < ceil(2^32 / (1 + exp(-2 beta h))) with the
                                    Metropolis draws; plain sweeps run the one-site kernel */
  SMC_FLAG_PACKED = 16           /* Ising spins (and +-1 couplings) at one bit per site
                                    (Sec. 2, multi-spin coding): the int8 planes' site
                                    order, site j in bit j & 31 of 32-bit word j >> 5,
                                    bit 1 = -1; L % 64 == 0; same chain as int8; no
                                    bond correlations; the fused schedule is ignored */
};

enum smc_bond_op { SMC_BOND_RESET = 0, SMC_BOND_ACCUMULATE = 1, SMC_BOND_READ = 2 };

typedef struct smc_params {
  int32_t d;            /* 2 or 3 */
  int32_t n;            /* 1 Ising, 2 XY, 3 Heisenberg */
  int32_t L;            /* even, >= 4 */
  int32_t J_kind;       /* enum smc_J_kind */
  uint64_t seed;        /* Philox key */
  uint32_t replica;     /* third counter word: chain / disorder-sample id */
  int32_t init;         /* enum smc_init_kind */
  double J0;            /* uniform coupling, or the scale of +-1 couplings, or the
                           mean of Gaussian couplings */
  double J_sigma;       /* standard deviation of Gaussian couplings */
  double delta;         /* XY: max rotation angle (rad); Heisenberg: cap half-angle */
  int32_t renorm_every; /* continuous spins: renormalise after sweeps with t % R == 0
                           (0 = never) */
  int32_t flags;        /* enum smc_flags */
  int32_t tile;         /* 0: plain sweeps; T > 0: the tiled k-hit schedule of Sec. 2
                           (Ising, uniform J; T = 16 or T % 32 == 0, L / T even;
                           2D T <= 256, 3D T = 16 or 32): tiles of edge T coloured by (tx+ty+tz) mod 2,
                           a sweep = for tile colour 0 then 1: `hits` times colour-0
                           sites then colour-1 sites of those tiles; hit h uses
                           counter word 3 = colour | purpose << 1 | h << 8 */
  int32_t hits;         /* k >= 1 for the tiled schedule (0 or 1 otherwise) */
} smc_params;

typedef struct smc_obs {
  int64_t E_int;  /* Ising, uniform or +-1 couplings: -sum_<ij> sign(J_ij) s_i s_j */
  int64_t M_int;  /* Ising: sum_i s_i */
  double E;       /* energy (E_int * J0 for integer couplings) */
  double M[3];    /* magnetisation vector */
  double absM;    /* |M| */
  int64_t sweep;  /* sweep counter t of the measured state (sweeps done since t = 0) */
} smc_obs;

typedef struct smc_lattice smc_lattice;

/* Bytes of the caller-owned buffers for parameters p (0 if p is invalid). */
size_t smc_spin_bytes(const smc_params* p);
size_t smc_coupling_bytes(const smc_params* p);
size_t smc_workspace_bytes(const smc_params* p);
/* Bytes of the bond-correlation accumulator: d*N int64 (Ising) or double. */
size_t smc_bond_bytes(const smc_params* p);

/*
 * Create a handle bound to caller-owned device buffers and a stream
 * (hipStream_t passed as void*; NULL = the null stream).  With init HOT or COLD
 * the library fills `spins` (hot start from the Philox init draws, cold = all
 * along +x / +1); with KEEP it leaves them.  For SMC_J_PM / SMC_J_FP32 the
 * couplings are generated from the seed unless SMC_FLAG_COUPLINGS_KEEP.
 * The sweep counter starts at 0.  The handle is host memory owned by the
 * library until smc_destroy.  Enqueues work; does not synchronise.
 */
int smc_init_lattice(smc_lattice** out, const smc_params* p, void* spins, void* J,
                     void* workspace, size_t workspace_bytes, void* stream);

/* Rebind the stream used by later calls (hipStream_t as void*). */
int smc_set_stream(smc_lattice* h, void* stream);

/*
 * n_sweeps sweeps (Sec. 2: colour 0 then colour 1, Eq. (2) acceptance) at
 * inverse temperature beta (finite and >= 0, or +infinity for a quench).
 * Sweep k uses counter t + k; afterwards t += n_sweeps.  Continuous spins are
 * renormalised after each sweep whose new t is a multiple of renorm_every.
 * Fails with SMC_ERANGE if t + n_sweeps > 2^32.  Asynchronous.
 */
int smc_sweep(smc_lattice* h, double beta, int64_t n_sweeps);

/*
 * smc_sweep followed by the observables of the final state, written as an
 * smc_obs to device memory dev_obs (8-byte aligned), without synchronising.
 * The reduction is fused into the last sweep's kernel where the kernel
 * supports it (no extra pass over the lattice); otherwise a separate
 * measurement runs.  n_sweeps = 0 measures the current state.
 */
int smc_sweep_measure(smc_lattice* h, double beta, int64_t n_sweeps, void* dev_obs);

/* One colour only, with counter t (t is not advanced).  Test hook used by the
 * single-spin and half-sweep parity protocols.  Asynchronous. */
int smc_half_sweep(smc_lattice* h, double beta, int colour);

/* Energy and magnetisation (Eq. (1)) of the current state, summed in int64
 * (Ising with integer couplings) or double.  Synchronises the stream. */
int smc_measure(smc_lattice* h, smc_obs* out);

/* Same, written as an smc_obs to device memory dev_obs (8-byte aligned)
 * without synchronising. */
int smc_measure_async(smc_lattice* h, void* dev_obs);

/*
 * For callers that cannot allocate device memory (code under stream capture,
 * tight serving loops, harnesses that forbid hipMalloc): smc_measure_async's
 * energy and magnetisation, with the same kernels, of a state given directly
 * -- no handle and no workspace.  p, spins and J as for smc_init_lattice
 * (p->init, seed, replica, delta, renorm_every, tile and hits are not used;
 * SMC_FLAG_PACKED selects the packed layout); the smc_obs record goes to
 * dev_obs (device, 8-byte aligned) with its `sweep` field set to `sweep`;
 * asynchronous on `stream` (hipStream_t as void*, on the current device).
 * The block partials of the reduction live in a static device array owned by
 * the library, one per GPU for the life of the process: 16384 partials
 * (768 KiB), enough for every int8 and continuous lattice and for packed
 * lattices with N/2 <= 2^27 (2D L <= 16384, 3D L <= 512); larger packed
 * lattices fail with SMC_EINVAL.  Calls no hipMalloc, hipFree or allocating
 * routine.  Every call on a GPU uses that GPU's one array: calls that overlap
 * on one GPU (two streams, two threads) race and must be ordered by the
 * caller.
 */
int smc_measure_noalloc(const smc_params* p, const void* spins, const void* J, int64_t sweep,
                        void* dev_obs, void* stream);

/*
 * Bond correlations s_i . s_{i+mu} for every bond (the per-bond statistic
 * behind d ln Z / d J_ij = beta <s_i . s_j>).  acc: caller-owned device buffer
 * of smc_bond_bytes(p) bytes, laid out [d][2][N/2] like J (int64 for Ising,
 * double otherwise).
 *   SMC_BOND_RESET       zero acc and the handle's sample count;
 *   SMC_BOND_ACCUMULATE  acc += s_i . s_{i+mu} for the current state, count += 1;
 *   SMC_BOND_READ        out_mean (device, double [d][2][N/2]) = acc / count.
 * Asynchronous.
 */
int smc_bond_correlations(smc_lattice* h, int op, void* acc, void* out_mean);
int smc_get_samples(const smc_lattice* h, int64_t* samples);

/* Continuous spins: s <- s / |s| now (asynchronous). */
int smc_renormalize(smc_lattice* h);

/* Check the state: Ising spins in {+1, -1}; continuous | |s| - 1 | < 1e-4 and
 * finite; couplings finite (and +-1 for SMC_J_PM).  Synchronises.  Returns
 * SMC_ESTATE if anything is out of range. */
int smc_validate(smc_lattice* h);

/* Checkpoint / resume: the whole state is (params, t, spins, J, accumulators,
 * sample count); the random numbers are stateless. */
int smc_get_sweep_index(const smc_lattice* h, uint64_t* t);
int smc_set_sweep_index(smc_lattice* h, uint64_t t);
int smc_set_samples(smc_lattice* h, int64_t samples);

/*
 * Pick the band height of the handle's banded kernel (int8 or packed Ising
 * streaming kernels, the continuous streaming kernel, the fused schedule):
 * every height the kernel takes (powers of two dividing L) is timed over a
 * few sweeps at inverse temperature beta on the handle's own spin buffer
 * (where placement in memory decides much of the speed), whose state is kept
 * in `scratch` -- a caller-owned device buffer of at least smc_spin_bytes(p)
 * bytes, 16-byte aligned -- and copied back, so the state and the sweep
 * counter are left as they were; the fastest height is kept.  Every height gives the same chain.  With
 * SMC_AUTOTUNE_CACHE naming a file, a choice stored there for the same
 * kernel, shape and device is taken without timing (scratch may then be
 * NULL), and new choices are added to it.  rows_out (optional) receives the
 * chosen height, 0 if the handle's kernel has no bands.  Synchronises.
 */
int smc_autotune(smc_lattice* h, double beta, void* scratch, size_t scratch_bytes,
                 uint32_t* rows_out);

/* Name of the kernel the handle's sweeps launch -- Ising: "ising_packed"
 * (one bit per site), "ising_fused", "ising_stream", "ising_chunk",
 * "ising_site", and for the tiled schedule "ising_tiles" (int8 tiles) or
 * "ising_tiles_packed" (tiles at one bit per site in LDS, Metropolis or heat
 * bath: 2D tile edge 16, 64 or 128, 3D tile edge 16); XY / Heisenberg:
 * "xy_stream", "xy_site",
 * "heisenberg_stream", "heisenberg_site" -- and in rows_per_band (optional)
 * the rows each lane walks for the banded kernels (packed, fused, stream,
 * xy_stream, heisenberg_stream), the tile edge for the tiled schedule, 0
 * otherwise. */
const char* smc_kernel_name(const smc_lattice* h, uint32_t* rows_per_band);

/* Free the handle (never the caller's buffers). */
int smc_destroy(smc_lattice* h);

/* ------------------------------------------------------------------------ */
/* Batches: many independent Ising lattices of uneven edge, temperature and */
/* disorder realisation swept together by one persistent launch (Sec. 2:   */
/* parallelisation over disorder realisations on top of the checkerboard   */
/* decomposition).  Lattice r (0 <= r < n_lattices) has edge L[r] (even,    */
/* 4..40 in 3D, 4..256 in 2D: L[r]^d <= 64 KiB), inverse temperature        */
/* beta[r] and replica replica[r] (r if NULL), and follows exactly the       */
/* single-lattice chain of smc_init_lattice with those parameters.          */
/* Buffers (caller-owned, device):                                          */
/*   spins  int8, lattice r's [2][N_r/2] planes at byte offset S_r;         */
/*   J      NULL (uniform J0) or int8 +-1, lattice r's [d][2][N_r/2] at C_r;  */
/*   offsets from smc_batch_offsets (each lattice starts 16-byte aligned).   */
/* ------------------------------------------------------------------------ */
typedef struct smc_batch smc_batch;

size_t smc_batch_spin_bytes(int32_t d, int32_t n_lattices, const int32_t* L);
size_t smc_batch_coupling_bytes(int32_t d, int32_t n_lattices, const int32_t* L);
/* Descriptor table, schedule and an autotuning copy of the spins. */
size_t smc_batch_workspace_bytes(int32_t d, int32_t n_lattices, const int32_t* L);
int smc_batch_offsets(int32_t d, int32_t n_lattices, const int32_t* L, int64_t* spin_offsets,
                      int64_t* coupling_offsets);

/* J_kind: SMC_J_UNIFORM or SMC_J_PM; init HOT / COLD / KEEP; with PM the
 * couplings are generated from (seed, replica[r]) unless couplings_keep. */
int smc_batch_init(smc_batch** out, int32_t d, int32_t J_kind, uint64_t seed, double J0,
                   int32_t init, int32_t couplings_keep, int32_t n_lattices, const int32_t* L,
                   const double* beta, const uint32_t* replica, void* spins, void* J,
                   void* workspace, size_t workspace_bytes, void* stream);

/* n_sweeps sweeps of every lattice in one launch (asynchronous).  With
 * dev_obs (n_lattices smc_obs, 8-byte aligned) the energy and magnetisation
 * of each lattice's final state are written there by the same launch. */
int smc_batch_sweep(smc_batch* b, int64_t n_sweeps, void* dev_obs);

/* As smc_batch_sweep, with E and M of every lattice recorded inside the same
 * launch after every measure_every sweeps (measure_every >= 1 dividing
 * n_sweeps): dev_obs holds (n_sweeps / measure_every) x n_lattices smc_obs,
 * record m * n_lattices + r = lattice r after sweep (m + 1) * measure_every
 * of the call (its `sweep` field holds the absolute sweep index).  The
 * series of Sec. 2's measurements without leaving the persistent launch.
 * EINVAL on a bad measure_every or a misaligned dev_obs. */
int smc_batch_sweep_series(smc_batch* b, int64_t n_sweeps, int64_t measure_every, void* dev_obs);

/* Time the workgroup sizes 64..1024, the lattice orders (largest first, as
 * given) and the paths (one bit per site where a lattice takes it, or one
 * byte per site throughout) on a scratch copy of the spins and keep the
 * fastest.  Results do not depend on the choice.  With SMC_AUTOTUNE_CACHE
 * naming a file, a choice stored there for the same batch shape and device
 * is taken without timing, and new choices are added to it.  Synchronises
 * the stream. */
int smc_batch_autotune(smc_batch* b, int32_t* threads_out, int32_t* largest_first_out);

/* The launch schedule: lanes per workgroup (one workgroup per lattice; a
 * multiple of 64 in [64, 1024], default 256) and the lattice order (largest
 * first or as given), as smc_batch_autotune sets them.  Results do not depend
 * on the schedule. */
int smc_batch_set_schedule(smc_batch* b, int32_t threads, int32_t largest_first);
int smc_batch_get_schedule(const smc_batch* b, int32_t* threads, int32_t* largest_first);

/* 1 if lattice r takes the packed path at the handle's current workgroup size
 * (3D, L % 8 == 0, L <= 40, at most two 32-site words of a colour per lane:
 * one bit per site in LDS, the bit-sliced decision of SMC_FLAG_PACKED -- Sec.
 * 2, multi-spin coding; the chain is the same), 0 if it takes the one byte
 * per site path (also for every lattice when SMC_BATCH_PACKED=0 was set at
 * init), negative on error. */
int smc_batch_lattice_packed(const smc_batch* b, int32_t r);

/* With enable != 0 later smc_batch_sweep calls replay one instantiated
 * hipGraph holding the launch (rebuilt when n_sweeps, dev_obs or the
 * sweep counter's host copy change shape). */
int smc_batch_use_graph(smc_batch* b, int32_t enable);

int smc_batch_get_sweep_index(const smc_batch* b, uint64_t* t);
int smc_batch_set_sweep_index(smc_batch* b, uint64_t t);
int smc_batch_destroy(smc_batch* b);

/* ------------------------------------------------------------------------ */
/* Chains: many independent Metropolis chains of one small Ising lattice    */
/* with shared real couplings J_b, for the derivatives of the partition     */
/* function of Eq. (1), Z = sum_s exp(beta sum_b J_b x_b), x_b = s_i s_j:    */
/*   d ln Z / d J_b  = beta <x_b>,                                          */
/*   d ln Z / d beta = sum_b J_b <x_b> = -<H>,                              */
/*   d <x_a> / d J_b = beta Cov(x_a, x_b)   (fluctuation-dissipation).      */
/* Chain k (0 <= k < n_chains) uses replica replica0 + k and follows         */
/* exactly the single-lattice chain of smc_init_lattice with FP32 couplings  */
/* (SMC_J_FP32) and that replica.  Bond b = (mu, c, j) couples site (c, j)   */
/* and its +mu neighbour; arrays over bonds have the coupling layout         */
/* [d][2][N/2].  2D: L a multiple of 4; 3D: L even; L^d (1 + 8 d) bytes must  */
/* fit one workgroup's LDS (160 KiB): 2D L <= 96, 3D L <= 18.                */
/* Buffers (caller-owned, device):                                          */
/*   J      float [d][2][N/2], read at every call (may be changed between);  */
/*   spins  int8, chain k's [2][N/2] planes at byte offset k N.              */
/* ------------------------------------------------------------------------ */
typedef struct smc_chains smc_chains;

size_t smc_chains_spin_bytes(int32_t d, int32_t L, int32_t n_chains);
size_t smc_chains_coupling_bytes(int32_t d, int32_t L);
/* Bytes of an array over bonds of int64 or double: 8 d N. */
size_t smc_chains_bond_bytes(int32_t d, int32_t L);
/* Per-chain covariance partials: 8 d N n_chains + 16 n_chains bytes. */
size_t smc_chains_workspace_bytes(int32_t d, int32_t L, int32_t n_chains);

/* init HOT / COLD / KEEP (hot starts from (seed, replica0 + k)). */
int smc_chains_init(smc_chains** out, int32_t d, int32_t L, int32_t n_chains, uint64_t seed,
                    uint32_t replica0, int32_t init, const float* J, void* spins,
                    void* workspace, size_t workspace_bytes, void* stream);

/* n_sweeps sweeps of every chain (asynchronous).  With dev_bond_sum (int64
 * [d][2][N/2], 8-byte aligned) the bond products x_b of every chain after
 * every sweep are added to it: after the call it has grown by
 * sum_{chains, sweeps} x_b.  NULL: sweeps only (burn-in). */
int smc_chains_sample(smc_chains* h, double beta, int64_t n_sweeps, int64_t* dev_bond_sum);

/* Replay of n_sweeps sampling sweeps from the current state and counter
 * (asynchronous): for every chain and sweep, with the sample's
 * G = sum_b g_b x_b - g_center, adds G x_b to dev_cov_acc[b] and G, G^2 to
 * dev_G_acc[0], dev_G_acc[1] (double, 8-byte aligned; summed over chains in
 * chain order, deterministic).  Started from the state and counter a
 * smc_chains_sample call started from, it visits the same configurations,
 * so that Cov(G, x_b) = cov_acc[b] / S - (G_acc[0] / S) <x_b> over its
 * S = n_chains n_sweeps samples, and the vector-Jacobian product of the
 * correlations is beta Cov(G, x_b).  g_center is one double in device
 * memory (NULL: 0), e.g. sum_b g_b <x_b> from smc_chains_dot; it only
 * conditions the sums. */
int smc_chains_covariance(smc_chains* h, double beta, int64_t n_sweeps, const double* dev_g,
                          const double* dev_g_center, double* dev_cov_acc, double* dev_G_acc);

/* Finishing the estimates (FP64 device arithmetic over the d N bonds, every
 * sum in a fixed order; all asynchronous on the handle's stream; arrays over
 * bonds in the coupling layout, double 8-byte and float 4-byte aligned).
 * With S = n_samples samples (chains x sweeps):
 *   smc_chains_mean      mean[b] = bond_sum[b] / S  (<x_b>; d ln Z / d J_b = beta <x_b>)
 *   smc_chains_dot       out[0] = sum_b a[b] w[b]
 *   smc_chains_vjp       the vector-jacobian product of <x> from a covariance
 *                        replay with weights g: Cov(G, x_b) = cov_acc[b] / S -
 *                        (G_acc[0] / S) mean[b]; grad_J[b] = (float)(beta Cov(G, x_b))
 *                        (d<x_a>/dJ_b = beta Cov(x_a, x_b)), grad_beta[0] =
 *                        sum_b J[b] Cov(G, x_b)  (d<x_a>/dbeta = Cov(x_a, sum_b J_b x_b))
 *   smc_chains_lnz_grad  d ln Z / d J_b = scale beta mean[b] into grad_J_f32 (float)
 *                        or grad_J_f64 (double) -- exactly one of them non-NULL --
 *                        and d ln Z / d beta = scale sum_b J[b] mean[b] into
 *                        grad_beta[0]; scale: one double in device memory (NULL: 1)
 *   smc_chains_fit_step  moment matching, ascent of the log-likelihood of data with
 *                        bond correlations target: J[b] += (float)(lr beta (target[b]
 *                        - mean[b]))
 * (Eq. (1): Z = sum_s exp(beta sum_b J_b x_b).) */
int smc_chains_mean(smc_chains* h, const int64_t* dev_bond_sum, int64_t n_samples, double* dev_mean);
int smc_chains_dot(smc_chains* h, const double* dev_a, const double* dev_w, double* dev_out);
int smc_chains_vjp(smc_chains* h, double beta, int64_t n_samples, const double* dev_cov_acc,
                   const double* dev_G_acc, const double* dev_mean, const float* dev_J,
                   float* dev_grad_J, double* dev_grad_beta);
int smc_chains_lnz_grad(smc_chains* h, double beta, const double* dev_mean, const float* dev_J,
                        const double* dev_scale, float* dev_grad_J_f32, double* dev_grad_J_f64,
                        double* dev_grad_beta);
int smc_chains_fit_step(smc_chains* h, double beta, double lr, const double* dev_target,
                        const double* dev_mean, float* dev_J);

/* One colour's half of sweep t for every chain (no accumulation; t is not
 * advanced).  Test hook for the counted near-threshold protocol of FP32
 * couplings (Eq. (2) decisions compared half-sweep by half-sweep).
 * Asynchronous. */
int smc_chains_half_sweep(smc_chains* h, double beta, int colour);

/* Kernel the handle's sweeps launch: "chains_pair" (at most 1024 site pairs
 * per colour, N <= 4096: one pair of sites per lane, state and couplings in
 * registers) or "chains_lds" (larger lattices, or SMC_CHAINS_KERNEL=lds in the
 * environment at init). */
const char* smc_chains_kernel_name(const smc_chains* h);

int smc_chains_get_sweep_index(const smc_chains* h, uint64_t* t);
int smc_chains_set_sweep_index(smc_chains* h, uint64_t t);
int smc_chains_destroy(smc_chains* h);

/* Conversions between int8 +-1 sites and the packed format (n_sites a
 * multiple of 32, any run of planes in storage order; asynchronous on
 * `stream`).  Packed: site k in bit k & 31 of word k >> 5, bit 1 = -1. */
int smc_pack_spins(const void* src_int8, void* dst_words, int64_t n_sites, void* stream);
int smc_unpack_spins(const void* src_words, void* dst_int8, int64_t n_sites, void* stream);

/* Measurement probes for the ceilings the sweep kernels are reported
 * against (asynchronous): kind 0 draws `reps` Philox4x32-10 blocks per lane
 * back to back (the random-number cost of every Ising kernel); kind 1 runs
 * `reps` iterations of eight independent chains of 32-bit xor / permute /
 * shift / add per lane (the practical integer VALU issue rate).  n_lanes a
 * positive multiple of 256; each lane writes one folded word to
 * dev_out[n_lanes] (uint32, caller-owned). */
int smc_probe(int32_t kind, uint32_t n_lanes, uint32_t reps, void* dev_out, void* stream);

/* The calling thread's last error message ("" if none). */
const char* smc_last_error(void);
const char* smc_version(void);

#ifdef __cplusplus
}
#endif

#endif /* SMC_H */
