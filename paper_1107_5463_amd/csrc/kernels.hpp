// kernels.hpp -- host-side launchers of the libsmc kernels (internal).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "device.hpp"
#include "launch_args.hpp"

namespace smc {

FastDiv make_fastdiv(uint32_t d);

// Raises kernel fn's dynamic-LDS limit on the current device to at least
// `bytes`, never lowering it: handles of different sizes share the kernels,
// and a later, smaller handle must not take LDS from an earlier one.
hipError_t allow_dynamic_lds(const void* fn, size_t bytes);

uint32_t stream_rows_per_band(const Geom& g, uint32_t min_waves);
int ising_variant_used(const IsingLaunch& a);  // the variant a launch resolves to
bool ising_half_sweep_measured(const IsingLaunch& a, int8_t* spins, uint32_t t, void* partials,
                               int64_t* nparts, hipStream_t st, hipError_t* err);

// Fused one-pass sweep (2D, uniform couplings): src -> dst, both [2][N/2].
bool ising_fused_supported(const Geom& g, int J_kind, uint32_t rows_per_band);
uint32_t fused_rows_per_band(const Geom& g, uint32_t min_blocks);
hipError_t launch_ising_sweep_fused(const IsingLaunch& a, const int8_t* src, int8_t* dst,
                                    uint32_t t, void* partials, int64_t* nparts, hipStream_t st);

hipError_t launch_ising_half_sweep(const IsingLaunch& a, int8_t* spins, uint32_t t,
                                   uint32_t colour, hipStream_t st);
// Chunk kernel requires L % 32 == 0 (plane rows are whole 16-byte chunks).
bool ising_chunk_supported(const Geom& g, int J_kind);

uint32_t cont_default_sites_per_lane(int n);
bool cont_sites_per_lane_ok(int n, uint32_t V);
bool cont_stream_supported(const Geom& g, uint32_t V, uint32_t H);
uint32_t cont_rows_per_band(const Geom& g, uint32_t V, uint32_t min_waves);
int cont_variant_used(const ContLaunch& a);
// Colour-1 half-sweep of the continuous streaming kernel with E and M of the
// resulting state reduced on the way (partials per block); false if the
// handle's kernel is not the streaming one.
bool cont_half_sweep_measured(const ContLaunch& a, float* spins, uint32_t t, void* partials,
                              int64_t* nparts, hipStream_t st, hipError_t* err);

hipError_t launch_cont_half_sweep(const ContLaunch& a, float* spins, uint32_t t,
                                  uint32_t colour, hipStream_t st);
hipError_t launch_renormalize(const Geom& g, int n, float* spins, hipStream_t st);

hipError_t launch_init_ising(const Geom& g, RngKey key, int hot, int8_t* spins, hipStream_t st);
hipError_t launch_init_continuous(const Geom& g, int n, RngKey key, int hot, float* spins,
                                  hipStream_t st);
hipError_t launch_init_couplings(const Geom& g, int J_kind, RngKey key, double J0, double sigma,
                                 void* J, hipStream_t st);

// With dev_obs, E and M of every lattice after every `every` sweeps (record m
// at dev_obs[m * n_lattices + lattice]; with n_sweeps = 0 one record).
hipError_t launch_batch(const BatchLaunch& a, int8_t* spins, const int8_t* J, uint32_t t0,
                        uint32_t n_sweeps, uint32_t every, void* dev_obs, hipStream_t st);
hipError_t batch_allow_lds(size_t bytes);
// Dynamic LDS of a batch launch with `threads` lanes per workgroup: the most
// any lattice needs -- its planes at one byte per site plus the per-lane tie
// queues, or, on the packed path, its planes and bond signs at one bit per
// site plus that path's tie queues.
size_t batch_lds_bytes(int d, bool pm, bool packed, const uint32_t* L, uint32_t n,
                       uint32_t threads);
// Whether a lattice of edge L takes the packed (one bit per site) path.
bool batch_lattice_packed(int d, uint32_t L, uint32_t threads);
// The kernel a batch launch uses (for building graph nodes); its arguments are
// (descs, order, key, spins, J, t0, n_sweeps, every, n_lattices, obs).
const void* batch_kernel_fn(int d, bool pm, bool measure);

// Number of per-block partials the measurement writes (workspace sizing).
int64_t measure_partials(const Geom& g);
// Reduce to an smc_obs-layout struct at dev_obs; partials: workspace scratch.
hipError_t launch_measure(const MeasureLaunch& a, const void* spins, void* partials,
                          void* dev_obs, hipStream_t st);
// Reduce nparts partials (written by a measuring sweep kernel) into dev_obs.
hipError_t launch_finish(const MeasureLaunch& a, const void* partials, int64_t nparts,
                         void* dev_obs, hipStream_t st);
// Partials a stand-alone measurement writes (packed spins: one per 256 words;
// otherwise at most the bounded grid's 2048 blocks).
int64_t measure_partials_standalone(const Geom& g, bool packed);
// Capacity, in partials, of the library's own measurement scratch (768 KiB).
constexpr int64_t kMeasureScratchPartials = 16384;
// Address on the current device of that scratch: a file-scope device array,
// one copy per GPU, looked up once per device and cached.
hipError_t measure_scratch(void** ptr);

hipError_t launch_bond_accumulate(const MeasureLaunch& a, const void* spins, void* acc,
                                  hipStream_t st);
hipError_t launch_bond_mean(const MeasureLaunch& a, const void* acc, int64_t samples,
                            double* out, hipStream_t st);
hipError_t launch_fill_zero(void* p, size_t bytes, hipStream_t st);

// Counts entries out of range into *dev_count (uint32 in device memory).
hipError_t launch_validate(const MeasureLaunch& a, const void* spins, uint32_t* dev_count,
                           hipStream_t st);

// Whether the pair kernel takes lattice g (at most 1024 site pairs per colour).
bool chains_pair_supported(const Geom& g);
size_t chains_lds_bytes(const Geom& g, int mode);
// Raise the dynamic-LDS limit of the chain kernels for lattice g.
hipError_t chains_allow_lds(const Geom& g);
hipError_t launch_chains_sample(const ChainsLaunch& a, int8_t* spins, uint32_t t0,
                                uint32_t n_sweeps, int64_t* bond_sum, hipStream_t st);
// Measurement probes: kind 0 Philox blocks, kind 1 integer VALU chains; reps
// blocks or iterations per lane, n_lanes a multiple of 256, out[n_lanes].
hipError_t launch_probe(int kind, uint32_t n_lanes, uint32_t reps, uint32_t* out, hipStream_t st);
// Finishing the derivative estimates over the d N bonds (FP64, deterministic).
hipError_t launch_chains_mean(const Geom& g, const int64_t* sum, int64_t n_samples, double* mean,
                              hipStream_t st);
hipError_t launch_chains_dot(const Geom& g, const double* a, const double* w, double* out,
                             hipStream_t st);
hipError_t launch_chains_vjp(const Geom& g, const double* cov_acc, const double* G_acc,
                             const double* mean, const float* J, int64_t n_samples, double beta,
                             float* grad_J, double* grad_beta, hipStream_t st);
hipError_t launch_chains_lnz_grad(const Geom& g, const double* mean, const float* J, double beta,
                                  const double* scale, float* gJ32, double* gJ64,
                                  double* grad_beta, hipStream_t st);
hipError_t launch_chains_fit_step(const Geom& g, const double* target, const double* mean,
                                  double rate, float* J, hipStream_t st);
// One colour's half of sweep t (no accumulation; t is not advanced).
hipError_t launch_chains_half_sweep(const ChainsLaunch& a, int8_t* spins, uint32_t t, int colour,
                                    hipStream_t st);
hipError_t launch_chains_covariance(const ChainsLaunch& a, int8_t* spins, uint32_t t0,
                                    uint32_t n_sweeps, const double* g, const double* gc, double* part,
                                    double* gpart, double* cov_acc, double* G_acc,
                                    hipStream_t st);

// Bit-packed Ising spins (32 sites per word, same plane order as int8).
bool packed_supported(const Geom& g, int J_kind);
uint32_t packed_rows_per_band(const Geom& g, uint32_t min_waves);
hipError_t launch_packed_half_sweep(const IsingLaunch& a, uint32_t* spins, const uint32_t* J,
                                    uint32_t t, uint32_t c, void* partials, int64_t* nparts,
                                    hipStream_t st);
hipError_t launch_pack(const int8_t* src, uint32_t* dst, int64_t n_words, hipStream_t st);
hipError_t launch_unpack(const uint32_t* src, int8_t* dst, int64_t n_words, hipStream_t st);
hipError_t launch_init_packed(const Geom& g, RngKey key, int mode, uint32_t* out, hipStream_t st);
hipError_t launch_measure_packed(const Geom& g, int J_kind, const uint32_t* s, const uint32_t* J,
                                 void* partials, int64_t* nparts, hipStream_t st);

// Tiled k-hit schedule (uniform couplings): one pass over the tiles of one colour.
size_t tile_lds_bytes(int d, uint32_t T);
bool tile_supported(const Geom& g, uint32_t T);
hipError_t tile_allow_lds(int d, size_t bytes);
hipError_t launch_tile_pass(const IsingLaunch& a, bool heatbath, uint32_t T, uint32_t hits,
                            int8_t* spins, uint32_t t, uint32_t tc, hipStream_t st, bool packed);
bool tile_packed_supported(const Geom& g, uint32_t T, bool heatbath);

}  // namespace smc
