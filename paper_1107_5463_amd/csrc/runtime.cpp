// runtime.cpp -- host runtime behind the C ABI declared in include/smc.h.
//
// Owns only the handle (host memory).  Every device buffer is the caller's;
// every call enqueues kernels on the handle's stream.  Boltzmann thresholds
// (the tabulated factors of Sec. 2) are built here in long double for each new
// beta: T[k] = ceil(2^32 exp(-beta dE_k)) with dE_k = 4 J0 (d - k) for k
// unsatisfied bonds.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstdint>
#include <cstdlib>
#include <cstring>
#include <numeric>
#include <string>
#include <vector>
#include <algorithm>
#include <map>
#include <mutex>
#include <utility>

#include "kernels.hpp"
#include "smc.h"

static_assert(sizeof(smc_obs) == 64, "smc_obs is eight 8-byte fields");

using namespace smc;

hipError_t smc::allow_dynamic_lds(const void* fn, size_t bytes) {
  static std::mutex mu;
  static std::map<std::pair<int, const void*>, size_t> granted;  // (device, kernel) -> limit set
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  std::lock_guard<std::mutex> lock(mu);
  size_t& g = granted[{dev, fn}];
  if (bytes <= g) return hipSuccess;
  e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
  if (e == hipSuccess) g = bytes;
  return e;
}

struct smc_lattice {
  smc_params p;
  Geom g;
  void* spins;
  void* J;
  char* ws;
  size_t ws_bytes;
  hipStream_t stream;
  uint64_t t;
  int64_t samples;
  bool tab_valid;
  double tab_beta;
  IsingTable tab;
  FastDiv divQ, divL;
  int ising_variant;         // IsingVariant (SMC_ISING_KERNEL overrides the automatic choice)
  uint32_t rows_per_band;    // streaming kernel band height (SMC_STREAM_ROWS overrides)
  bool use_fused;            // SMC_FLAG_SCHEDULE_FUSED and the fused kernel supports the shape
  uint32_t fused_rows;       // fused kernel band height (SMC_FUSED_ROWS overrides)
  uint32_t packed_rows;      // packed kernel band height (SMC_PACKED_ROWS overrides)
  int packed_ties;           // packed kernels' ties: 0 group, 1 lane, 2 group fallback (SMC_PACKED_TIES)
  bool tile_packed;          // tiled schedule: bit-packed tiles where they apply (SMC_TILE_KERNEL=byte: off)
  int cont_variant;          // ContVariant (SMC_CONT_KERNEL overrides the automatic choice)
  uint32_t cont_rows;        // continuous streaming band height (SMC_CONT_ROWS overrides)
  uint32_t cont_spl;         // continuous streaming sites per lane (SMC_CONT_SPL overrides)
  FastDiv divQc;             // continuous streaming lanes per plane row
  // workspace carve-up
  void* obs_slot;      // smc_obs (64 B)
  uint32_t* counter;   // validation counter
  void* partials;      // reduction partials
  void* alt_spins;     // second spin buffer (fused schedule)
};

namespace {

thread_local std::string g_err;

int fail(int code, const std::string& msg) {
  g_err = msg;
  return code;
}

int check(hipError_t e, const char* what) {
  if (e == hipSuccess) return SMC_OK;
  return fail(SMC_EDEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

constexpr size_t kAlign = 256;
constexpr size_t kPartialBytes = 48;  // one reduction partial (measure.hip)

size_t round_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

Geom make_geom(const smc_params* p);

bool params_ok(const smc_params* p, std::string& why) {
  if (!p) { why = "params is NULL"; return false; }
  if (p->d != 2 && p->d != 3) { why = "d must be 2 or 3"; return false; }
  if (p->n < 1 || p->n > 3) { why = "n must be 1, 2 or 3"; return false; }
  if (p->L < 4 || (p->L & 1)) { why = "L must be even and >= 4"; return false; }
  const double N = std::pow((double)p->L, p->d);
  if (N >= 4294967296.0) { why = "lattice too large (N must be < 2^32)"; return false; }
  if (p->J_kind < 0 || p->J_kind > 2) { why = "J_kind must be 0, 1 or 2"; return false; }
  if (p->init < 0 || p->init > 2) { why = "init must be HOT, COLD or KEEP"; return false; }
  if (!std::isfinite(p->J0)) { why = "J0 must be finite"; return false; }
  if (!std::isfinite(p->J_sigma) || p->J_sigma < 0) { why = "J_sigma must be finite and >= 0"; return false; }
  if (p->renorm_every < 0) { why = "renorm_every must be >= 0"; return false; }
  if (p->n > 1) {
    if (!std::isfinite(p->delta) || p->delta <= 0.0) { why = "delta must be finite and > 0"; return false; }
    if (p->n == 3 && p->delta > M_PI) { why = "Heisenberg cap half-angle must be <= pi"; return false; }
  }
  if (p->flags & ~(SMC_FLAG_FAST_MATH | SMC_FLAG_SCHEDULE_FUSED | SMC_FLAG_GENERIC_KERNEL |
                   SMC_FLAG_COUPLINGS_KEEP | SMC_FLAG_PACKED | SMC_FLAG_HEATBATH)) {
    why = "unknown flag bits";
    return false;
  }
  if (p->flags & SMC_FLAG_HEATBATH) {
    if (p->n != 1) { why = "the heat-bath rule is Ising only (n = 1)"; return false; }
    if (p->J_kind == SMC_J_FP32) { why = "the heat-bath rule takes uniform or +-1 couplings"; return false; }
    if (p->flags & SMC_FLAG_PACKED) { why = "packed spins run the Metropolis rule"; return false; }
  }
  if (p->tile < 0) { why = "tile must be >= 0"; return false; }
  if (p->tile == 0 && (p->hits < 0 || p->hits > 1)) { why = "hits must be 0 or 1 without tiles"; return false; }
  if (p->tile > 0) {
    if (p->n != 1 || p->J_kind != SMC_J_UNIFORM || (p->flags & SMC_FLAG_PACKED)) {
      why = "the tiled schedule takes int8 Ising spins with uniform couplings";
      return false;
    }
    if (p->hits < 1 || p->hits > (1 << 23)) { why = "hits must be in [1, 2^23]"; return false; }
    if (!tile_supported(make_geom(p), (uint32_t)p->tile)) {
      why = "tile must be 16 or a multiple of 32 dividing L with L / tile even, and fit LDS";
      return false;
    }
  }
  if (p->flags & SMC_FLAG_PACKED) {
    if (p->n != 1) { why = "packed spins are Ising only (n = 1)"; return false; }
    if (p->J_kind == SMC_J_FP32) { why = "packed spins take uniform or +-1 couplings"; return false; }
    if (!packed_supported(make_geom(p), p->J_kind)) {
      why = "packed spins need L % 64 == 0 and at most 2^24 rows of L sites per colour plane";
      return false;
    }
  }
  return true;
}

bool is_packed(const smc_params* p) { return (p->flags & SMC_FLAG_PACKED) != 0; }

int64_t n_sites(const smc_params* p) {
  int64_t N = 1;
  for (int k = 0; k < p->d; ++k) N *= p->L;
  return N;
}

Geom make_geom(const smc_params* p) {
  Geom g;
  g.L = p->L;
  g.d = p->d;
  g.R = p->L / 2;
  g.rows = p->d == 2 ? p->L : p->L * p->L;
  g.Nh = n_sites(p) / 2;
  return g;
}

size_t spin_bytes(const smc_params* p) {
  if (is_packed(p)) return (size_t)n_sites(p) / 8;
  return (size_t)n_sites(p) * (p->n == 1 ? 1 : 4 * (size_t)p->n);
}

size_t partial_bytes(const smc_params* p) {
  const Geom g = make_geom(p);
  return round_up((size_t)measure_partials(g) * kPartialBytes, kAlign);
}

bool beta_ok(double beta) { return !std::isnan(beta) && beta >= 0.0; }

RngKey key_of(const smc_lattice* h) {
  return RngKey{(uint32_t)(h->p.seed & 0xffffffffu), (uint32_t)(h->p.seed >> 32), h->p.replica};
}

// Integer Boltzmann thresholds per class k of unsatisfied bonds (k = 0..2d),
// dE_k = 4 J0 (d - k): T = ceil(2^32 exp(-beta dE)) in long double.
IsingTable make_table(int d, double J0, double beta) {
  IsingTable tab;
  std::memset(&tab, 0, sizeof(tab));
  uint8_t th[8] = {0}, al[8] = {0};
  for (int k = 0; k <= 2 * d; ++k) {
    const long double dE = 4.0L * (long double)J0 * (long double)(d - k);
    bool always = false;
    uint64_t T = 0;
    if (!(dE > 0.0L)) {
      always = true;
    } else if (std::isinf(beta)) {
      T = 0;
    } else {
      const long double x = std::ldexp(std::exp(-(long double)beta * dE), 32);
      const long double c = std::ceil(x);
      if (c >= 4294967296.0L) always = true;
      else T = (uint64_t)c;
    }
    if (always) {
      // the fast kernels test only the threshold byte: 0xFF with a refinement
      // fraction of 2^24 accepts on every draw (prefix < 255, or prefix = 255
      // and any 24-bit refinement word)
      al[k] = 0xFF;
      th[k] = 0xFF;
      tab.frac[k] = 0x1000000u;
    } else {
      th[k] = (uint8_t)(T >> 24);
      tab.frac[k] = (uint32_t)(T & 0xFFFFFFu);
    }
  }
  tab.th_lo = th[0] | (th[1] << 8) | (th[2] << 16) | ((uint32_t)th[3] << 24);
  tab.th_hi = th[4] | (th[5] << 8) | (th[6] << 16) | ((uint32_t)th[7] << 24);
  tab.al_lo = al[0] | (al[1] << 8) | (al[2] << 16) | ((uint32_t)al[3] << 24);
  tab.al_hi = al[4] | (al[5] << 8) | (al[6] << 16) | ((uint32_t)al[7] << 24);
  return tab;
}

// Heat-bath thresholds per class npos (neighbours with sign(J) s = +1):
// T = ceil(2^32 / (1 + exp(-2 beta J0 (2 npos - 2d)))) in long double;
// T >= 2^32 is stored as threshold byte 0xFF with fraction 2^24 (always +1).
IsingTable make_table_hb(int d, double J0, double beta) {
  IsingTable tab;
  std::memset(&tab, 0, sizeof(tab));
  uint8_t th[8] = {0};
  for (int np = 0; np <= 2 * d; ++np) {
    const long double h = (long double)J0 * (long double)(2 * np - 2 * d);
    uint64_t T;
    if (std::isinf(beta)) {
      T = h > 0 ? 4294967296ull : (h < 0 ? 0ull : 2147483648ull);
    } else {
      const long double x = std::ldexp(1.0L / (1.0L + std::exp(-2.0L * (long double)beta * h)), 32);
      const long double c = std::ceil(x);
      T = c >= 4294967296.0L ? 4294967296ull : (uint64_t)c;
    }
    if (T >= 4294967296ull) {
      th[np] = 0xFF;
      tab.frac[np] = 0x1000000u;
    } else {
      th[np] = (uint8_t)(T >> 24);
      tab.frac[np] = (uint32_t)(T & 0xFFFFFFu);
    }
  }
  tab.th_lo = th[0] | (th[1] << 8) | (th[2] << 16) | ((uint32_t)th[3] << 24);
  tab.th_hi = th[4] | (th[5] << 8) | (th[6] << 16) | ((uint32_t)th[7] << 24);
  return tab;
}

void build_table(smc_lattice* h, double beta) {
  if (h->tab_valid && h->tab_beta == beta) return;
  h->tab = (h->p.flags & SMC_FLAG_HEATBATH) ? make_table_hb(h->p.d, h->p.J0, beta)
                                            : make_table(h->p.d, h->p.J0, beta);
  h->tab_beta = beta;
  h->tab_valid = true;
}

MeasureLaunch measure_args(const smc_lattice* h, int64_t sweep) {
  MeasureLaunch m;
  m.g = h->g;
  m.n = h->p.n;
  m.J_kind = h->p.J_kind;
  m.J = h->J;
  m.J0 = h->p.J0;
  m.sweep = sweep;
  return m;
}

IsingLaunch ising_args(smc_lattice* h, double beta) {
  if (h->p.J_kind != SMC_J_FP32) build_table(h, beta);
  IsingLaunch a;
  a.g = h->g;
  a.key = key_of(h);
  a.tab = h->tab;
  a.J_kind = h->p.J_kind;
  a.J = h->J;
  a.beta = (float)beta;
  a.variant = (h->p.flags & SMC_FLAG_GENERIC_KERNEL) ? kVariantSite : h->ising_variant;
  a.rows_per_band = h->rows_per_band;
  a.divQ = h->divQ;
  a.divL = h->divL;
  a.heatbath = (h->p.flags & SMC_FLAG_HEATBATH) ? 1 : 0;
  a.packed_ties = h->packed_ties;
  return a;
}

// E and M of a state (any spin format) into dev_obs, the block partials in
// `partials` (a handle's workspace, or the library's scratch).
hipError_t measure_state(const smc_params& p, const Geom& g, const void* spins, const void* J,
                         void* partials, int64_t sweep, void* dev_obs, hipStream_t st) {
  MeasureLaunch m;
  m.g = g;
  m.n = p.n;
  m.J_kind = p.J_kind;
  m.J = p.J_kind == SMC_J_UNIFORM ? nullptr : J;
  m.J0 = p.J0;
  m.sweep = sweep;
  if (is_packed(&p)) {
    int64_t nparts = 0;
    const hipError_t e = launch_measure_packed(g, p.J_kind, (const uint32_t*)spins,
                                               (const uint32_t*)m.J, partials, &nparts, st);
    if (e != hipSuccess) return e;
    return launch_finish(m, partials, nparts, dev_obs, st);
  }
  return launch_measure(m, spins, partials, dev_obs, st);
}

// E and M of the handle's current state into dev_obs.
hipError_t measure_any(smc_lattice* h, int64_t sweep, void* dev_obs) {
  return measure_state(h->p, h->g, h->spins, h->J, h->partials, sweep, dev_obs, h->stream);
}

ContLaunch cont_args(const smc_lattice* h, double beta) {
  ContLaunch a;
  std::memset(&a, 0, sizeof(a));
  a.g = h->g;
  a.n = h->p.n;
  a.key = key_of(h);
  a.J_kind = h->p.J_kind;
  a.J0 = (float)h->p.J0;
  a.J0d = h->p.J0;
  a.J = h->J;
  a.beta = (float)beta;
  a.delta = (float)h->p.delta;
  a.one_minus_cos_cap = (float)(1.0 - std::cos(h->p.delta));
  a.fast_math = (h->p.flags & SMC_FLAG_FAST_MATH) ? 1 : 0;
  a.variant = h->cont_variant;
  a.rows_per_band = h->cont_rows;
  a.sites_per_lane = h->cont_spl;
  a.divQ = h->divQc;
  a.divL = h->divL;
  return a;
}

int half_sweep_impl(smc_lattice* h, double beta, uint32_t t, uint32_t colour) {
  if (is_packed(&h->p)) {
    IsingLaunch a = ising_args(h, beta);
    a.rows_per_band = h->packed_rows;
    return check(launch_packed_half_sweep(a, (uint32_t*)h->spins, (const uint32_t*)h->J, t, colour,
                                          nullptr, nullptr, h->stream),
                 "packed Ising half-sweep launch");
  }
  if (h->p.n == 1) {
    const IsingLaunch a = ising_args(h, beta);
    return check(launch_ising_half_sweep(a, (int8_t*)h->spins, t, colour, h->stream),
                 "Ising half-sweep launch");
  }
  const ContLaunch a = cont_args(h, beta);
  return check(launch_cont_half_sweep(a, (float*)h->spins, t, colour, h->stream),
               "continuous half-sweep launch");
}

// One in-place two-pass sweep with counter t; with dev_obs the observables of
// the result are written there (fused into the colour-1 pass when the
// streaming kernel runs, else by a separate measurement).
int two_pass_sweep(smc_lattice* h, double beta, uint32_t t, void* dev_obs) {
  int rc = half_sweep_impl(h, beta, t, 0u);
  if (rc != SMC_OK) return rc;
  if (dev_obs && is_packed(&h->p)) {
    IsingLaunch a = ising_args(h, beta);
    a.rows_per_band = h->packed_rows;
    int64_t nparts = 0;
    rc = check(launch_packed_half_sweep(a, (uint32_t*)h->spins, (const uint32_t*)h->J, t, 1u,
                                        h->partials, &nparts, h->stream),
               "measured packed half-sweep launch");
    if (rc != SMC_OK) return rc;
    return check(launch_finish(measure_args(h, (int64_t)t + 1), h->partials, nparts, dev_obs, h->stream),
                 "measurement finish launch");
  }
  if (dev_obs && h->p.n == 1) {
    const IsingLaunch a = ising_args(h, beta);
    int64_t nparts = 0;
    hipError_t err = hipSuccess;
    if (ising_half_sweep_measured(a, (int8_t*)h->spins, t, h->partials, &nparts, h->stream, &err)) {
      rc = check(err, "measured Ising half-sweep launch");
      if (rc != SMC_OK) return rc;
      return check(launch_finish(measure_args(h, (int64_t)t + 1), h->partials, nparts, dev_obs, h->stream),
                   "measurement finish launch");
    }
  }
  if (dev_obs && h->p.n > 1) {
    const ContLaunch a = cont_args(h, beta);
    int64_t nparts = 0;
    hipError_t err = hipSuccess;
    if (cont_half_sweep_measured(a, (float*)h->spins, t, h->partials, &nparts, h->stream, &err)) {
      rc = check(err, "measured continuous half-sweep launch");
      if (rc != SMC_OK) return rc;
      return check(launch_finish(measure_args(h, (int64_t)t + 1), h->partials, nparts, dev_obs, h->stream),
                   "measurement finish launch");
    }
  }
  rc = half_sweep_impl(h, beta, t, 1u);
  if (rc != SMC_OK) return rc;
  if (dev_obs)
    return check(measure_any(h, (int64_t)t + 1, dev_obs),
                 "measurement launch");
  return SMC_OK;
}

// n sweeps from t with the fused kernel, ping-ponging through the workspace
// buffer; an odd count starts with one in-place two-pass sweep so that the
// state always ends in the caller's buffer.
int fused_sweeps(smc_lattice* h, double beta, int64_t n, void* dev_obs) {
  int64_t k = 0;
  if (n % 2 == 1) {
    const int rc = two_pass_sweep(h, beta, (uint32_t)h->t, n == 1 ? dev_obs : nullptr);
    if (rc != SMC_OK) return rc;
    h->t += 1;
    k = 1;
  }
  const IsingLaunch a = ising_args(h, beta);
  IsingLaunch af = a;
  af.rows_per_band = h->fused_rows;
  int8_t* A = (int8_t*)h->spins;
  int8_t* B = (int8_t*)h->alt_spins;
  for (; k < n; k += 2) {
    const bool last = k + 2 >= n;
    int rc = check(launch_ising_sweep_fused(af, A, B, (uint32_t)h->t, nullptr, nullptr, h->stream),
                   "fused sweep launch");
    if (rc != SMC_OK) return rc;
    int64_t nparts = 0;
    void* parts = (last && dev_obs) ? h->partials : nullptr;
    rc = check(launch_ising_sweep_fused(af, B, A, (uint32_t)h->t + 1, parts, &nparts, h->stream),
               "fused sweep launch");
    if (rc != SMC_OK) return rc;
    h->t += 2;
    if (parts) {
      rc = check(launch_finish(measure_args(h, h->t), h->partials, nparts, dev_obs, h->stream),
                 "measurement finish launch");
      if (rc != SMC_OK) return rc;
    }
  }
  return SMC_OK;
}

// Tiled k-hit sweeps: per sweep one pass over each tile colour.
int tiled_sweeps(smc_lattice* h, double beta, int64_t n_sweeps, void* dev_obs) {
  const IsingLaunch a = ising_args(h, beta);
  const bool hb = (h->p.flags & SMC_FLAG_HEATBATH) != 0;
  for (int64_t k = 0; k < n_sweeps; ++k) {
    for (uint32_t tc = 0; tc < 2; ++tc) {
      const int rc = check(launch_tile_pass(a, hb, (uint32_t)h->p.tile, (uint32_t)h->p.hits,
                                            (int8_t*)h->spins, (uint32_t)h->t, tc, h->stream,
                                            h->tile_packed),
                           "tile pass launch");
      if (rc != SMC_OK) return rc;
    }
    h->t += 1;
  }
  if (dev_obs) return check(measure_any(h, h->t, dev_obs), "measurement launch");
  return SMC_OK;
}

int sweeps_impl(smc_lattice* h, double beta, int64_t n_sweeps, void* dev_obs) {
  if (h->p.tile > 0) return tiled_sweeps(h, beta, n_sweeps, dev_obs);
  if (h->use_fused) return fused_sweeps(h, beta, n_sweeps, dev_obs);
  for (int64_t k = 0; k < n_sweeps; ++k) {
    const bool last = k + 1 == n_sweeps;
    const bool renorm = h->p.n > 1 && h->p.renorm_every > 0 &&
                        (h->t + 1) % (uint64_t)h->p.renorm_every == 0;
    int rc = two_pass_sweep(h, beta, (uint32_t)h->t, (last && !renorm) ? dev_obs : nullptr);
    if (rc != SMC_OK) return rc;
    h->t += 1;
    if (renorm) {
      rc = check(launch_renormalize(h->g, h->p.n, (float*)h->spins, h->stream), "renormalisation launch");
      if (rc != SMC_OK) return rc;
      if (last && dev_obs)
        return check(measure_any(h, h->t, dev_obs),
                     "measurement launch");
    }
  }
  return SMC_OK;
}

// ---------------------------------------------------------------------------
// Autotuning of schedules, with a cache of the choices in the file named by
// SMC_AUTOTUNE_CACHE (lines "key value"; the key names the kernel, the shape
// and the device).
// ---------------------------------------------------------------------------
std::mutex g_cache_mu;

std::string device_tag() {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return "dev?";
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, dev) != hipSuccess) return "dev?";
  return std::string(prop.gcnArchName) + ",cu" + std::to_string(prop.multiProcessorCount);
}

std::map<std::string, std::string> cache_read(const char* path) {
  std::map<std::string, std::string> m;
  FILE* f = std::fopen(path, "r");
  if (!f) return m;
  char line[1024];
  while (std::fgets(line, sizeof(line), f)) {
    std::string l(line);
    while (!l.empty() && (l.back() == '\n' || l.back() == '\r')) l.pop_back();
    const size_t sp = l.find(' ');
    if (sp == std::string::npos || sp == 0) continue;
    m[l.substr(0, sp)] = l.substr(sp + 1);
  }
  std::fclose(f);
  return m;
}

bool cache_get(const std::string& key, std::string& value) {
  const char* path = std::getenv("SMC_AUTOTUNE_CACHE");
  if (!path || !*path) return false;
  std::lock_guard<std::mutex> lock(g_cache_mu);
  const auto m = cache_read(path);
  const auto it = m.find(key);
  if (it == m.end()) return false;
  value = it->second;
  return true;
}

void cache_put(const std::string& key, const std::string& value) {
  const char* path = std::getenv("SMC_AUTOTUNE_CACHE");
  if (!path || !*path) return;
  std::lock_guard<std::mutex> lock(g_cache_mu);
  auto m = cache_read(path);
  m[key] = value;
  const std::string tmp = std::string(path) + ".tmp";
  FILE* f = std::fopen(tmp.c_str(), "w");
  if (!f) return;
  for (const auto& kv : m) std::fprintf(f, "%s %s\n", kv.first.c_str(), kv.second.c_str());
  std::fclose(f);
  std::rename(tmp.c_str(), path);
}

// The band height field of the handle's banded kernel and its candidates
// (powers of two dividing L that the kernel takes); nullptr if the handle's
// sweeps run a kernel without bands.
uint32_t* band_field(smc_lattice* h, std::vector<uint32_t>& cand, const char** what) {
  cand.clear();
  const Geom& g = h->g;
  auto pow2 = [&](uint32_t lo, uint32_t hi, auto ok) {
    for (uint32_t H = lo; H <= hi; H *= 2)
      if ((uint32_t)g.L % H == 0 && ok(H)) cand.push_back(H);
  };
  if (h->p.tile > 0) return nullptr;
  if (h->use_fused) {
    *what = "fused";
    pow2(4, 64, [&](uint32_t H) { return ising_fused_supported(g, h->p.J_kind, H); });
    return &h->fused_rows;
  }
  if (is_packed(&h->p)) {
    *what = "packed";
    pow2(1, 64, [](uint32_t) { return true; });
    return &h->packed_rows;
  }
  if (h->p.n > 1) {
    ContLaunch a = cont_args(h, 0.0);
    if (cont_variant_used(a) != kContStream) return nullptr;
    *what = h->p.n == 2 ? "xy_stream" : "heisenberg_stream";
    pow2(4, 64, [&](uint32_t H) { return cont_stream_supported(g, h->cont_spl, H); });
    return &h->cont_rows;
  }
  IsingLaunch a = ising_args(h, 0.0);
  if (ising_variant_used(a) != kVariantStream) return nullptr;
  *what = "ising_stream";
  pow2(4, 64, [&](uint32_t H) {
    a.rows_per_band = H;
    return ising_variant_used(a) == kVariantStream;
  });
  return &h->rows_per_band;
}

}  // namespace

extern "C" {

int smc_autotune(smc_lattice* h, double beta, void* scratch, size_t scratch_bytes,
                 uint32_t* rows_out) {
  if (!h) return fail(SMC_EINVAL, "handle is NULL");
  if (!beta_ok(beta) || std::isinf(beta)) return fail(SMC_EINVAL, "beta must be finite and >= 0");
  std::vector<uint32_t> cand;
  const char* what = "";
  uint32_t* field = band_field(h, cand, &what);
  if (!field || cand.empty()) {
    if (rows_out) *rows_out = 0;
    return SMC_OK;
  }
  const std::string key = std::string(what) + ":d" + std::to_string(h->p.d) + ":n" +
                          std::to_string(h->p.n) + ":L" + std::to_string(h->p.L) + ":J" +
                          std::to_string(h->p.J_kind) + ":" + device_tag();
  std::string cached;
  if (cache_get(key, cached)) {
    const uint32_t v = (uint32_t)std::strtoul(cached.c_str(), nullptr, 10);
    if (std::find(cand.begin(), cand.end(), v) != cand.end()) {
      *field = v;
      if (rows_out) *rows_out = v;
      return SMC_OK;
    }
  }
  const size_t sb = spin_bytes(&h->p);
  if (!scratch || ((uintptr_t)scratch & 15) || scratch_bytes < sb)
    return fail(SMC_EINVAL, "scratch must be 16-byte aligned and hold " + std::to_string(sb) +
                                " bytes (a copy of the spins)");
  int rc = check(hipMemcpyAsync(scratch, h->spins, sb, hipMemcpyDeviceToDevice, h->stream),
                 "scratch copy");
  if (rc != SMC_OK) return rc;
  hipEvent_t e0, e1;
  if ((rc = check(hipEventCreate(&e0), "event create")) != SMC_OK) return rc;
  if ((rc = check(hipEventCreate(&e1), "event create")) != SMC_OK) {
    (void)hipEventDestroy(e0);
    return rc;
  }
  // sweeps of the handle's own buffer (its placement in memory and in the
  // Infinity Cache is what the timed sweeps will see), restored from the
  // scratch copy afterwards
  const uint64_t t_saved = h->t;
  const uint32_t saved_rows = *field;
  // Timings of K sweeps each (about 2e9 attempts), after a warm-up that
  // brings the clocks to their sustained state; the candidates are timed in
  // turn over three rounds (so a drift of the clocks touches them alike) and
  // ranked by their median.  The default height is kept unless another is
  // more than 2 % faster.
  const double N = (double)n_sites(&h->p);
  const int64_t K = std::max<int64_t>(4, std::min<int64_t>(128, (int64_t)std::ceil(2e9 / N)));
  const char* vb = std::getenv("SMC_AUTOTUNE_VERBOSE");
  const bool verbose = vb && *vb && *vb != '0';
  constexpr int kRounds = 3;
  std::vector<std::vector<float>> times(cand.size());
  rc = sweeps_impl(h, beta, 2 * K, nullptr);
  for (int round = 0; round < kRounds && rc == SMC_OK; ++round) {
    for (size_t i = 0; i < cand.size() && rc == SMC_OK; ++i) {
      *field = cand[i];
      rc = sweeps_impl(h, beta, 1, nullptr);  // a launch at the new height before timing it
      if (rc == SMC_OK) rc = check(hipEventRecord(e0, h->stream), "event record");
      if (rc == SMC_OK) rc = sweeps_impl(h, beta, K, nullptr);
      if (rc == SMC_OK) rc = check(hipEventRecord(e1, h->stream), "event record");
      if (rc == SMC_OK) rc = check(hipEventSynchronize(e1), "event synchronise");
      float ms = 0.0f;
      if (rc == SMC_OK) rc = check(hipEventElapsedTime(&ms, e0, e1), "event time");
      if (rc == SMC_OK) times[i].push_back(ms);
      if (rc == SMC_OK && verbose)
        std::fprintf(stderr, "smc_autotune %s: rows %u, %lld sweeps, %.3f ms\n", what, cand[i],
                     (long long)K, ms);
      h->t = t_saved;
    }
  }
  uint32_t best_H = saved_rows;
  if (rc == SMC_OK) {
    auto median = [](std::vector<float> v) {
      std::sort(v.begin(), v.end());
      return v[v.size() / 2];
    };
    float best = 1e30f, deflt = -1.0f;
    for (size_t i = 0; i < cand.size(); ++i) {
      const float m = median(times[i]);
      if (cand[i] == saved_rows) deflt = m;
      if (m < best) {
        best = m;
        best_H = cand[i];
      }
    }
    if (deflt > 0.0f && deflt <= 1.02f * best) best_H = saved_rows;
  }
  h->t = t_saved;
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  const int rc_restore = check(hipMemcpyAsync(h->spins, scratch, sb, hipMemcpyDeviceToDevice,
                                              h->stream), "state restore");
  if (rc == SMC_OK) rc = rc_restore;
  if (rc == SMC_OK) rc = check(hipStreamSynchronize(h->stream), "stream synchronise");
  if (rc != SMC_OK) {
    *field = saved_rows;
    return rc;
  }
  *field = best_H;
  cache_put(key, std::to_string(best_H));
  if (rows_out) *rows_out = best_H;
  return SMC_OK;
}

size_t smc_spin_bytes(const smc_params* p) {
  std::string why;
  return params_ok(p, why) ? spin_bytes(p) : 0;
}

size_t smc_coupling_bytes(const smc_params* p) {
  std::string why;
  if (!params_ok(p, why) || p->J_kind == SMC_J_UNIFORM) return 0;
  if (is_packed(p)) return (size_t)n_sites(p) * p->d / 8;
  return (size_t)n_sites(p) * p->d * (p->J_kind == SMC_J_PM ? 1 : 4);
}

size_t smc_workspace_bytes(const smc_params* p) {
  std::string why;
  if (!params_ok(p, why)) return 0;
  size_t b = 2 * kAlign;  // observable slot + counter
  b += partial_bytes(p);
  if ((p->flags & SMC_FLAG_SCHEDULE_FUSED) && !is_packed(p)) b += round_up(spin_bytes(p), kAlign);
  return b;
}

size_t smc_bond_bytes(const smc_params* p) {
  std::string why;
  return params_ok(p, why) && !is_packed(p) ? (size_t)n_sites(p) * p->d * 8 : 0;
}

int smc_init_lattice(smc_lattice** out, const smc_params* p, void* spins, void* J,
                     void* workspace, size_t workspace_bytes, void* stream) {
  g_err.clear();
  if (!out) return fail(SMC_EINVAL, "out is NULL");
  *out = nullptr;
  std::string why;
  if (!params_ok(p, why)) return fail(SMC_EINVAL, why);
  if (!spins || ((uintptr_t)spins & 15)) return fail(SMC_EINVAL, "spins must be non-NULL and 16-byte aligned");
  if (p->J_kind != SMC_J_UNIFORM && (!J || ((uintptr_t)J & 15)))
    return fail(SMC_EINVAL, "J must be non-NULL and 16-byte aligned for PM / FP32 couplings");
  if (!workspace || ((uintptr_t)workspace & (kAlign - 1)))
    return fail(SMC_EINVAL, "workspace must be non-NULL and 256-byte aligned");
  if (workspace_bytes < smc_workspace_bytes(p))
    return fail(SMC_EINVAL, "workspace too small: need " + std::to_string(smc_workspace_bytes(p)) +
                                " bytes");
  smc_lattice* h = new (std::nothrow) smc_lattice();
  if (!h) return fail(SMC_EINVAL, "out of host memory");
  h->p = *p;
  h->g = make_geom(p);
  h->spins = spins;
  h->J = p->J_kind == SMC_J_UNIFORM ? nullptr : J;
  h->ws = (char*)workspace;
  h->ws_bytes = workspace_bytes;
  h->stream = (hipStream_t)stream;
  h->t = 0;
  h->samples = 0;
  h->tab_valid = false;
  h->divQ = make_fastdiv((uint32_t)(h->g.R / 16 > 0 ? h->g.R / 16 : 1));
  h->divL = make_fastdiv((uint32_t)h->g.L);
  h->ising_variant = kVariantAuto;
  if (const char* v = std::getenv("SMC_ISING_KERNEL")) {
    const std::string s(v);
    h->ising_variant = s == "site" ? kVariantSite : s == "chunk" ? kVariantChunk
                     : s == "stream" ? kVariantStream : s == "fused_wave" ? kVariantFusedWave
                     : kVariantAuto;
  }
  // at least 2048 waves (two per SIMD): longer bands re-read fewer halo rows,
  // and the software-pipelined ring keeps enough loads in flight per wave
  h->rows_per_band = stream_rows_per_band(h->g, 2048);
  if (const char* v = std::getenv("SMC_STREAM_ROWS")) {
    const long H = std::strtol(v, nullptr, 10);
    if (H >= 1 && H <= 64 && H <= h->g.L && h->g.L % H == 0) h->rows_per_band = (uint32_t)H;
  }
  h->obs_slot = h->ws;
  h->counter = (uint32_t*)(h->ws + kAlign);
  h->partials = h->ws + 2 * kAlign;
  h->alt_spins = (p->flags & SMC_FLAG_SCHEDULE_FUSED) ? (void*)(h->ws + 2 * kAlign + partial_bytes(p))
                                                      : nullptr;
  h->fused_rows = fused_rows_per_band(h->g, 512);
  if (const char* v = std::getenv("SMC_FUSED_ROWS")) {
    const long H = std::strtol(v, nullptr, 10);
    if (H >= 1 && H <= 64 && H <= h->g.L && h->g.L % H == 0) h->fused_rows = (uint32_t)H;
  }
  h->packed_rows = packed_rows_per_band(h->g, 8192);
  h->packed_ties = 0;
  h->tile_packed = true;
  if (const char* v = std::getenv("SMC_TILE_KERNEL")) h->tile_packed = std::string(v) != "byte";
  if (const char* v = std::getenv("SMC_PACKED_TIES")) {
    const std::string s(v);
    if (s == "lane") h->packed_ties = 1;
    if (s == "group" || s == "wave") h->packed_ties = 0;
    if (s == "fallback") h->packed_ties = 2;
  }
  if (const char* v = std::getenv("SMC_PACKED_ROWS")) {
    const long H = std::strtol(v, nullptr, 10);
    if (H >= 1 && H <= 64 && H <= h->g.L && h->g.L % H == 0) h->packed_rows = (uint32_t)H;
  }
  h->cont_variant = (p->flags & SMC_FLAG_GENERIC_KERNEL) ? kContRow : kContAuto;
  if (const char* v = std::getenv("SMC_CONT_KERNEL")) {
    const std::string s(v);
    if (s == "row") h->cont_variant = kContRow;
    if (s == "stream") h->cont_variant = kContStream;
  }
  h->cont_spl = p->n > 1 ? cont_default_sites_per_lane(p->n) : 1;
  if (const char* v = std::getenv("SMC_CONT_SPL")) {
    const long V = std::strtol(v, nullptr, 10);
    if (p->n > 1 && V > 0 && cont_sites_per_lane_ok(p->n, (uint32_t)V)) h->cont_spl = (uint32_t)V;
  }
  h->cont_rows = p->n > 1 ? cont_rows_per_band(h->g, h->cont_spl, 2048) : 4;
  if (const char* v = std::getenv("SMC_CONT_ROWS")) {
    const long H = std::strtol(v, nullptr, 10);
    if (H >= 4 && H <= 64 && H % 4 == 0 && H <= h->g.L && h->g.L % H == 0) h->cont_rows = (uint32_t)H;
  }
  {
    const uint32_t Qc = (uint32_t)h->g.R / h->cont_spl;
    h->divQc = make_fastdiv(Qc > 0 ? Qc : 1);
  }
  h->use_fused = p->n == 1 && !is_packed(p) && p->tile == 0 && !(p->flags & SMC_FLAG_HEATBATH) &&
                 (p->flags & SMC_FLAG_SCHEDULE_FUSED) &&
                 !(p->flags & SMC_FLAG_GENERIC_KERNEL) &&
                 ising_fused_supported(h->g, p->J_kind, h->fused_rows);
  const RngKey key = key_of(h);
  int rc = SMC_OK;
  if (p->tile > 0)
    rc = check(tile_allow_lds(p->d, tile_lds_bytes(p->d, (uint32_t)p->tile)), "tile LDS attribute");
  if (rc == SMC_OK && is_packed(p)) {
    if (p->J_kind == SMC_J_PM && !(p->flags & SMC_FLAG_COUPLINGS_KEEP))
      rc = check(launch_init_packed(h->g, key, 2, (uint32_t*)h->J, h->stream), "coupling init launch");
    if (rc == SMC_OK && p->init != SMC_INIT_KEEP)
      rc = check(launch_init_packed(h->g, key, p->init == SMC_INIT_HOT ? 0 : 1, (uint32_t*)spins,
                                    h->stream),
                 "spin init launch");
  } else if (rc == SMC_OK && p->J_kind != SMC_J_UNIFORM && !(p->flags & SMC_FLAG_COUPLINGS_KEEP)) {
    rc = check(launch_init_couplings(h->g, p->J_kind, key, p->J0, p->J_sigma, h->J, h->stream),
               "coupling init launch");
  }
  if (rc == SMC_OK && p->init != SMC_INIT_KEEP && !is_packed(p)) {
    const int hot = p->init == SMC_INIT_HOT;
    if (p->n == 1)
      rc = check(launch_init_ising(h->g, key, hot, (int8_t*)spins, h->stream), "spin init launch");
    else
      rc = check(launch_init_continuous(h->g, p->n, key, hot, (float*)spins, h->stream),
                 "spin init launch");
  }
  if (rc != SMC_OK) {
    delete h;
    return rc;
  }
  *out = h;
  return SMC_OK;
}

int smc_set_stream(smc_lattice* h, void* stream) {
  if (!h) return fail(SMC_EINVAL, "handle is NULL");
  h->stream = (hipStream_t)stream;
  return SMC_OK;
}

int smc_sweep(smc_lattice* h, double beta, int64_t n_sweeps) {
  if (!h) return fail(SMC_EINVAL, "handle is NULL");
  if (!beta_ok(beta)) return fail(SMC_EINVAL, "beta must be >= 0 (or +inf), not NaN");
  if (n_sweeps < 0) return fail(SMC_EINVAL, "n_sweeps must be >= 0");
  if (h->t + (uint64_t)n_sweeps > 4294967296ull)
    return fail(SMC_ERANGE, "sweep counter would exceed 2^32");
  return sweeps_impl(h, beta, n_sweeps, nullptr);
}

int smc_sweep_measure(smc_lattice* h, double beta, int64_t n_sweeps, void* dev_obs) {
  if (!h) return fail(SMC_EINVAL, "handle is NULL");
  if (!beta_ok(beta)) return fail(SMC_EINVAL, "beta must be >= 0 (or +inf), not NaN");
  if (n_sweeps < 0) return fail(SMC_EINVAL, "n_sweeps must be >= 0");
  if (!dev_obs || ((uintptr_t)dev_obs & 7)) return fail(SMC_EINVAL, "dev_obs must be 8-byte aligned");
  if (h->t + (uint64_t)n_sweeps > 4294967296ull)
    return fail(SMC_ERANGE, "sweep counter would exceed 2^32");
  if (n_sweeps == 0)
    return check(measure_any(h, h->t, dev_obs),
                 "measurement launch");
  return sweeps_impl(h, beta, n_sweeps, dev_obs);
}

int smc_half_sweep(smc_lattice* h, double beta, int colour) {
  if (!h) return fail(SMC_EINVAL, "handle is NULL");
  if (!beta_ok(beta)) return fail(SMC_EINVAL, "beta must be >= 0 (or +inf), not NaN");
  if (colour != 0 && colour != 1) return fail(SMC_EINVAL, "colour must be 0 or 1");
  if (h->p.tile > 0) return fail(SMC_ESTATE, "half-sweeps are not defined for the tiled schedule");
  if (h->t > 0xffffffffull) return fail(SMC_ERANGE, "sweep counter exceeds 2^32 - 1");
  return half_sweep_impl(h, beta, (uint32_t)h->t, (uint32_t)colour);
}

int smc_measure_async(smc_lattice* h, void* dev_obs) {
  if (!h) return fail(SMC_EINVAL, "handle is NULL");
  if (!dev_obs || ((uintptr_t)dev_obs & 7)) return fail(SMC_EINVAL, "dev_obs must be 8-byte aligned");
  return check(measure_any(h, h->t, dev_obs),
               "measurement launch");
}

int smc_measure_noalloc(const smc_params* p, const void* spins, const void* J, int64_t sweep,
                        void* dev_obs, void* stream) {
  g_err.clear();
  std::string why;
  if (!params_ok(p, why)) return fail(SMC_EINVAL, why);
  if (!spins || ((uintptr_t)spins & 15)) return fail(SMC_EINVAL, "spins must be non-NULL and 16-byte aligned");
  if (p->J_kind != SMC_J_UNIFORM && (!J || ((uintptr_t)J & 15)))
    return fail(SMC_EINVAL, "J must be non-NULL and 16-byte aligned for PM / FP32 couplings");
  if (!dev_obs || ((uintptr_t)dev_obs & 7)) return fail(SMC_EINVAL, "dev_obs must be 8-byte aligned");
  const Geom g = make_geom(p);
  const int64_t need = measure_partials_standalone(g, is_packed(p));
  if (need > kMeasureScratchPartials)
    return fail(SMC_EINVAL, "lattice too large for the allocation-free measurement: it needs " +
                                std::to_string(need) + " reduction partials, the library's scratch holds " +
                                std::to_string(kMeasureScratchPartials) +
                                " (packed spins: N/2 <= 2^27 sites); use smc_measure_async");
  void* scr = nullptr;
  const int rc = check(measure_scratch(&scr), "measurement scratch address");
  if (rc != SMC_OK) return rc;
  return check(measure_state(*p, g, spins, J, scr, sweep, dev_obs, (hipStream_t)stream),
               "measurement launch");
}

int smc_probe(int32_t kind, uint32_t n_lanes, uint32_t reps, void* dev_out, void* stream) {
  g_err.clear();
  if (kind != 0 && kind != 1) return fail(SMC_EINVAL, "kind must be 0 (Philox) or 1 (VALU)");
  if (n_lanes == 0 || n_lanes % 256) return fail(SMC_EINVAL, "n_lanes must be a positive multiple of 256");
  if (!dev_out || ((uintptr_t)dev_out & 3)) return fail(SMC_EINVAL, "out must be 4-byte aligned");
  return check(launch_probe(kind, n_lanes, reps, (uint32_t*)dev_out, (hipStream_t)stream),
               "probe launch");
}

int smc_measure(smc_lattice* h, smc_obs* out) {
  if (!h) return fail(SMC_EINVAL, "handle is NULL");
  if (!out) return fail(SMC_EINVAL, "out is NULL");
  int rc = smc_measure_async(h, h->obs_slot);
  if (rc != SMC_OK) return rc;
  smc_obs tmp;
  rc = check(hipMemcpyAsync(&tmp, h->obs_slot, sizeof(smc_obs), hipMemcpyDeviceToHost, h->stream),
             "observable copy");
  if (rc != SMC_OK) return rc;
  rc = check(hipStreamSynchronize(h->stream), "stream synchronise");
  if (rc != SMC_OK) return rc;
  *out = tmp;
  return SMC_OK;
}

int smc_bond_correlations(smc_lattice* h, int op, void* acc, void* out_mean) {
  if (!h) return fail(SMC_EINVAL, "handle is NULL");
  if (is_packed(&h->p)) return fail(SMC_ESTATE, "bond correlations are not available for packed spins");
  if (!acc || ((uintptr_t)acc & 7)) return fail(SMC_EINVAL, "acc must be non-NULL and 8-byte aligned");
  const MeasureLaunch m = measure_args(h, h->t);
  switch (op) {
    case SMC_BOND_RESET:
      h->samples = 0;
      return check(launch_fill_zero(acc, smc_bond_bytes(&h->p), h->stream), "bond reset launch");
    case SMC_BOND_ACCUMULATE: {
      const int rc = check(launch_bond_accumulate(m, h->spins, acc, h->stream), "bond accumulate launch");
      if (rc == SMC_OK) h->samples += 1;
      return rc;
    }
    case SMC_BOND_READ:
      if (!out_mean || ((uintptr_t)out_mean & 7))
        return fail(SMC_EINVAL, "out_mean must be non-NULL and 8-byte aligned");
      return check(launch_bond_mean(m, acc, h->samples, (double*)out_mean, h->stream),
                   "bond mean launch");
    default:
      return fail(SMC_EINVAL, "op must be RESET, ACCUMULATE or READ");
  }
}

int smc_get_samples(const smc_lattice* h, int64_t* samples) {
  if (!h || !samples) return fail(SMC_EINVAL, "NULL argument");
  *samples = h->samples;
  return SMC_OK;
}

int smc_set_samples(smc_lattice* h, int64_t samples) {
  if (!h || samples < 0) return fail(SMC_EINVAL, "bad argument");
  h->samples = samples;
  return SMC_OK;
}

int smc_renormalize(smc_lattice* h) {
  if (!h) return fail(SMC_EINVAL, "handle is NULL");
  if (h->p.n == 1) return SMC_OK;
  return check(launch_renormalize(h->g, h->p.n, (float*)h->spins, h->stream), "renormalisation launch");
}

int smc_validate(smc_lattice* h) {
  if (!h) return fail(SMC_EINVAL, "handle is NULL");
  if (is_packed(&h->p)) return SMC_OK;  // every bit pattern is a valid state
  int rc = check(launch_fill_zero(h->counter, 4, h->stream), "counter reset");
  if (rc != SMC_OK) return rc;
  rc = check(launch_validate(measure_args(h, h->t), h->spins, h->counter, h->stream), "validate launch");
  if (rc != SMC_OK) return rc;
  uint32_t bad = 0;
  rc = check(hipMemcpyAsync(&bad, h->counter, 4, hipMemcpyDeviceToHost, h->stream), "counter copy");
  if (rc != SMC_OK) return rc;
  rc = check(hipStreamSynchronize(h->stream), "stream synchronise");
  if (rc != SMC_OK) return rc;
  if (bad) return fail(SMC_ESTATE, std::to_string(bad) + " spins or couplings out of range");
  return SMC_OK;
}

int smc_get_sweep_index(const smc_lattice* h, uint64_t* t) {
  if (!h || !t) return fail(SMC_EINVAL, "NULL argument");
  *t = h->t;
  return SMC_OK;
}

int smc_set_sweep_index(smc_lattice* h, uint64_t t) {
  if (!h) return fail(SMC_EINVAL, "handle is NULL");
  if (t > 4294967296ull) return fail(SMC_ERANGE, "sweep index must be <= 2^32");
  h->t = t;
  return SMC_OK;
}

const char* smc_kernel_name(const smc_lattice* h, uint32_t* rows_per_band) {
  if (rows_per_band) *rows_per_band = 0;
  if (!h) return "";
  if (h->p.n > 1) {
    const ContLaunch a = cont_args(h, 0.0);
    const bool stream = cont_variant_used(a) == kContStream;
    if (stream && rows_per_band) *rows_per_band = h->cont_rows;
    if (h->p.n == 2) return stream ? "xy_stream" : "xy_site";
    return stream ? "heisenberg_stream" : "heisenberg_site";
  }
  if (is_packed(&h->p)) {
    if (rows_per_band) *rows_per_band = h->packed_rows;
    return "ising_packed";
  }
  if (h->p.tile > 0) {
    if (rows_per_band) *rows_per_band = (uint32_t)h->p.tile;
    const bool hb = (h->p.flags & SMC_FLAG_HEATBATH) != 0;
    return h->tile_packed && tile_packed_supported(h->g, (uint32_t)h->p.tile, hb) ? "ising_tiles_packed"
                                                                                : "ising_tiles";
  }
  if (h->use_fused) {
    if (rows_per_band) *rows_per_band = h->fused_rows;
    return "ising_fused";
  }
  IsingLaunch a;
  std::memset(&a, 0, sizeof(a));
  a.g = h->g;
  a.J_kind = h->p.J_kind;
  a.variant = (h->p.flags & SMC_FLAG_GENERIC_KERNEL) ? kVariantSite : h->ising_variant;
  a.rows_per_band = h->rows_per_band;
  a.heatbath = (h->p.flags & SMC_FLAG_HEATBATH) ? 1 : 0;
  switch (ising_variant_used(a)) {
    case kVariantStream:
      if (rows_per_band) *rows_per_band = h->rows_per_band;
      return "ising_stream";
    case kVariantChunk: return "ising_chunk";
    default: return "ising_site";
  }
}

int smc_destroy(smc_lattice* h) {
  delete h;
  return SMC_OK;
}

int smc_pack_spins(const void* src, void* dst, int64_t n_sites, void* stream) {
  if (n_sites < 0 || n_sites % 32) return fail(SMC_EINVAL, "n_sites must be a non-negative multiple of 32");
  if (n_sites && (!src || !dst || ((uintptr_t)src & 15) || ((uintptr_t)dst & 3)))
    return fail(SMC_EINVAL, "src must be 16-byte and dst 4-byte aligned");
  return check(launch_pack((const int8_t*)src, (uint32_t*)dst, n_sites / 32, (hipStream_t)stream),
               "pack launch");
}

int smc_unpack_spins(const void* src, void* dst, int64_t n_sites, void* stream) {
  if (n_sites < 0 || n_sites % 32) return fail(SMC_EINVAL, "n_sites must be a non-negative multiple of 32");
  if (n_sites && (!src || !dst || ((uintptr_t)src & 3) || ((uintptr_t)dst & 15)))
    return fail(SMC_EINVAL, "src must be 4-byte and dst 16-byte aligned");
  return check(launch_unpack((const uint32_t*)src, (int8_t*)dst, n_sites / 32, (hipStream_t)stream),
               "unpack launch");
}

const char* smc_last_error(void) { return g_err.c_str(); }

const char* smc_version(void) { return "libsmc 0.1 (gfx950)"; }

}  // extern "C"

// ===========================================================================
// Batches
// ===========================================================================
struct smc_batch {
  int d, J_kind;
  uint64_t seed;
  double J0;
  int32_t n;
  std::vector<int32_t> L;
  std::vector<uint32_t> Lu;  // the edges as unsigned (LDS sizing)
  bool packed;               // lattices may take the packed path (SMC_BATCH_PACKED=0 disables)
  std::vector<int64_t> soff, joff;
  std::vector<BatchDesc> desc;
  std::vector<uint32_t> orders;  // [largest first | as given]
  void* spins;
  void* J;
  hipStream_t stream;
  uint64_t t;
  BatchDesc* desc_dev;
  uint32_t* order_dev;
  void* scratch;
  size_t spin_bytes, max_sites;
  uint32_t threads;
  bool largest_first;
  bool use_graph;
  hipGraph_t graph;
  hipGraphExec_t exec;
  hipGraphNode_t node;
  int64_t graph_n;
  uint32_t graph_every;
  void* graph_obs;
  uint32_t graph_threads;
  bool graph_largest;
};

namespace {

size_t round16(size_t v) { return (v + 15) / 16 * 16; }

bool batch_shape_ok(int32_t d, int32_t n, const int32_t* L, std::string& why) {
  if (d != 2 && d != 3) { why = "d must be 2 or 3"; return false; }
  if (n < 1 || !L) { why = "need n_lattices >= 1 and an edge array"; return false; }
  for (int32_t r = 0; r < n; ++r) {
    if (L[r] < 4 || (L[r] & 1)) { why = "every L must be even and >= 4"; return false; }
    const double N = std::pow((double)L[r], d);
    if (N > 65536.0) { why = "every lattice must have L^d <= 65536 sites"; return false; }
  }
  return true;
}

void batch_layout(int32_t d, int32_t n, const int32_t* L, std::vector<int64_t>& so,
                  std::vector<int64_t>& jo, size_t& sbytes, size_t& jbytes) {
  so.resize(n);
  jo.resize(n);
  size_t s = 0, j = 0;
  for (int32_t r = 0; r < n; ++r) {
    size_t N = 1;
    for (int k = 0; k < d; ++k) N *= (size_t)L[r];
    so[r] = (int64_t)s;
    jo[r] = (int64_t)j;
    s += round16(N);
    j += round16(N * d);
  }
  sbytes = s;
  jbytes = j;
}

size_t batch_ws_parts(int32_t d, int32_t n, const int32_t* L, size_t* desc_b, size_t* order_b,
                      size_t* scratch_b) {
  std::vector<int64_t> so, jo;
  size_t sb, jb;
  batch_layout(d, n, L, so, jo, sb, jb);
  *desc_b = round_up(sizeof(BatchDesc) * (size_t)n, kAlign);
  *order_b = round_up(sizeof(uint32_t) * 2 * (size_t)n, kAlign);
  *scratch_b = round_up(sb, kAlign);
  return *desc_b + *order_b + *scratch_b;
}

int batch_launch(smc_batch* b, int8_t* spins, uint32_t t0, uint32_t n_sweeps, uint32_t every,
                 void* dev_obs, uint32_t threads, bool largest_first) {
  BatchLaunch a;
  a.d = b->d;
  a.pm = b->J_kind == SMC_J_PM;
  a.n_lattices = (uint32_t)b->n;
  a.threads = threads;
  a.max_sites = b->max_sites;
  a.lds_bytes = batch_lds_bytes(b->d, b->J_kind == SMC_J_PM, b->packed, b->Lu.data(), (uint32_t)b->n,
                                threads);
  a.descs = b->desc_dev;
  a.order = b->order_dev + (largest_first ? 0 : b->n);
  a.key = RngKey{(uint32_t)(b->seed & 0xffffffffu), (uint32_t)(b->seed >> 32), 0u};
  return check(launch_batch(a, spins, (const int8_t*)b->J, t0, n_sweeps, every, dev_obs, b->stream),
               "batch sweep launch");
}

void batch_drop_graph(smc_batch* b) {
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  b->exec = nullptr;
  b->graph = nullptr;
  b->node = nullptr;
}

// One graph node holding the batch kernel; its arguments are refreshed in
// the instantiated graph before every replay.
int batch_graph_sweep(smc_batch* b, uint32_t n_sweeps, uint32_t every, void* dev_obs) {
  const BatchDesc* descs = b->desc_dev;
  const uint32_t* order = b->order_dev + (b->largest_first ? 0 : b->n);
  RngKey key{(uint32_t)(b->seed & 0xffffffffu), (uint32_t)(b->seed >> 32), 0u};
  int8_t* spins = (int8_t*)b->spins;
  const int8_t* J = (const int8_t*)b->J;
  uint32_t t0 = (uint32_t)b->t;
  void* obs = dev_obs;
  uint32_t nl = (uint32_t)b->n;
  void* args[] = {&descs, &order, &key, &spins, &J, &t0, &n_sweeps, &every, &nl, &obs};
  hipKernelNodeParams kp;
  std::memset(&kp, 0, sizeof(kp));
  kp.func = const_cast<void*>(batch_kernel_fn(b->d, b->J_kind == SMC_J_PM, dev_obs != nullptr));
  kp.gridDim = dim3((unsigned)b->n);
  kp.blockDim = dim3(b->threads);
  kp.sharedMemBytes =
      (unsigned)batch_lds_bytes(b->d, b->J_kind == SMC_J_PM, b->packed, b->Lu.data(), (uint32_t)b->n,
                                b->threads);
  kp.kernelParams = args;
  kp.extra = nullptr;
  const bool same = b->exec && b->graph_n == (int64_t)n_sweeps && b->graph_obs == dev_obs &&
                    b->graph_every == every &&
                    b->graph_threads == b->threads && b->graph_largest == b->largest_first;
  if (!same) {
    batch_drop_graph(b);
    int rc = check(hipGraphCreate(&b->graph, 0), "graph create");
    if (rc != SMC_OK) return rc;
    rc = check(hipGraphAddKernelNode(&b->node, b->graph, nullptr, 0, &kp), "graph kernel node");
    if (rc != SMC_OK) return rc;
    rc = check(hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0), "graph instantiate");
    if (rc != SMC_OK) return rc;
    b->graph_n = n_sweeps;
    b->graph_every = every;
    b->graph_obs = dev_obs;
    b->graph_threads = b->threads;
    b->graph_largest = b->largest_first;
  } else {
    const int rc = check(hipGraphExecKernelNodeSetParams(b->exec, b->node, &kp), "graph node update");
    if (rc != SMC_OK) return rc;
  }
  return check(hipGraphLaunch(b->exec, b->stream), "graph launch");
}

}  // namespace

extern "C" {

size_t smc_batch_spin_bytes(int32_t d, int32_t n, const int32_t* L) {
  std::string why;
  if (!batch_shape_ok(d, n, L, why)) return 0;
  std::vector<int64_t> so, jo;
  size_t sb, jb;
  batch_layout(d, n, L, so, jo, sb, jb);
  return sb;
}

size_t smc_batch_coupling_bytes(int32_t d, int32_t n, const int32_t* L) {
  std::string why;
  if (!batch_shape_ok(d, n, L, why)) return 0;
  std::vector<int64_t> so, jo;
  size_t sb, jb;
  batch_layout(d, n, L, so, jo, sb, jb);
  return jb;
}

size_t smc_batch_workspace_bytes(int32_t d, int32_t n, const int32_t* L) {
  std::string why;
  if (!batch_shape_ok(d, n, L, why)) return 0;
  size_t a, o, s;
  return batch_ws_parts(d, n, L, &a, &o, &s);
}

int smc_batch_offsets(int32_t d, int32_t n, const int32_t* L, int64_t* spin_offsets,
                      int64_t* coupling_offsets) {
  std::string why;
  if (!batch_shape_ok(d, n, L, why)) return fail(SMC_EINVAL, why);
  std::vector<int64_t> so, jo;
  size_t sb, jb;
  batch_layout(d, n, L, so, jo, sb, jb);
  for (int32_t r = 0; r < n; ++r) {
    if (spin_offsets) spin_offsets[r] = so[r];
    if (coupling_offsets) coupling_offsets[r] = jo[r];
  }
  return SMC_OK;
}

int smc_batch_init(smc_batch** out, int32_t d, int32_t J_kind, uint64_t seed, double J0,
                   int32_t init, int32_t couplings_keep, int32_t n, const int32_t* L,
                   const double* beta, const uint32_t* replica, void* spins, void* J,
                   void* workspace, size_t workspace_bytes, void* stream) {
  g_err.clear();
  if (!out) return fail(SMC_EINVAL, "out is NULL");
  *out = nullptr;
  std::string why;
  if (!batch_shape_ok(d, n, L, why)) return fail(SMC_EINVAL, why);
  if (J_kind != SMC_J_UNIFORM && J_kind != SMC_J_PM)
    return fail(SMC_EINVAL, "batches take uniform or +-1 couplings");
  if (!std::isfinite(J0)) return fail(SMC_EINVAL, "J0 must be finite");
  if (init < 0 || init > 2) return fail(SMC_EINVAL, "init must be HOT, COLD or KEEP");
  if (!beta) return fail(SMC_EINVAL, "beta array is NULL");
  for (int32_t r = 0; r < n; ++r)
    if (!beta_ok(beta[r])) return fail(SMC_EINVAL, "every beta must be >= 0 (or +inf), not NaN");
  if (!spins || ((uintptr_t)spins & 15)) return fail(SMC_EINVAL, "spins must be 16-byte aligned");
  if (J_kind == SMC_J_PM && (!J || ((uintptr_t)J & 15)))
    return fail(SMC_EINVAL, "J must be non-NULL and 16-byte aligned for +-1 couplings");
  size_t desc_b, order_b, scratch_b;
  const size_t need = batch_ws_parts(d, n, L, &desc_b, &order_b, &scratch_b);
  if (!workspace || ((uintptr_t)workspace & (kAlign - 1)))
    return fail(SMC_EINVAL, "workspace must be non-NULL and 256-byte aligned");
  if (workspace_bytes < need)
    return fail(SMC_EINVAL, "workspace too small: need " + std::to_string(need) + " bytes");
  smc_batch* b = new (std::nothrow) smc_batch();
  if (!b) return fail(SMC_EINVAL, "out of host memory");
  b->d = d;
  b->J_kind = J_kind;
  b->seed = seed;
  b->J0 = J0;
  b->n = n;
  b->L.assign(L, L + n);
  b->Lu.assign(L, L + n);
  b->packed = true;
  if (const char* v = std::getenv("SMC_BATCH_PACKED"))
    if (std::string(v) == "0") b->packed = false;
  size_t jb;
  batch_layout(d, n, L, b->soff, b->joff, b->spin_bytes, jb);
  b->spins = spins;
  b->J = J_kind == SMC_J_PM ? J : nullptr;
  b->stream = (hipStream_t)stream;
  b->t = 0;
  b->desc_dev = (BatchDesc*)workspace;
  b->order_dev = (uint32_t*)((char*)workspace + desc_b);
  b->scratch = (char*)workspace + desc_b + order_b;
  b->threads = 256;
  b->largest_first = true;
  b->use_graph = false;
  b->graph = nullptr;
  b->exec = nullptr;
  b->node = nullptr;
  b->graph_n = -1;
  b->graph_every = 0;
  b->graph_obs = nullptr;
  b->max_sites = 0;
  b->desc.resize(n);
  for (int32_t r = 0; r < n; ++r) {
    BatchDesc& x = b->desc[r];
    std::memset(&x, 0, sizeof(x));
    const uint32_t Lr = (uint32_t)L[r];
    size_t N = 1;
    for (int k = 0; k < d; ++k) N *= Lr;
    b->max_sites = std::max(b->max_sites, N);
    x.L = Lr;
    x.R = Lr / 2;
    x.Nh = (uint32_t)(N / 2);
    x.replica = replica ? replica[r] : (uint32_t)r;
    const FastDiv dr = make_fastdiv(x.R), dl = make_fastdiv(Lr);
    x.divR_m = dr.m;
    x.divR_s = dr.s;
    x.divL_m = dl.m;
    x.divL_s = dl.s;
    const IsingTable tab = make_table(d, J0, beta[r]);
    x.th_lo = tab.th_lo;
    x.th_hi = tab.th_hi;
    x.al_lo = tab.al_lo;
    x.al_hi = tab.al_hi;
    for (int k = 0; k < 7; ++k) x.frac[k] = tab.frac[k];
    x.spin_off_lo = (uint32_t)((uint64_t)b->soff[r] & 0xffffffffu);
    x.spin_off_hi = (uint32_t)((uint64_t)b->soff[r] >> 32);
    x.J_off_lo = (uint32_t)((uint64_t)b->joff[r] & 0xffffffffu);
    x.J_off_hi = (uint32_t)((uint64_t)b->joff[r] >> 32);
    x.J0 = J0;
    x.packed = b->packed ? 1u : 0u;
  }
  std::vector<uint32_t> idx(n);
  std::iota(idx.begin(), idx.end(), 0u);
  std::vector<uint32_t> largest = idx;
  std::stable_sort(largest.begin(), largest.end(),
                   [&](uint32_t a, uint32_t c) { return b->desc[a].Nh > b->desc[c].Nh; });
  b->orders = largest;
  b->orders.insert(b->orders.end(), idx.begin(), idx.end());
  // the largest workgroup (1024 lanes) with the largest lattice may pass the
  // default 64 KiB of dynamic LDS
  size_t lds_max = 0;
  for (uint32_t th = 64; th <= 1024; th *= 2)
    lds_max = std::max(lds_max, batch_lds_bytes(d, J_kind == SMC_J_PM, b->packed, b->Lu.data(),
                                                (uint32_t)n, th));
  int rc = check(batch_allow_lds(lds_max), "batch LDS attribute");
  if (rc == SMC_OK)
    rc = check(hipMemcpyAsync(b->desc_dev, b->desc.data(), sizeof(BatchDesc) * n,
                              hipMemcpyHostToDevice, b->stream), "descriptor upload");
  if (rc == SMC_OK)
    rc = check(hipMemcpyAsync(b->order_dev, b->orders.data(), sizeof(uint32_t) * 2 * n,
                              hipMemcpyHostToDevice, b->stream), "schedule upload");
  for (int32_t r = 0; rc == SMC_OK && r < n; ++r) {
    smc_params p;
    std::memset(&p, 0, sizeof(p));
    p.d = d;
    p.n = 1;
    p.L = L[r];
    const Geom g = make_geom(&p);
    const RngKey key{(uint32_t)(seed & 0xffffffffu), (uint32_t)(seed >> 32), b->desc[r].replica};
    if (J_kind == SMC_J_PM && !couplings_keep)
      rc = check(launch_init_couplings(g, SMC_J_PM, key, J0, 0.0, (int8_t*)J + b->joff[r], b->stream),
                 "coupling init launch");
    if (rc == SMC_OK && init != SMC_INIT_KEEP)
      rc = check(launch_init_ising(g, key, init == SMC_INIT_HOT, (int8_t*)spins + b->soff[r], b->stream),
                 "spin init launch");
  }
  if (rc == SMC_OK) rc = check(hipStreamSynchronize(b->stream), "stream synchronise");
  if (rc != SMC_OK) {
    delete b;
    return rc;
  }
  *out = b;
  return SMC_OK;
}

int smc_batch_sweep_series(smc_batch* b, int64_t n_sweeps, int64_t measure_every, void* dev_obs) {
  if (!b) return fail(SMC_EINVAL, "handle is NULL");
  if (n_sweeps < 0) return fail(SMC_EINVAL, "n_sweeps must be >= 0");
  if (dev_obs && ((uintptr_t)dev_obs & 7)) return fail(SMC_EINVAL, "dev_obs must be 8-byte aligned");
  if (dev_obs && n_sweeps > 0 && (measure_every < 1 || n_sweeps % measure_every != 0))
    return fail(SMC_EINVAL, "measure_every must be >= 1 and divide n_sweeps");
  if (b->t + (uint64_t)n_sweeps > 4294967296ull)
    return fail(SMC_ERANGE, "sweep counter would exceed 2^32");
  if (n_sweeps == 0 && !dev_obs) return SMC_OK;
  const uint32_t every = dev_obs && n_sweeps > 0 ? (uint32_t)measure_every : 1u;
  int rc;
  if (b->use_graph)
    rc = batch_graph_sweep(b, (uint32_t)n_sweeps, every, dev_obs);
  else
    rc = batch_launch(b, (int8_t*)b->spins, (uint32_t)b->t, (uint32_t)n_sweeps, every, dev_obs,
                      b->threads, b->largest_first);
  if (rc == SMC_OK) b->t += (uint64_t)n_sweeps;
  return rc;
}

int smc_batch_sweep(smc_batch* b, int64_t n_sweeps, void* dev_obs) {
  return smc_batch_sweep_series(b, n_sweeps, n_sweeps > 0 ? n_sweeps : 1, dev_obs);
}

// Upload the descriptor table with every lattice's packed-path flag set to
// b->packed.
static int batch_upload_desc(smc_batch* b) {
  for (auto& x : b->desc) x.packed = b->packed ? 1u : 0u;
  return check(hipMemcpyAsync(b->desc_dev, b->desc.data(), sizeof(BatchDesc) * b->desc.size(),
                              hipMemcpyHostToDevice, b->stream), "descriptor upload");
}

int smc_batch_autotune(smc_batch* b, int32_t* threads_out, int32_t* largest_first_out) {
  if (!b) return fail(SMC_EINVAL, "handle is NULL");
  // the cache key: shape of the batch (edges in order) and the device
  uint64_t hsh = 1469598103934665603ull;
  for (int32_t r = 0; r < b->n; ++r) hsh = (hsh ^ (uint64_t)b->L[r]) * 1099511628211ull;
  char hx[24];
  std::snprintf(hx, sizeof(hx), "%016llx", (unsigned long long)hsh);
  const std::string key = "batch:d" + std::to_string(b->d) + ":J" + std::to_string(b->J_kind) +
                          ":n" + std::to_string(b->n) + ":L" + hx + ":" + device_tag();
  const bool packed_allowed = b->packed;
  std::string cached;
  if (cache_get(key, cached)) {
    unsigned th = 0;
    int lf = 0, pk = 0;
    if (std::sscanf(cached.c_str(), "%u,%d,%d", &th, &lf, &pk) == 3 && th >= 64 && th <= 1024 &&
        th % 64 == 0) {
      b->threads = th;
      b->largest_first = lf != 0;
      b->packed = packed_allowed && pk != 0;
      const int rc = batch_upload_desc(b);
      if (rc != SMC_OK) return rc;
      if (threads_out) *threads_out = (int32_t)th;
      if (largest_first_out) *largest_first_out = lf != 0 ? 1 : 0;
      return SMC_OK;
    }
  }
  int rc = check(hipMemcpyAsync(b->scratch, b->spins, b->spin_bytes, hipMemcpyDeviceToDevice,
                                b->stream), "scratch copy");
  if (rc != SMC_OK) return rc;
  hipEvent_t e0, e1;
  if ((rc = check(hipEventCreate(&e0), "event create")) != SMC_OK) return rc;
  if ((rc = check(hipEventCreate(&e1), "event create")) != SMC_OK) {
    (void)hipEventDestroy(e0);
    return rc;
  }
  // workgroup size x lattice order x path (one bit per site where a lattice
  // allows it, or one byte per site throughout), each timed over 8 sweeps in
  // turn for three rounds after a warm-up, ranked by the median (the chain on
  // the scratch copy is discarded: any counter will do)
  const uint32_t cand[5] = {64, 128, 256, 512, 1024};
  struct Cand { uint32_t threads; bool largest, packed; std::vector<float> ms; };
  std::vector<Cand> cands;
  for (int pk = packed_allowed ? 1 : 0; pk >= 0; --pk)
    for (int lf = 1; lf >= 0; --lf)
      for (int c = 0; c < 5; ++c) cands.push_back(Cand{cand[c], lf != 0, pk != 0, {}});
  rc = batch_launch(b, (int8_t*)b->scratch, (uint32_t)b->t, 16, 1, nullptr, b->threads, b->largest_first);
  for (int round = 0; round < 3 && rc == SMC_OK; ++round) {
    for (size_t i = 0; i < cands.size() && rc == SMC_OK; ++i) {
      Cand& x = cands[i];
      if (b->packed != x.packed || i == 0) {
        b->packed = x.packed;
        rc = batch_upload_desc(b);
        if (rc != SMC_OK) break;
      }
      rc = batch_launch(b, (int8_t*)b->scratch, (uint32_t)b->t, 1, 1, nullptr, x.threads, x.largest);
      if (rc == SMC_OK) rc = check(hipEventRecord(e0, b->stream), "event record");
      if (rc == SMC_OK)
        rc = batch_launch(b, (int8_t*)b->scratch, (uint32_t)b->t, 8, 1, nullptr, x.threads, x.largest);
      if (rc == SMC_OK) rc = check(hipEventRecord(e1, b->stream), "event record");
      if (rc == SMC_OK) rc = check(hipEventSynchronize(e1), "event synchronise");
      float ms = 0.0f;
      if (rc == SMC_OK) rc = check(hipEventElapsedTime(&ms, e0, e1), "event time");
      if (rc == SMC_OK) x.ms.push_back(ms);
    }
  }
  float best = 1e30f;
  uint32_t best_threads = b->threads;
  bool best_largest = b->largest_first;
  bool best_packed = packed_allowed;
  for (auto& x : cands) {
    if (x.ms.empty()) continue;
    std::sort(x.ms.begin(), x.ms.end());
    const float m = x.ms[x.ms.size() / 2];
    if (m < best) {
      best = m;
      best_threads = x.threads;
      best_largest = x.largest;
      best_packed = x.packed;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  b->packed = best_packed;
  if (rc == SMC_OK) rc = batch_upload_desc(b);
  if (rc != SMC_OK) return rc;
  b->threads = best_threads;
  b->largest_first = best_largest;
  cache_put(key, std::to_string(best_threads) + "," + (best_largest ? "1" : "0") + "," +
                     (best_packed ? "1" : "0"));
  if (threads_out) *threads_out = (int32_t)best_threads;
  if (largest_first_out) *largest_first_out = best_largest ? 1 : 0;
  return SMC_OK;
}

int smc_batch_set_schedule(smc_batch* b, int32_t threads, int32_t largest_first) {
  if (!b) return fail(SMC_EINVAL, "handle is NULL");
  if (threads < 64 || threads > 1024 || threads % 64)
    return fail(SMC_EINVAL, "threads must be a multiple of 64 in [64, 1024]");
  b->threads = (uint32_t)threads;
  b->largest_first = largest_first != 0;
  return SMC_OK;
}

int smc_batch_get_schedule(const smc_batch* b, int32_t* threads, int32_t* largest_first) {
  if (!b) return fail(SMC_EINVAL, "handle is NULL");
  if (threads) *threads = (int32_t)b->threads;
  if (largest_first) *largest_first = b->largest_first ? 1 : 0;
  return SMC_OK;
}

int smc_batch_lattice_packed(const smc_batch* b, int32_t r) {
  if (!b) return fail(SMC_EINVAL, "handle is NULL");
  if (r < 0 || r >= b->n) return fail(SMC_EINVAL, "lattice index out of range");
  return b->packed && batch_lattice_packed(b->d, (uint32_t)b->L[r], b->threads) ? 1 : 0;
}

int smc_batch_use_graph(smc_batch* b, int32_t enable) {
  if (!b) return fail(SMC_EINVAL, "handle is NULL");
  b->use_graph = enable != 0;
  if (!b->use_graph) batch_drop_graph(b);
  return SMC_OK;
}

int smc_batch_get_sweep_index(const smc_batch* b, uint64_t* t) {
  if (!b || !t) return fail(SMC_EINVAL, "NULL argument");
  *t = b->t;
  return SMC_OK;
}

int smc_batch_set_sweep_index(smc_batch* b, uint64_t t) {
  if (!b) return fail(SMC_EINVAL, "handle is NULL");
  if (t > 4294967296ull) return fail(SMC_ERANGE, "sweep index must be <= 2^32");
  b->t = t;
  return SMC_OK;
}

int smc_batch_destroy(smc_batch* b) {
  if (b) batch_drop_graph(b);
  delete b;
  return SMC_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Chains of one small lattice with shared FP32 couplings (derivatives of ln Z)
// ---------------------------------------------------------------------------
struct smc_chains {
  int d, L;
  int32_t n_chains;
  Geom g;
  RngKey key;  // replica = replica of chain 0
  const float* J;
  void* spins;
  double* part;   // [n_chains][d N] covariance partials
  double* gpart;  // [n_chains][2]
  hipStream_t stream;
  uint64_t t;
  int pair_kernel;  // the register-resident pair kernel (SMC_CHAINS_KERNEL=lds forces the other)
};

namespace {

bool chains_shape_ok(int32_t d, int32_t L, int32_t n_chains, std::string& why) {
  if (d != 2 && d != 3) return why = "d must be 2 or 3", false;
  if (L < 4 || L > 1024) return why = "L must be in [4, 1024]", false;
  if (d == 2 ? (L % 4) : (L % 2)) return why = d == 2 ? "L must be a multiple of 4" : "L must be even", false;
  if (n_chains < 1 || n_chains > (1 << 20)) return why = "n_chains must be in [1, 2^20]", false;
  smc_params p;
  std::memset(&p, 0, sizeof(p));
  p.d = d;
  p.n = 1;
  p.L = L;
  const Geom g = make_geom(&p);
  if (chains_lds_bytes(g, 1) > 160 * 1024)
    return why = "lattice too large for one workgroup's LDS (L^d (1 + 8 d) bytes > 160 KiB)", false;
  return true;
}

size_t chains_sites(int32_t d, int32_t L) {
  size_t N = 1;
  for (int k = 0; k < d; ++k) N *= (size_t)L;
  return N;
}

ChainsLaunch chains_args(const smc_chains* h, double beta) {
  ChainsLaunch a;
  a.g = h->g;
  a.key = h->key;
  a.J = h->J;
  a.beta = (float)beta;
  a.n_chains = (uint32_t)h->n_chains;
  a.divR = make_fastdiv((uint32_t)h->g.R);
  a.divL = make_fastdiv((uint32_t)h->g.L);
  a.pair_kernel = h->pair_kernel;
  return a;
}

bool al8(const void* p) { return p && !((uintptr_t)p & 7); }
bool al4(const void* p) { return p && !((uintptr_t)p & 3); }

}  // namespace

extern "C" {

size_t smc_chains_spin_bytes(int32_t d, int32_t L, int32_t n_chains) {
  std::string why;
  if (!chains_shape_ok(d, L, n_chains, why)) return 0;
  return chains_sites(d, L) * (size_t)n_chains;
}

size_t smc_chains_coupling_bytes(int32_t d, int32_t L) {
  std::string why;
  if (!chains_shape_ok(d, L, 1, why)) return 0;
  return chains_sites(d, L) * (size_t)d * sizeof(float);
}

size_t smc_chains_bond_bytes(int32_t d, int32_t L) {
  std::string why;
  if (!chains_shape_ok(d, L, 1, why)) return 0;
  return chains_sites(d, L) * (size_t)d * 8;
}

size_t smc_chains_workspace_bytes(int32_t d, int32_t L, int32_t n_chains) {
  std::string why;
  if (!chains_shape_ok(d, L, n_chains, why)) return 0;
  return round_up((size_t)n_chains * chains_sites(d, L) * d * sizeof(double), kAlign) +
         round_up((size_t)n_chains * 2 * sizeof(double), kAlign);
}

int smc_chains_init(smc_chains** out, int32_t d, int32_t L, int32_t n_chains, uint64_t seed,
                    uint32_t replica0, int32_t init, const float* J, void* spins,
                    void* workspace, size_t workspace_bytes, void* stream) {
  g_err.clear();
  if (!out) return fail(SMC_EINVAL, "out is NULL");
  *out = nullptr;
  std::string why;
  if (!chains_shape_ok(d, L, n_chains, why)) return fail(SMC_EINVAL, why);
  if (init < 0 || init > 2) return fail(SMC_EINVAL, "init must be HOT, COLD or KEEP");
  if (!J || ((uintptr_t)J & 3)) return fail(SMC_EINVAL, "J must be non-NULL and 4-byte aligned");
  if (!spins || ((uintptr_t)spins & 15)) return fail(SMC_EINVAL, "spins must be 16-byte aligned");
  if ((uint64_t)replica0 + (uint64_t)n_chains > 4294967296ull)
    return fail(SMC_EINVAL, "replica0 + n_chains must not exceed 2^32");
  const size_t need = smc_chains_workspace_bytes(d, L, n_chains);
  if (!workspace || ((uintptr_t)workspace & (kAlign - 1)))
    return fail(SMC_EINVAL, "workspace must be non-NULL and 256-byte aligned");
  if (workspace_bytes < need)
    return fail(SMC_EINVAL, "workspace too small: need " + std::to_string(need) + " bytes");
  smc_chains* h = new (std::nothrow) smc_chains();
  if (!h) return fail(SMC_EINVAL, "out of host memory");
  smc_params p;
  std::memset(&p, 0, sizeof(p));
  p.d = d;
  p.n = 1;
  p.L = L;
  h->d = d;
  h->L = L;
  h->n_chains = n_chains;
  h->g = make_geom(&p);
  h->key = RngKey{(uint32_t)(seed & 0xffffffffu), (uint32_t)(seed >> 32), replica0};
  h->J = J;
  h->spins = spins;
  h->part = (double*)workspace;
  h->gpart = (double*)((char*)workspace +
                       round_up((size_t)n_chains * chains_sites(d, L) * d * sizeof(double), kAlign));
  h->stream = (hipStream_t)stream;
  h->t = 0;
  h->pair_kernel = chains_pair_supported(h->g) ? 1 : 0;
  if (const char* v = std::getenv("SMC_CHAINS_KERNEL"))
    if (std::string(v) == "lds") h->pair_kernel = 0;
  int rc = check(chains_allow_lds(h->g), "chains LDS attribute");
  const size_t N = chains_sites(d, L);
  for (int32_t k = 0; rc == SMC_OK && init != SMC_INIT_KEEP && k < n_chains; ++k) {
    const RngKey key{h->key.k0, h->key.k1, replica0 + (uint32_t)k};
    rc = check(launch_init_ising(h->g, key, init == SMC_INIT_HOT, (int8_t*)spins + (size_t)k * N,
                                 h->stream),
               "spin init launch");
  }
  if (rc == SMC_OK) rc = check(hipStreamSynchronize(h->stream), "stream synchronise");
  if (rc != SMC_OK) {
    delete h;
    return rc;
  }
  *out = h;
  return SMC_OK;
}

int smc_chains_sample(smc_chains* h, double beta, int64_t n_sweeps, int64_t* dev_bond_sum) {
  if (!h) return fail(SMC_EINVAL, "handle is NULL");
  if (!beta_ok(beta)) return fail(SMC_EINVAL, "beta must be >= 0 (or +inf), not NaN");
  if (n_sweeps < 0) return fail(SMC_EINVAL, "n_sweeps must be >= 0");
  if (dev_bond_sum && ((uintptr_t)dev_bond_sum & 7))
    return fail(SMC_EINVAL, "bond_sum must be 8-byte aligned");
  if (h->t + (uint64_t)n_sweeps > 4294967296ull)
    return fail(SMC_ERANGE, "sweep counter would exceed 2^32");
  const ChainsLaunch a = chains_args(h, beta);
  int64_t left = n_sweeps;
  while (left > 0) {
    // int32 per-bond sums in LDS: at most 2^30 sweeps per launch
    const uint32_t n = (uint32_t)std::min<int64_t>(left, (int64_t)1 << 30);
    const int rc = check(launch_chains_sample(a, (int8_t*)h->spins, (uint32_t)h->t, n,
                                              dev_bond_sum, h->stream),
                         "chains sample launch");
    if (rc != SMC_OK) return rc;
    h->t += n;
    left -= n;
  }
  return SMC_OK;
}

int smc_chains_half_sweep(smc_chains* h, double beta, int colour) {
  if (!h) return fail(SMC_EINVAL, "handle is NULL");
  if (!beta_ok(beta)) return fail(SMC_EINVAL, "beta must be >= 0 (or +inf), not NaN");
  if (colour != 0 && colour != 1) return fail(SMC_EINVAL, "colour must be 0 or 1");
  if (h->t >= 4294967296ull) return fail(SMC_ERANGE, "sweep counter is past 2^32 - 1");
  return check(launch_chains_half_sweep(chains_args(h, beta), (int8_t*)h->spins, (uint32_t)h->t,
                                        colour, h->stream),
               "chains half-sweep launch");
}

const char* smc_chains_kernel_name(const smc_chains* h) {
  if (!h) return "";
  return h->pair_kernel ? "chains_pair" : "chains_lds";
}

int smc_chains_covariance(smc_chains* h, double beta, int64_t n_sweeps, const double* dev_g,
                          const double* dev_g_center, double* dev_cov_acc, double* dev_G_acc) {
  if (!h) return fail(SMC_EINVAL, "handle is NULL");
  if (!beta_ok(beta)) return fail(SMC_EINVAL, "beta must be >= 0 (or +inf), not NaN");
  if (n_sweeps < 0) return fail(SMC_EINVAL, "n_sweeps must be >= 0");
  if ((uintptr_t)dev_g_center & 7) return fail(SMC_EINVAL, "g_center must be 8-byte aligned (or NULL)");
  if (!dev_g || !dev_cov_acc || !dev_G_acc || ((uintptr_t)dev_g & 7) ||
      ((uintptr_t)dev_cov_acc & 7) || ((uintptr_t)dev_G_acc & 7))
    return fail(SMC_EINVAL, "g, cov_acc and G_acc must be non-NULL and 8-byte aligned");
  if (h->t + (uint64_t)n_sweeps > 4294967296ull)
    return fail(SMC_ERANGE, "sweep counter would exceed 2^32");
  if (n_sweeps == 0) return SMC_OK;
  const ChainsLaunch a = chains_args(h, beta);
  const int rc = check(launch_chains_covariance(a, (int8_t*)h->spins, (uint32_t)h->t,
                                                (uint32_t)n_sweeps, dev_g, dev_g_center, h->part,
                                                h->gpart, dev_cov_acc, dev_G_acc, h->stream),
                       "chains covariance launch");
  if (rc != SMC_OK) return rc;
  h->t += (uint64_t)n_sweeps;
  return SMC_OK;
}

int smc_chains_mean(smc_chains* h, const int64_t* dev_bond_sum, int64_t n_samples,
                    double* dev_mean) {
  if (!h) return fail(SMC_EINVAL, "handle is NULL");
  if (n_samples < 1) return fail(SMC_EINVAL, "n_samples must be >= 1");
  if (!al8(dev_bond_sum) || !al8(dev_mean))
    return fail(SMC_EINVAL, "bond_sum and mean must be non-NULL and 8-byte aligned");
  return check(launch_chains_mean(h->g, dev_bond_sum, n_samples, dev_mean, h->stream),
               "chains mean launch");
}

int smc_chains_dot(smc_chains* h, const double* dev_a, const double* dev_w, double* dev_out) {
  if (!h) return fail(SMC_EINVAL, "handle is NULL");
  if (!al8(dev_a) || !al8(dev_w) || !al8(dev_out))
    return fail(SMC_EINVAL, "a, b and out must be non-NULL and 8-byte aligned");
  return check(launch_chains_dot(h->g, dev_a, dev_w, dev_out, h->stream), "chains dot launch");
}

int smc_chains_vjp(smc_chains* h, double beta, int64_t n_samples, const double* dev_cov_acc,
                   const double* dev_G_acc, const double* dev_mean, const float* dev_J,
                   float* dev_grad_J, double* dev_grad_beta) {
  if (!h) return fail(SMC_EINVAL, "handle is NULL");
  if (!std::isfinite(beta) || beta < 0.0) return fail(SMC_EINVAL, "beta must be finite and >= 0");
  if (n_samples < 1) return fail(SMC_EINVAL, "n_samples must be >= 1");
  if (!al8(dev_cov_acc) || !al8(dev_G_acc) || !al8(dev_mean) || !al8(dev_grad_beta) ||
      !al4(dev_J) || !al4(dev_grad_J))
    return fail(SMC_EINVAL, "buffers must be non-NULL and aligned (double 8, float 4 bytes)");
  return check(launch_chains_vjp(h->g, dev_cov_acc, dev_G_acc, dev_mean, dev_J, n_samples, beta,
                                 dev_grad_J, dev_grad_beta, h->stream),
               "chains vjp launch");
}

int smc_chains_lnz_grad(smc_chains* h, double beta, const double* dev_mean, const float* dev_J,
                        const double* dev_scale, float* dev_grad_J_f32, double* dev_grad_J_f64,
                        double* dev_grad_beta) {
  if (!h) return fail(SMC_EINVAL, "handle is NULL");
  if (!std::isfinite(beta) || beta < 0.0) return fail(SMC_EINVAL, "beta must be finite and >= 0");
  if (!al8(dev_mean) || !al4(dev_J) || !al8(dev_grad_beta) || ((uintptr_t)dev_scale & 7))
    return fail(SMC_EINVAL, "mean, J and grad_beta must be non-NULL and aligned");
  if ((dev_grad_J_f32 != nullptr) == (dev_grad_J_f64 != nullptr))
    return fail(SMC_EINVAL, "exactly one of grad_J_f32 and grad_J_f64 must be given");
  if ((dev_grad_J_f32 && !al4(dev_grad_J_f32)) || (dev_grad_J_f64 && !al8(dev_grad_J_f64)))
    return fail(SMC_EINVAL, "grad_J must be aligned");
  return check(launch_chains_lnz_grad(h->g, dev_mean, dev_J, beta, dev_scale, dev_grad_J_f32,
                                      dev_grad_J_f64, dev_grad_beta, h->stream),
               "chains ln Z gradient launch");
}

int smc_chains_fit_step(smc_chains* h, double beta, double lr, const double* dev_target,
                        const double* dev_mean, float* dev_J) {
  if (!h) return fail(SMC_EINVAL, "handle is NULL");
  if (!std::isfinite(beta) || beta < 0.0) return fail(SMC_EINVAL, "beta must be finite and >= 0");
  if (!std::isfinite(lr)) return fail(SMC_EINVAL, "lr must be finite");
  if (!al8(dev_target) || !al8(dev_mean) || !al4(dev_J))
    return fail(SMC_EINVAL, "target, mean (8) and J (4) must be non-NULL and aligned");
  return check(launch_chains_fit_step(h->g, dev_target, dev_mean, lr * beta, dev_J, h->stream),
               "chains fit step launch");
}

int smc_chains_get_sweep_index(const smc_chains* h, uint64_t* t) {
  if (!h || !t) return fail(SMC_EINVAL, "NULL argument");
  *t = h->t;
  return SMC_OK;
}

int smc_chains_set_sweep_index(smc_chains* h, uint64_t t) {
  if (!h) return fail(SMC_EINVAL, "handle is NULL");
  if (t > 4294967296ull) return fail(SMC_ERANGE, "sweep index must be <= 2^32");
  h->t = t;
  return SMC_OK;
}

int smc_chains_destroy(smc_chains* h) {
  delete h;
  return SMC_OK;
}

}  // extern "C"
