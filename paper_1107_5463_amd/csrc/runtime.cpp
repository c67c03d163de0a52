// runtime.cpp -- host runtime behind the C ABI declared in include/smc.h.
//
// Owns only the handle (host memory).  Every device buffer is the caller's;
// every call enqueues kernels on the handle's stream.  Boltzmann thresholds
// (the tabulated factors of Sec. 2) are built here in long double for each new
// beta: T[k] = ceil(2^32 exp(-beta dE_k)) with dE_k = 4 J0 (d - k) for k
// unsatisfied bonds.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <cstdlib>
#include <cstring>
#include <string>

#include "kernels.hpp"
#include "smc.h"

using namespace smc;

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
                   SMC_FLAG_COUPLINGS_KEEP)) {
    why = "unknown flag bits";
    return false;
  }
  return true;
}

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

void build_table(smc_lattice* h, double beta) {
  if (h->tab_valid && h->tab_beta == beta) return;
  IsingTable tab;
  std::memset(&tab, 0, sizeof(tab));
  uint8_t th[8] = {0}, al[8] = {0};
  const int d = h->p.d;
  for (int k = 0; k <= 2 * d; ++k) {
    const long double dE = 4.0L * (long double)h->p.J0 * (long double)(d - k);
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
  h->tab = tab;
  h->tab_beta = beta;
  h->tab_valid = true;
}

MeasureLaunch measure_args(const smc_lattice* h) {
  MeasureLaunch m;
  m.g = h->g;
  m.n = h->p.n;
  m.J_kind = h->p.J_kind;
  m.J = h->J;
  m.J0 = h->p.J0;
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
  return a;
}

int half_sweep_impl(smc_lattice* h, double beta, uint32_t t, uint32_t colour) {
  if (h->p.n == 1) {
    const IsingLaunch a = ising_args(h, beta);
    return check(launch_ising_half_sweep(a, (int8_t*)h->spins, t, colour, h->stream),
                 "Ising half-sweep launch");
  }
  ContLaunch a;
  a.g = h->g;
  a.n = h->p.n;
  a.key = key_of(h);
  a.J_kind = h->p.J_kind;
  a.J0 = (float)h->p.J0;
  a.J = h->J;
  a.beta = (float)beta;
  a.delta = (float)h->p.delta;
  a.one_minus_cos_cap = (float)(1.0 - std::cos(h->p.delta));
  a.fast_math = (h->p.flags & SMC_FLAG_FAST_MATH) ? 1 : 0;
  return check(launch_cont_half_sweep(a, (float*)h->spins, t, colour, h->stream),
               "continuous half-sweep launch");
}

// One in-place two-pass sweep with counter t; with dev_obs the observables of
// the result are written there (fused into the colour-1 pass when the
// streaming kernel runs, else by a separate measurement).
int two_pass_sweep(smc_lattice* h, double beta, uint32_t t, void* dev_obs) {
  int rc = half_sweep_impl(h, beta, t, 0u);
  if (rc != SMC_OK) return rc;
  if (dev_obs && h->p.n == 1) {
    const IsingLaunch a = ising_args(h, beta);
    int64_t nparts = 0;
    hipError_t err = hipSuccess;
    if (ising_half_sweep_measured(a, (int8_t*)h->spins, t, h->partials, &nparts, h->stream, &err)) {
      rc = check(err, "measured Ising half-sweep launch");
      if (rc != SMC_OK) return rc;
      return check(launch_finish(measure_args(h), h->partials, nparts, dev_obs, h->stream),
                   "measurement finish launch");
    }
  }
  rc = half_sweep_impl(h, beta, t, 1u);
  if (rc != SMC_OK) return rc;
  if (dev_obs)
    return check(launch_measure(measure_args(h), h->spins, h->partials, dev_obs, h->stream),
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
      rc = check(launch_finish(measure_args(h), h->partials, nparts, dev_obs, h->stream),
                 "measurement finish launch");
      if (rc != SMC_OK) return rc;
    }
  }
  return SMC_OK;
}

int sweeps_impl(smc_lattice* h, double beta, int64_t n_sweeps, void* dev_obs) {
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
        return check(launch_measure(measure_args(h), h->spins, h->partials, dev_obs, h->stream),
                     "measurement launch");
    }
  }
  return SMC_OK;
}

}  // namespace

extern "C" {

size_t smc_spin_bytes(const smc_params* p) {
  std::string why;
  return params_ok(p, why) ? spin_bytes(p) : 0;
}

size_t smc_coupling_bytes(const smc_params* p) {
  std::string why;
  if (!params_ok(p, why) || p->J_kind == SMC_J_UNIFORM) return 0;
  return (size_t)n_sites(p) * p->d * (p->J_kind == SMC_J_PM ? 1 : 4);
}

size_t smc_workspace_bytes(const smc_params* p) {
  std::string why;
  if (!params_ok(p, why)) return 0;
  size_t b = 2 * kAlign;  // observable slot + counter
  b += partial_bytes(p);
  if (p->flags & SMC_FLAG_SCHEDULE_FUSED) b += round_up(spin_bytes(p), kAlign);
  return b;
}

size_t smc_bond_bytes(const smc_params* p) {
  std::string why;
  return params_ok(p, why) ? (size_t)n_sites(p) * p->d * 8 : 0;
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
                     : s == "stream" ? kVariantStream : kVariantAuto;
  }
  h->rows_per_band = stream_rows_per_band(h->g, 8192);
  if (const char* v = std::getenv("SMC_STREAM_ROWS")) {
    const long H = std::strtol(v, nullptr, 10);
    if (H >= 1 && H <= h->g.L && h->g.L % H == 0) h->rows_per_band = (uint32_t)H;
  }
  h->obs_slot = h->ws;
  h->counter = (uint32_t*)(h->ws + kAlign);
  h->partials = h->ws + 2 * kAlign;
  h->alt_spins = (p->flags & SMC_FLAG_SCHEDULE_FUSED) ? (void*)(h->ws + 2 * kAlign + partial_bytes(p))
                                                      : nullptr;
  h->fused_rows = fused_rows_per_band(h->g, 1024);
  if (const char* v = std::getenv("SMC_FUSED_ROWS")) {
    const long H = std::strtol(v, nullptr, 10);
    if (H >= 1 && H <= h->g.L && h->g.L % H == 0) h->fused_rows = (uint32_t)H;
  }
  h->use_fused = p->n == 1 && (p->flags & SMC_FLAG_SCHEDULE_FUSED) &&
                 !(p->flags & SMC_FLAG_GENERIC_KERNEL) &&
                 ising_fused_supported(h->g, p->J_kind, h->fused_rows);
  const RngKey key = key_of(h);
  int rc = SMC_OK;
  if (p->J_kind != SMC_J_UNIFORM && !(p->flags & SMC_FLAG_COUPLINGS_KEEP))
    rc = check(launch_init_couplings(h->g, p->J_kind, key, p->J0, p->J_sigma, h->J, h->stream),
               "coupling init launch");
  if (rc == SMC_OK && p->init != SMC_INIT_KEEP) {
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
    return check(launch_measure(measure_args(h), h->spins, h->partials, dev_obs, h->stream),
                 "measurement launch");
  return sweeps_impl(h, beta, n_sweeps, dev_obs);
}

int smc_half_sweep(smc_lattice* h, double beta, int colour) {
  if (!h) return fail(SMC_EINVAL, "handle is NULL");
  if (!beta_ok(beta)) return fail(SMC_EINVAL, "beta must be >= 0 (or +inf), not NaN");
  if (colour != 0 && colour != 1) return fail(SMC_EINVAL, "colour must be 0 or 1");
  if (h->t > 0xffffffffull) return fail(SMC_ERANGE, "sweep counter exceeds 2^32 - 1");
  return half_sweep_impl(h, beta, (uint32_t)h->t, (uint32_t)colour);
}

int smc_measure_async(smc_lattice* h, void* dev_obs) {
  if (!h) return fail(SMC_EINVAL, "handle is NULL");
  if (!dev_obs || ((uintptr_t)dev_obs & 7)) return fail(SMC_EINVAL, "dev_obs must be 8-byte aligned");
  return check(launch_measure(measure_args(h), h->spins, h->partials, dev_obs, h->stream),
               "measurement launch");
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
  if (!acc || ((uintptr_t)acc & 7)) return fail(SMC_EINVAL, "acc must be non-NULL and 8-byte aligned");
  const MeasureLaunch m = measure_args(h);
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
  int rc = check(launch_fill_zero(h->counter, 4, h->stream), "counter reset");
  if (rc != SMC_OK) return rc;
  rc = check(launch_validate(measure_args(h), h->spins, h->counter, h->stream), "validate launch");
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
  if (h->p.n == 2) return "xy_site";
  if (h->p.n == 3) return "heisenberg_site";
  if (h->use_fused) {
    if (rows_per_band) *rows_per_band = h->fused_rows;
    return "ising_fused";
  }
  IsingLaunch a;
  a.g = h->g;
  a.J_kind = h->p.J_kind;
  a.variant = (h->p.flags & SMC_FLAG_GENERIC_KERNEL) ? kVariantSite : h->ising_variant;
  a.rows_per_band = h->rows_per_band;
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

const char* smc_last_error(void) { return g_err.c_str(); }

const char* smc_version(void) { return "libsmc 0.1 (gfx950)"; }

}  // extern "C"
