// launch_args.hpp -- the argument structures the libsmc kernels receive
// (internal).  Kept apart from the launchers' declarations (kernels.hpp): a
// kernel's code depends on these layouts, not on the host-side function list.
#pragma once

#include <stdint.h>

#include "device.hpp"

namespace smc {

struct RngKey {
  uint32_t k0, k1;   // seed low / high word
  uint32_t replica;  // counter word 2
};

// Exact unsigned 32-bit division by a runtime constant (Granlund-Montgomery):
// q = (hi + ((n - hi) >> 1)) >> (l - 1) with hi = umulhi(m, n).
struct FastDiv {
  uint32_t d, m, s;
};

enum IsingVariant { kVariantAuto = 0, kVariantSite = 1, kVariantChunk = 2, kVariantStream = 3,
                    kVariantFusedWave = 4 };  // fused schedule: wave-segment kernel (no barriers)

struct IsingLaunch {
  Geom g;
  RngKey key;
  IsingTable tab;    // integer thresholds (uniform and +-1 couplings)
  int J_kind;        // 0 uniform, 1 +-1 int8, 2 FP32
  const void* J;     // [d][2][N/2] or null
  float beta;        // FP32 couplings only
  int variant;       // IsingVariant
  uint32_t rows_per_band;  // streaming kernel: rows walked by one lane (divides L)
  int heatbath;      // rule: 0 Metropolis, 1 heat bath (table holds p_+ thresholds)
  int packed_ties;   // bit-packed kernels' exact ties: 0 resolved by the workgroup, 1 by each
                     // lane, 2 by the workgroup's fallback (tied words numbered per wave;
                     // the tile kernels: each lane)
  FastDiv divQ;      // chunks per plane row
  FastDiv divL;      // edge length
};

struct ContLaunch {
  Geom g;
  int n;             // 2 or 3
  RngKey key;
  int J_kind;
  float J0;
  const void* J;
  float beta;
  float delta;       // XY max angle
  float one_minus_cos_cap;  // Heisenberg 1 - cos(theta_max)
  int fast_math;
  int variant;              // ContVariant
  uint32_t rows_per_band;   // streaming kernel band height
  uint32_t sites_per_lane;  // streaming kernel: XY 4 or 2, Heisenberg 2 or 1
  FastDiv divQ;             // lanes per plane row (R / sites per lane)
  FastDiv divL;             // edge length
  double J0d;               // uniform coupling in FP64 (fused measurement)
};

enum ContVariant { kContAuto = 0, kContRow = 1, kContStream = 2 };

// One lattice of a batch (device table, written by the host runtime).
struct BatchDesc {
  uint32_t L, R, Nh, replica;
  uint32_t divR_m, divR_s, divL_m, divL_s;  // FastDiv constants for R and L
  uint32_t th_lo, th_hi;                    // threshold bytes (always-accept classes: 0xFF)
  uint32_t spin_off_lo, spin_off_hi;        // byte offset of its [2][Nh] spins
  uint32_t J_off_lo, J_off_hi;              // byte offset of its [d][2][Nh] couplings
  uint32_t frac[7];                         // refinement fractions (2^24: always)
  uint32_t al_lo, al_hi;                    // byte k = 0xFF if class k always accepts
  uint32_t packed;                          // 1: may take the packed path (one bit per site)
  double J0;
};

struct BatchLaunch {
  int d;
  bool pm;                 // +-1 couplings (else uniform)
  uint32_t n_lattices;
  uint32_t threads;        // workgroup size (one workgroup per lattice)
  size_t max_sites;        // the largest L^d
  size_t lds_bytes;        // dynamic LDS of a workgroup (batch_lds_bytes)
  const BatchDesc* descs;  // device
  const uint32_t* order;   // device: workgroup -> lattice
  RngKey key;              // replica is taken from each descriptor
};

struct MeasureLaunch {
  Geom g;
  int n;
  int J_kind;
  const void* J;
  double J0;
  int64_t sweep;  // sweep counter of the measured state
};

// Independent chains of one small Ising lattice with shared FP32 couplings.
struct ChainsLaunch {
  Geom g;
  RngKey key;        // key.replica = replica of chain 0
  const float* J;    // [d][2][Nh]
  float beta;
  uint32_t n_chains;
  FastDiv divR, divL;  // plane row length L/2, edge L
  int pair_kernel;     // one pair of sites per lane, state in registers (N/4 <= 1024)
};

}  // namespace smc
