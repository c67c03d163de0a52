// chains.hip -- many independent Metropolis chains of one small Ising lattice
// with shared real couplings J_b, for the derivatives of ln Z (Eq. (1)):
//   d ln Z / d J_b = beta <x_b>,  d ln Z / d beta = sum_b J_b <x_b> = -<H>,
// with x_b = s_i s_j the product across bond b; and for the gradient of the
// correlations themselves (fluctuation-dissipation):
//   d <x_a> / d J_b = beta Cov(x_a, x_b).
//
// One workgroup runs one chain entirely in LDS: both colour planes, plus a
// per-bond accumulator (int32 sums of x_b for sampling, FP64 sums of
// (G - c) x_b for the covariance pass).  Chain k uses replica replica0 + k in
// the Philox counter, so chain k reproduces the single-lattice chain with FP32
// couplings and that replica bit for bit (same site rule: local field summed
// in FP32 over +x, -x, +y, -y, +z, -z; accept iff dE <= 0 or
// u < exp(-beta dE) with word j & 3 of block j >> 2).  A lane handles pairs
// of consecutive same-colour sites (half of a four-site Philox block, which
// both lanes of the block draw: twice the lanes of one block per lane, for a
// latency-bound kernel) and always the same pairs.  Every bond has exactly
// one colour-1 and one colour-0 end: the bond products of a sample are added
// in the colour-1 pass by the lane that has just updated the colour-1 end
// (no separate pass), and the covariance pass adds (G - c) x_b from the
// colour-0 ends, so no accumulator entry has two writers.
//
// The covariance pass replays the sampling sweeps: with the same start state
// and counters it visits exactly the same configurations, and needs no stored
// samples.  Per sample it forms G = sum_b g_b x_b (a workgroup reduction in a
// fixed order), then adds (G - c) x_b to bond b's accumulator.
#include "chunk.hpp"

namespace smc {

constexpr size_t kRed = 32;  // doubles of reduction scratch (one per wave + the total)

// In-plane indices of the 2d neighbours (+x, -x, +y, -y, +z, -z) of site
// (c, j) of the other colour's plane, in 32-bit arithmetic.
template <int D>
__device__ __forceinline__ void neighbours32(uint32_t j, uint32_t c, const FastDiv& dR,
                                             const FastDiv& dL, uint32_t nb[6]) {
  const uint32_t R = dR.d, L = dL.d;
  const uint32_t r = fdiv(j, dR);
  const uint32_t rowb = r * R;
  const uint32_t jx = j - rowb;
  uint32_t y = r, z = 0;
  if (D == 3) {
    z = fdiv(r, dL);
    y = r - z * L;
  }
  const uint32_t p = (c + r + z) & 1u;  // (c + y + z) & 1 with L even
  // neighbour rows: the own row's offset plus or minus a row / plane stride,
  // the periodic wrap as a select
  const uint32_t sYw = (L - 1) * R, sZ = L * R, sZw = (L - 1) * L * R;
  nb[0] = jx + p == R ? rowb : j + p;              // x + 1
  nb[1] = jx + p == 0 ? rowb + R - 1 : j + p - 1;  // x - 1
  nb[2] = y + 1 == L ? j - sYw : j + R;
  nb[3] = y == 0 ? j + sYw : j - R;
  nb[4] = nb[5] = 0;
  if (D == 3) {
    nb[4] = z + 1 == L ? j - sZw : j + sZ;
    nb[5] = z == 0 ? j + sZw : j - sZ;
  }
}

// JL: the couplings staged in LDS next to the chain (when they fit), else
// read from global memory (L2-resident: all chains share them).
// only_colour >= 0 (MODE 2, one sweep): that colour's half of sweep t0 alone.
template <int D, int MODE, bool JL>  // MODE 0: sample, 1: covariance, 2: sweeps only
__global__ __launch_bounds__(1024) void chains_kernel(const ChainsLaunch a, int8_t* __restrict__ spins,
                                                     const uint32_t t0, const uint32_t n_sweeps,
                                                     const int only_colour,
                                                     int64_t* __restrict__ bond_sum,
                                                     const double* __restrict__ gvec,
                                                     const double* __restrict__ gcp,
                                                     double* __restrict__ part,
                                                     double* __restrict__ gpart) {
  extern __shared__ __align__(16) unsigned char smem[];
  const double gc = (MODE == 1 && gcp) ? *gcp : 0.0;
  const Geom g = a.g;
  const int64_t Nh = g.Nh;
  const uint32_t NhU = (uint32_t)Nh;
  const uint32_t N = 2u * NhU;
  const uint32_t nb = (uint32_t)D * N;  // bonds
  const uint32_t chain = blockIdx.x;
  const uint32_t replica = a.key.replica + chain;
  int8_t* gs = spins + (uint64_t)chain * N;
  // LDS: kRed doubles of reduction scratch, the accumulator (4 or 8 bytes per
  // bond), the couplings (JL), then both colour planes
  constexpr size_t kAcc = MODE == 1 ? 8 : 4;  // bytes per bond (chains_lds_bytes)
  double* red = reinterpret_cast<double*>(smem);
  int32_t* acc_i = reinterpret_cast<int32_t*>(smem + kRed * sizeof(double));
  double* acc_d = reinterpret_cast<double*>(smem + kRed * sizeof(double));
  float* Jl = reinterpret_cast<float*>(smem + kRed * sizeof(double) + (size_t)nb * kAcc);
  int8_t* lat = reinterpret_cast<int8_t*>(smem + kRed * sizeof(double) + (size_t)nb * kAcc +
                                          (JL ? (size_t)nb * 4 : 0));
  const float* J = JL ? Jl : a.J;
  const float bl2e = beta_log2e(a.beta);

  for (uint32_t w = threadIdx.x; w < N / 4; w += blockDim.x)
    reinterpret_cast<uint32_t*>(lat)[w] = reinterpret_cast<const uint32_t*>(gs)[w];
  if (JL)
    for (uint32_t b = threadIdx.x; b < nb; b += blockDim.x) Jl[b] = a.J[b];
  for (uint32_t b = threadIdx.x; b < nb; b += blockDim.x) {
    if (MODE == 0) acc_i[b] = 0;
    if (MODE == 1) acc_d[b] = 0.0;
  }
  __syncthreads();

  const uint32_t pairs = (uint32_t)Nh / 2;
  double Gsum = 0.0, G2sum = 0.0;
  for (uint32_t sw = 0; sw < n_sweeps; ++sw) {
    const uint32_t t = t0 + sw;
    double Gp = 0.0;
    for (uint32_t c = 0; c < 2; ++c) {
      if (MODE == 2 && only_colour >= 0 && c != (uint32_t)only_colour) continue;
      int8_t* own = lat + c * Nh;
      const int8_t* oth = lat + (1 - c) * Nh;
      for (uint32_t pi = threadIdx.x; pi < pairs; pi += blockDim.x) {
        const Rand4 r = philox(pi >> 1, t, replica, tag(c, kContinuous), a.key.k0, a.key.k1);
#pragma unroll
        for (uint32_t b = 0; b < 2; ++b) {
          const uint32_t j = 2 * pi + b;
          uint32_t nb[6];
          neighbours32<D>(j, c, a.divR, a.divL, nb);
          const int si = own[j];
          float h = 0.0f;
#pragma unroll
          for (int mu = 0; mu < D; ++mu) {
            const float jp = J[(2 * mu + c) * NhU + j];
            const float jm = J[(2 * mu + 1 - c) * NhU + nb[2 * mu + 1]];
            h += jp * (float)oth[nb[2 * mu]];
            h += jm * (float)oth[nb[2 * mu + 1]];
          }
          const float dE = 2.0f * (float)si * h;
          const bool accept = metropolis_fp32(dE, u01f(word_of(r.w, j & 3u)), bl2e);
          if (accept) own[j] = (int8_t)(-si);
          if (MODE != 2 && c == 1) {
            // the sweep's configuration is final at this colour-1 site: the
            // products across its 2d bonds (every bond has exactly one
            // colour-1 end, so this lane alone adds to them)
            const int sn = accept ? -si : si;
#pragma unroll
            for (int mu = 0; mu < D; ++mu) {
              const int xpv = sn * oth[nb[2 * mu]];      // bond (mu, colour 1, j)
              const int xmv = sn * oth[nb[2 * mu + 1]];  // bond (mu, colour 0, -mu neighbour)
              const uint32_t bp = (2 * mu + 1) * NhU + j;
              const uint32_t bm = (2 * mu) * NhU + nb[2 * mu + 1];
              if (MODE == 0) {
                acc_i[bp] += xpv;
                acc_i[bm] += xmv;
              } else {
                Gp += gvec[bp] * (double)xpv;
                Gp += gvec[bm] * (double)xmv;
              }
            }
          }
        }
      }
      __syncthreads();
    }
    if (MODE != 1) continue;
    {
      // G of this sample: wave sums, then the waves in order
      double v = Gp;
      for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
      const uint32_t wave = threadIdx.x >> 6, nw = (blockDim.x + 63) >> 6;
      if ((threadIdx.x & 63) == 0) red[1 + wave] = v;
      __syncthreads();
      if (threadIdx.x == 0) {
        double s = 0.0;
        for (uint32_t k = 0; k < nw; ++k) s += red[1 + k];
        red[0] = s;
        const double gcen = s - gc;
        Gsum += gcen;
        G2sum += gcen * gcen;
      }
      __syncthreads();
    }
    // (G - c) x_b for every bond, owned by its colour-0 end (no lane writes a
    // colour-0 site before the next sweep's colour-0 pass, in which the same
    // lane owns it)
    const double Gc = red[0] - gc;
    for (uint32_t pi = threadIdx.x; pi < pairs; pi += blockDim.x) {
#pragma unroll
      for (uint32_t b = 0; b < 2; ++b) {
        const uint32_t j = 2 * pi + b;
        uint32_t nb[6];
        neighbours32<D>(j, 0u, a.divR, a.divL, nb);
        const int s0 = lat[j];
#pragma unroll
        for (int mu = 0; mu < D; ++mu) {
          const uint32_t ip = nb[2 * mu], im = nb[2 * mu + 1];
          const int xpv = s0 * lat[NhU + ip];  // bond (mu, colour 0, j)
          const int xmv = s0 * lat[NhU + im];  // bond (mu, colour 1, im)
          acc_d[(2 * mu) * NhU + j] += Gc * (double)xpv;
          acc_d[(2 * mu + 1) * NhU + im] += Gc * (double)xmv;
        }
      }
    }
    // the next colour-0 pass writes only sites whose bonds this lane owns
  }
  __syncthreads();
  for (uint32_t w = threadIdx.x; w < N / 4; w += blockDim.x)
    reinterpret_cast<uint32_t*>(gs)[w] = reinterpret_cast<const uint32_t*>(lat)[w];
  if (MODE == 0) {
    for (uint32_t b = threadIdx.x; b < nb; b += blockDim.x)
      if (acc_i[b] != 0)
        atomicAdd(reinterpret_cast<unsigned long long*>(bond_sum + b),
                  (unsigned long long)(int64_t)acc_i[b]);
  } else if (MODE == 1) {
    double* pc = part + (uint64_t)chain * nb;
    for (uint32_t b = threadIdx.x; b < nb; b += blockDim.x) pc[b] = acc_d[b];
    if (threadIdx.x == 0) {
      gpart[2 * chain] = Gsum;
      gpart[2 * chain + 1] = G2sum;
    }
  }
}

// J * s for a spin s = +-1 held as a sign-extended int (-1 has bit 31 set):
// a sign flip, exactly the product.
__device__ __forceinline__ float signed_by(float J, int s) {
  return __int_as_float(__float_as_int(J) ^ (s & (int)0x80000000));
}

// Exchange a value with the neighbouring lane (lanes 2q and 2q + 1 swap):
// DPP quad permutation [1, 0, 3, 2].
__device__ __forceinline__ uint32_t swap_pair_lanes(uint32_t v) {
  return (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0xB1, 0xF, 0xF, false);
}

// Chains of lattices with at most one pair of same-colour sites per lane
// (N/4 <= 1024, e.g. 2D L = 64): lane q owns sites 2q and 2q + 1 of BOTH
// colour planes for the whole call and keeps their spins, the byte offsets
// of their 2d neighbours in LDS and the couplings of their 2d bonds in
// registers (the couplings are read once per call), so a site update is the
// field sum, the decision and one LDS store.  The two lanes of a four-site
// Philox block draw one block each per sweep -- the even lane colour 0's,
// the odd lane colour 1's -- and swap the halves the other needs, so no
// block is drawn twice.  Bond products of colour-1 sites (each bond has
// exactly one colour-1 end) are counted in registers: a sum of
// s_i ^ s_j = -2 per unsatisfied bond, so sum x_b = samples + that sum.
// Same decisions as chains_kernel: local field summed in FP32 over +x, -x,
// +y, -y, +z, -z (the terms are exact sign flips of J), dE = 2 s h, accept
// iff dE <= 0 or u < exp(-beta dE) (metropolis_fp32).
// MODE 0: sample (bond sums), 1: covariance replay, 2: sweeps only (with
// only_colour >= 0 and one sweep: that colour's half of sweep t0 alone).
template <int D, int MODE>
__global__ __launch_bounds__(1024) void chains_pair_kernel(const ChainsLaunch a,
                                                          int8_t* __restrict__ spins,
                                                          const uint32_t t0, const uint32_t n_sweeps,
                                                          const int only_colour,
                                                          int64_t* __restrict__ bond_sum,
                                                          const double* __restrict__ gvec,
                                                          const double* __restrict__ gcp,
                                                          double* __restrict__ part,
                                                          double* __restrict__ gpart) {
  constexpr int B = 2 * D;  // bonds (neighbours) per site
  extern __shared__ __align__(16) unsigned char smem[];
  const double gc = (MODE == 1 && gcp) ? *gcp : 0.0;
  const uint32_t NhU = (uint32_t)a.g.Nh;
  const uint32_t N = 2u * NhU;
  const uint32_t pairs = NhU / 2;
  const uint32_t chain = blockIdx.x;
  const uint32_t replica = a.key.replica + chain;
  const uint32_t q = threadIdx.x;
  const bool active = q < pairs;
  int8_t* gs = spins + (uint64_t)chain * N;
  double* red = reinterpret_cast<double*>(smem);
  int8_t* lat = reinterpret_cast<int8_t*>(smem + kRed * sizeof(double));
  const float bl2e = beta_log2e(a.beta);

  for (uint32_t w = q; w < N / 4; w += blockDim.x)
    reinterpret_cast<uint32_t*>(lat)[w] = reinterpret_cast<const uint32_t*>(gs)[w];
  __syncthreads();

  // the lane's four sites: (c, 2q + b)
  uint32_t off[2][2][B];  // LDS byte offsets of the neighbours (other plane)
  float Jv[2][2][B];      // couplings of the bonds to them
  int sv[2][2];           // the sites' spins
#pragma unroll
  for (uint32_t c = 0; c < 2; ++c)
#pragma unroll
    for (uint32_t b = 0; b < 2; ++b) {
      const uint32_t j = active ? 2 * q + b : 0u;
      uint32_t nb[6];
      neighbours32<D>(j, c, a.divR, a.divL, nb);
#pragma unroll
      for (int mu = 0; mu < D; ++mu) {
        off[c][b][2 * mu] = (1 - c) * NhU + nb[2 * mu];
        off[c][b][2 * mu + 1] = (1 - c) * NhU + nb[2 * mu + 1];
        Jv[c][b][2 * mu] = a.J[(2 * mu + c) * NhU + j];
        Jv[c][b][2 * mu + 1] = a.J[(2 * mu + 1 - c) * NhU + nb[2 * mu + 1]];
      }
      sv[c][b] = lat[c * NhU + j];
    }

  // colour-1 sites' bonds: m = 2 mu -> bond (mu, 1, j), m = 2 mu + 1 -> bond
  // (mu, 0, -mu neighbour of j)
  // (with the covariance weights g_b of those bonds: the covariance replay of
  // 3D lattices runs chains_kernel, whose chains are the same)
  static_assert(MODE != 1 || D == 2, "3D covariance replays run chains_kernel");
  auto bond_of = [&](uint32_t b, int m) -> uint32_t {
    const uint32_t mu = (uint32_t)m >> 1;
    return (m & 1) ? (2 * mu) * NhU + off[1][b][m] : (2 * mu + 1) * NhU + 2 * q + b;
  };
  int32_t acc[2][B];
  double accd[2][B];
  double gv[2][B];
#pragma unroll
  for (uint32_t b = 0; b < 2; ++b)
#pragma unroll
    for (int m = 0; m < B; ++m) {
      acc[b][m] = 0;
      accd[b][m] = 0.0;
      gv[b][m] = (MODE == 1 && active) ? gvec[bond_of(b, m)] : 0.0;
    }

  const uint32_t odd = q & 1u;
  double Gsum = 0.0, G2sum = 0.0;
  for (uint32_t sw = 0; sw < n_sweeps; ++sw) {
    const uint32_t t = t0 + sw;
    // the even lane draws colour 0's block of this pair's four sites, the
    // odd lane colour 1's; each keeps the two words of its own sites and
    // sends the other two
    const Rand4 r = philox(q >> 1, t, replica, tag(odd, kContinuous), a.key.k0, a.key.k1);
    const uint32_t got0 = swap_pair_lanes(odd ? r.w[0] : r.w[2]);
    const uint32_t got1 = swap_pair_lanes(odd ? r.w[1] : r.w[3]);
    uint32_t wd[2][2];
    wd[0][0] = odd ? got0 : r.w[0];
    wd[0][1] = odd ? got1 : r.w[1];
    wd[1][0] = odd ? r.w[2] : got0;
    wd[1][1] = odd ? r.w[3] : got1;
    uint32_t xneg = 0;  // bit (b, m): bond product of a colour-1 site is -1
#pragma unroll
    for (uint32_t c = 0; c < 2; ++c) {
      if (MODE == 2 && only_colour >= 0 && c != (uint32_t)only_colour) continue;
#pragma unroll
      for (uint32_t b = 0; b < 2; ++b) {
        int nv[B];
#pragma unroll
        for (int m = 0; m < B; ++m) nv[m] = lat[off[c][b][m]];
        float h = signed_by(Jv[c][b][0], nv[0]);
#pragma unroll
        for (int m = 1; m < B; ++m) h += signed_by(Jv[c][b][m], nv[m]);
        const int si = sv[c][b];
        const float dE = 2.0f * signed_by(h, si);
        const bool accept = metropolis_fp32(dE, u01f(wd[c][b]), bl2e);
        const int sn = accept ? -si : si;
        sv[c][b] = sn;
        if (active && accept) lat[c * NhU + 2 * q + b] = (int8_t)sn;
        if (MODE != 2 && c == 1) {
#pragma unroll
          for (int m = 0; m < B; ++m) {
            if (MODE == 0) acc[b][m] += sn ^ nv[m];
            if (MODE == 1) xneg |= (uint32_t)(sn != nv[m]) << (b * B + m);
          }
        }
      }
      __syncthreads();
    }
    if (MODE != 1) continue;
    // G of this sample (wave sums, then the waves in order), then (G - c) x_b
    double Gp = 0.0;
#pragma unroll
    for (uint32_t b = 0; b < 2; ++b)
#pragma unroll
      for (int m = 0; m < B; ++m) Gp += ((xneg >> (b * B + m)) & 1u) ? -gv[b][m] : gv[b][m];
    double v = Gp;
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    const uint32_t wave = q >> 6, nw = (blockDim.x + 63) >> 6;
    if ((q & 63) == 0) red[1 + wave] = v;
    __syncthreads();
    if (q == 0) {
      double sg = 0.0;
      for (uint32_t k = 0; k < nw; ++k) sg += red[1 + k];
      red[0] = sg;
      const double gcen = sg - gc;
      Gsum += gcen;
      G2sum += gcen * gcen;
    }
    __syncthreads();
    const double Gc = red[0] - gc;
#pragma unroll
    for (uint32_t b = 0; b < 2; ++b)
#pragma unroll
      for (int m = 0; m < B; ++m) accd[b][m] += ((xneg >> (b * B + m)) & 1u) ? -Gc : Gc;
    // red[0] is rewritten only after the next sweep's two barriers
  }

  for (uint32_t w = q; w < N / 4; w += blockDim.x)
    reinterpret_cast<uint32_t*>(gs)[w] = reinterpret_cast<const uint32_t*>(lat)[w];
  if (MODE == 2 || !active) return;
  const uint32_t nbonds = (uint32_t)D * N;
#pragma unroll
  for (uint32_t b = 0; b < 2; ++b)
#pragma unroll
    for (int m = 0; m < B; ++m) {
      const uint32_t bond = bond_of(b, m);
      if (MODE == 0)
        atomicAdd(reinterpret_cast<unsigned long long*>(bond_sum + bond),
                  (unsigned long long)((int64_t)n_sweeps + acc[b][m]));
      else
        part[(uint64_t)chain * nbonds + bond] = accd[b][m];
    }
  if (MODE == 1 && q == 0) {
    gpart[2 * chain] = Gsum;
    gpart[2 * chain + 1] = G2sum;
  }
}

// Sum the per-chain covariance partials into the caller's accumulators in
// chain order (deterministic).
__global__ __launch_bounds__(256) void chains_reduce_kernel(const double* __restrict__ part,
                                                            const double* __restrict__ gpart,
                                                            const uint32_t n_chains,
                                                            const uint32_t nb,
                                                            double* __restrict__ cov_acc,
                                                            double* __restrict__ G_acc) {
  const uint32_t b = blockIdx.x * 256 + threadIdx.x;
  if (b < nb) {
    double s = 0.0;
    for (uint32_t k = 0; k < n_chains; ++k) s += part[(uint64_t)k * nb + b];
    cov_acc[b] += s;
  }
  if (blockIdx.x == 0 && threadIdx.x < 2) {
    double s = 0.0;
    for (uint32_t k = 0; k < n_chains; ++k) s += gpart[2 * k + threadIdx.x];
    G_acc[threadIdx.x] += s;
  }
}

// ---------------------------------------------------------------------------
// Finishing the derivative estimates over the d N bonds (FP64; every sum over
// bonds is taken by one workgroup in a fixed order, so results are
// deterministic).  With S samples (chains x sweeps):
//   <x_b> = bond_sum_b / S;
//   Cov(G, x_b) = cov_acc_b / S - (G_acc_0 / S) <x_b>   (G_acc_0 = sum (G - c));
//   vector-Jacobian product of <x>: beta Cov(G, x_b) for J_b and
//   sum_b J_b Cov(G, x_b) for beta;
//   ln Z: d/dJ_b = beta <x_b>, d/dbeta = sum_b J_b <x_b>;
//   moment matching: J_b += lr beta (target_b - <x_b>).
// ---------------------------------------------------------------------------
constexpr int kFinishThreads = 256;

// Sum of v over the workgroup in a fixed order (all threads get it).
__device__ double block_sum_fixed(double v, double* sh) {
  sh[threadIdx.x] = v;
  __syncthreads();
  for (unsigned s = kFinishThreads / 2; s > 0; s >>= 1) {
    if (threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
    __syncthreads();
  }
  const double r = sh[0];
  __syncthreads();
  return r;
}

__global__ __launch_bounds__(256) void chains_mean_kernel(const int64_t* __restrict__ sum,
                                                          const uint32_t nb, const double S,
                                                          double* __restrict__ mean) {
  const uint32_t b = blockIdx.x * 256 + threadIdx.x;
  if (b < nb) mean[b] = (double)sum[b] / S;
}

// out[0] = sum_b a_b w_b
__global__ __launch_bounds__(kFinishThreads) void chains_dot_kernel(const double* __restrict__ a,
                                                                    const double* __restrict__ w,
                                                                    const uint32_t nb,
                                                                    double* __restrict__ out) {
  __shared__ double sh[kFinishThreads];
  double v = 0.0;
  for (uint32_t b = threadIdx.x; b < nb; b += kFinishThreads) v += a[b] * w[b];
  v = block_sum_fixed(v, sh);
  if (threadIdx.x == 0) out[0] = v;
}

__global__ __launch_bounds__(kFinishThreads) void chains_vjp_kernel(
    const double* __restrict__ cov_acc, const double* __restrict__ G_acc,
    const double* __restrict__ mean, const float* __restrict__ J, const uint32_t nb,
    const double S, const double beta, float* __restrict__ grad_J, double* __restrict__ grad_beta) {
  __shared__ double sh[kFinishThreads];
  const double gm = G_acc[0] / S;
  double v = 0.0;
  for (uint32_t b = threadIdx.x; b < nb; b += kFinishThreads) {
    const double cov = cov_acc[b] / S - gm * mean[b];
    grad_J[b] = (float)(beta * cov);
    v += (double)J[b] * cov;
  }
  v = block_sum_fixed(v, sh);
  if (threadIdx.x == 0) grad_beta[0] = v;
}

// scale: the upstream gradient of ln Z (1 if NULL); the J gradient goes to
// gJ32 (float) or gJ64 (double), whichever is given.
__global__ __launch_bounds__(kFinishThreads) void chains_lnz_grad_kernel(
    const double* __restrict__ mean, const float* __restrict__ J, const uint32_t nb,
    const double beta, const double* __restrict__ scale, float* __restrict__ gJ32,
    double* __restrict__ gJ64, double* __restrict__ grad_beta) {
  __shared__ double sh[kFinishThreads];
  const double sc = scale ? scale[0] : 1.0;
  const double sb = sc * beta;
  double v = 0.0;
  for (uint32_t b = threadIdx.x; b < nb; b += kFinishThreads) {
    const double gj = sb * mean[b];
    if (gJ32) gJ32[b] = (float)gj;
    if (gJ64) gJ64[b] = gj;
    v += (double)J[b] * mean[b];
  }
  v = block_sum_fixed(v, sh);
  if (threadIdx.x == 0) grad_beta[0] = sc * v;
}

__global__ __launch_bounds__(256) void chains_fit_step_kernel(const double* __restrict__ target,
                                                              const double* __restrict__ mean,
                                                              const uint32_t nb, const double rate,
                                                              float* __restrict__ J) {
  const uint32_t b = blockIdx.x * 256 + threadIdx.x;
  if (b < nb) J[b] = J[b] + (float)(rate * (target[b] - mean[b]));
}

static uint32_t n_bonds(const Geom& g) { return (uint32_t)(g.d * 2 * g.Nh); }

hipError_t launch_chains_mean(const Geom& g, const int64_t* sum, int64_t n_samples, double* mean,
                              hipStream_t st) {
  const uint32_t nb = n_bonds(g);
  hipLaunchKernelGGL(chains_mean_kernel, dim3((nb + 255) / 256), dim3(256), 0, st, sum, nb,
                     (double)n_samples, mean);
  return hipGetLastError();
}

hipError_t launch_chains_dot(const Geom& g, const double* a, const double* w, double* out,
                             hipStream_t st) {
  hipLaunchKernelGGL(chains_dot_kernel, dim3(1), dim3(kFinishThreads), 0, st, a, w, n_bonds(g), out);
  return hipGetLastError();
}

hipError_t launch_chains_vjp(const Geom& g, const double* cov_acc, const double* G_acc,
                             const double* mean, const float* J, int64_t n_samples, double beta,
                             float* grad_J, double* grad_beta, hipStream_t st) {
  hipLaunchKernelGGL(chains_vjp_kernel, dim3(1), dim3(kFinishThreads), 0, st, cov_acc, G_acc, mean,
                     J, n_bonds(g), (double)n_samples, beta, grad_J, grad_beta);
  return hipGetLastError();
}

hipError_t launch_chains_lnz_grad(const Geom& g, const double* mean, const float* J, double beta,
                                  const double* scale, float* gJ32, double* gJ64,
                                  double* grad_beta, hipStream_t st) {
  hipLaunchKernelGGL(chains_lnz_grad_kernel, dim3(1), dim3(kFinishThreads), 0, st, mean, J,
                     n_bonds(g), beta, scale, gJ32, gJ64, grad_beta);
  return hipGetLastError();
}

hipError_t launch_chains_fit_step(const Geom& g, const double* target, const double* mean,
                                  double rate, float* J, hipStream_t st) {
  const uint32_t nb = n_bonds(g);
  hipLaunchKernelGGL(chains_fit_step_kernel, dim3((nb + 255) / 256), dim3(256), 0, st, target,
                     mean, nb, rate, J);
  return hipGetLastError();
}

// LDS of one chain: reduction scratch, per-bond accumulator (int32 when
// sampling or sweeping only, double for the covariance), both planes.
size_t chains_lds_bytes(const Geom& g, int mode) {
  const size_t N = 2 * (size_t)g.Nh;
  return kRed * sizeof(double) + (size_t)g.d * N * (mode == 1 ? 8 : 4) + N;
}

constexpr size_t kLdsMax = 160 * 1024;

// The same with the couplings staged in LDS, if that fits (else 0).
static size_t chains_lds_bytes_jl(const Geom& g, int mode) {
  const size_t b = chains_lds_bytes(g, mode) + (size_t)g.d * 2 * (size_t)g.Nh * 4;
  return b <= kLdsMax ? b : 0;
}

// LDS of the pair kernel: reduction scratch and both planes.
static size_t chains_pair_lds_bytes(const Geom& g) { return kRed * sizeof(double) + 2 * (size_t)g.Nh; }

bool chains_pair_supported(const Geom& g) { return g.Nh / 2 <= 1024; }

// Workgroup size: one lane per pair of sites of a colour, in whole waves,
// at most 1024.
static uint32_t chains_threads(const Geom& g) {
  const uint32_t pairs = (uint32_t)(g.Nh / 2);
  const uint32_t t = (pairs + 63) / 64 * 64;
  return t < 64 ? 64 : (t > 1024 ? 1024 : t);
}

static const void* chains_fn(int d, int mode, bool jl) {
#define SMC_CF(DD, JJ) \
  (mode == 0 ? (const void*)chains_kernel<DD, 0, JJ> \
             : (mode == 1 ? (const void*)chains_kernel<DD, 1, JJ> : (const void*)chains_kernel<DD, 2, JJ>))
  if (d == 2) return jl ? SMC_CF(2, true) : SMC_CF(2, false);
  return jl ? SMC_CF(3, true) : SMC_CF(3, false);
#undef SMC_CF
}

hipError_t chains_allow_lds(const Geom& g) {
  for (int mode = 0; mode < 3; ++mode) {
    const size_t ljl = chains_lds_bytes_jl(g, mode);
    const size_t b = ljl ? ljl : chains_lds_bytes(g, mode);
    const hipError_t e = allow_dynamic_lds(chains_fn(g.d, mode, ljl != 0), b);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

// One launch of n_sweeps sweeps (mode 0: bond sums, 1: covariance partials,
// 2: sweeps only, or one colour's half of sweep t0 with only_colour >= 0).
static hipError_t launch_chains(const ChainsLaunch& a, int mode, int8_t* spins, uint32_t t0,
                                uint32_t n_sweeps, int only_colour, int64_t* bond_sum,
                                const double* g, const double* gc, double* part, double* gpart,
                                hipStream_t st) {
  const dim3 grid(a.n_chains), block(chains_threads(a.g));
  if (a.pair_kernel && !(mode == 1 && a.g.d == 3)) {
    const size_t lds = chains_pair_lds_bytes(a.g);
#define SMC_CP(DD, MM)                                                                              \
  hipLaunchKernelGGL((chains_pair_kernel<DD, MM>), grid, block, lds, st, a, spins, t0, n_sweeps, \
                     only_colour, bond_sum, g, gc, part, gpart)
    if (a.g.d == 2) {
      if (mode == 0) SMC_CP(2, 0); else if (mode == 1) SMC_CP(2, 1); else SMC_CP(2, 2);
    } else {
      if (mode == 0) SMC_CP(3, 0); else SMC_CP(3, 2);
    }
#undef SMC_CP
    return hipGetLastError();
  }
  const size_t ljl = chains_lds_bytes_jl(a.g, mode);
  const bool jl = ljl != 0;
  const size_t lds = jl ? ljl : chains_lds_bytes(a.g, mode);
#define SMC_CS(DD, MM, JJ)                                                                     \
  hipLaunchKernelGGL((chains_kernel<DD, MM, JJ>), grid, block, lds, st, a, spins, t0, n_sweeps, \
                     only_colour, bond_sum, g, gc, part, gpart)
#define SMC_CM(DD, JJ) \
  do { if (mode == 0) SMC_CS(DD, 0, JJ); else if (mode == 1) SMC_CS(DD, 1, JJ); else SMC_CS(DD, 2, JJ); } while (0)
  if (a.g.d == 2) {
    if (jl) SMC_CM(2, true); else SMC_CM(2, false);
  } else {
    if (jl) SMC_CM(3, true); else SMC_CM(3, false);
  }
#undef SMC_CM
#undef SMC_CS
  return hipGetLastError();
}

hipError_t launch_chains_sample(const ChainsLaunch& a, int8_t* spins, uint32_t t0,
                                uint32_t n_sweeps, int64_t* bond_sum, hipStream_t st) {
  return launch_chains(a, bond_sum ? 0 : 2, spins, t0, n_sweeps, -1, bond_sum, nullptr, nullptr,
                       nullptr, nullptr, st);
}

hipError_t launch_chains_half_sweep(const ChainsLaunch& a, int8_t* spins, uint32_t t,
                                    int colour, hipStream_t st) {
  return launch_chains(a, 2, spins, t, 1, colour, nullptr, nullptr, nullptr, nullptr, nullptr, st);
}

hipError_t launch_chains_covariance(const ChainsLaunch& a, int8_t* spins, uint32_t t0,
                                    uint32_t n_sweeps, const double* g, const double* gc, double* part,
                                    double* gpart, double* cov_acc, double* G_acc,
                                    hipStream_t st) {
  hipError_t e = launch_chains(a, 1, spins, t0, n_sweeps, -1, nullptr, g, gc, part, gpart, st);
  if (e != hipSuccess) return e;
  const uint32_t nb = (uint32_t)(a.g.d * 2 * a.g.Nh);
  hipLaunchKernelGGL(chains_reduce_kernel, dim3((nb + 255) / 256), dim3(256), 0, st, part, gpart,
                     a.n_chains, nb, cov_acc, G_acc);
  return hipGetLastError();
}

}  // namespace smc
