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
template <int D, int MODE, bool JL>  // MODE 0: sample, 1: covariance, 2: sweeps only
__global__ __launch_bounds__(1024) void chains_kernel(const ChainsLaunch a, int8_t* __restrict__ spins,
                                                     const uint32_t t0, const uint32_t n_sweeps,
                                                     int64_t* __restrict__ bond_sum,
                                                     const double* __restrict__ gvec,
                                                     const double gc, double* __restrict__ part,
                                                     double* __restrict__ gpart) {
  extern __shared__ __align__(16) unsigned char smem[];
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
  const float beta = a.beta;

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
          const bool accept = dE <= 0.0f || u01f(word_of(r.w, j & 3u)) < expf(-beta * dE);
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

hipError_t launch_chains_sample(const ChainsLaunch& a, int8_t* spins, uint32_t t0,
                                uint32_t n_sweeps, int64_t* bond_sum, hipStream_t st) {
  const int mode = bond_sum ? 0 : 2;
  const size_t ljl = chains_lds_bytes_jl(a.g, mode);
  const bool jl = ljl != 0;
  const size_t lds = jl ? ljl : chains_lds_bytes(a.g, mode);
  const dim3 grid(a.n_chains), block(chains_threads(a.g));
#define SMC_CS(DD, MM, JJ)                                                                     \
  hipLaunchKernelGGL((chains_kernel<DD, MM, JJ>), grid, block, lds, st, a, spins, t0, n_sweeps, \
                     bond_sum, nullptr, 0.0, nullptr, nullptr)
  if (a.g.d == 2) {
    if (mode == 0) { if (jl) SMC_CS(2, 0, true); else SMC_CS(2, 0, false); }
    else { if (jl) SMC_CS(2, 2, true); else SMC_CS(2, 2, false); }
  } else {
    if (mode == 0) { if (jl) SMC_CS(3, 0, true); else SMC_CS(3, 0, false); }
    else { if (jl) SMC_CS(3, 2, true); else SMC_CS(3, 2, false); }
  }
#undef SMC_CS
  return hipGetLastError();
}

hipError_t launch_chains_covariance(const ChainsLaunch& a, int8_t* spins, uint32_t t0,
                                    uint32_t n_sweeps, const double* g, double gc, double* part,
                                    double* gpart, double* cov_acc, double* G_acc,
                                    hipStream_t st) {
  const size_t ljl = chains_lds_bytes_jl(a.g, 1);
  const bool jl = ljl != 0;
  const size_t lds = jl ? ljl : chains_lds_bytes(a.g, 1);
  const dim3 grid(a.n_chains), block(chains_threads(a.g));
#define SMC_CC(DD, JJ)                                                                         \
  hipLaunchKernelGGL((chains_kernel<DD, 1, JJ>), grid, block, lds, st, a, spins, t0, n_sweeps, \
                     nullptr, g, gc, part, gpart)
  if (a.g.d == 2) {
    if (jl) SMC_CC(2, true); else SMC_CC(2, false);
  } else {
    if (jl) SMC_CC(3, true); else SMC_CC(3, false);
  }
#undef SMC_CC
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const uint32_t nb = (uint32_t)(a.g.d * 2 * a.g.Nh);
  hipLaunchKernelGGL(chains_reduce_kernel, dim3((nb + 255) / 256), dim3(256), 0, st, part, gpart,
                     a.n_chains, nb, cov_acc, G_acc);
  return hipGetLastError();
}

}  // namespace smc
