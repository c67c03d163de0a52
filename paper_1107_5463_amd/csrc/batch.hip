// batch.hip -- many independent Ising lattices of uneven size, temperature and
// disorder realisation in one persistent launch (the paper's trivial
// parallelism over disorder realisations on top of the checkerboard
// decomposition, Sec. 2).
//
// One workgroup owns one lattice: it stages both colour planes (L^d bytes,
// at most 64 KiB) in LDS, runs every sweep of the call there -- colour 0,
// barrier, colour 1, barrier -- and writes the planes back once, so HBM is
// touched only at the start and the end.  Couplings stay in global memory
// (they are re-read from L2 / Infinity Cache).  Lattice r uses replica r in
// the Philox counter, so each lattice reproduces the single-lattice chain
// with that replica bit for bit.  A lane walks groups of 16 consecutive
// same-colour sites (one Philox block of prefix bytes per group); the
// decision per site is the integer threshold test of the single-lattice
// kernels with its exact tie refinement.  With MEASURE the workgroup also
// reduces E and M of its final state from LDS.
#include "chunk.hpp"
#include "reduce.hpp"

namespace smc {

template <int D, bool PM, bool MEASURE>
__global__ __launch_bounds__(512) void batch_kernel(const BatchDesc* __restrict__ descs,
                                                    const uint32_t* __restrict__ order,
                                                    const RngKey key, int8_t* __restrict__ spins,
                                                    const int8_t* __restrict__ J,
                                                    const uint32_t t0, const uint32_t n_sweeps,
                                                    ObsOut* __restrict__ obs) {
  extern __shared__ int8_t lat[];  // [2][Nh] spins of this lattice
  const uint32_t li = __builtin_amdgcn_readfirstlane(order[blockIdx.x]);
  const BatchDesc* dp = descs + li;
  const uint32_t L = __builtin_amdgcn_readfirstlane(dp->L);
  const uint32_t R = __builtin_amdgcn_readfirstlane(dp->R);
  const uint32_t Nh = __builtin_amdgcn_readfirstlane(dp->Nh);
  FastDiv divR, divL;
  divR.d = R;
  divR.m = (uint32_t)__builtin_amdgcn_readfirstlane(dp->divR_m);
  divR.s = (uint32_t)__builtin_amdgcn_readfirstlane(dp->divR_s);
  divL.d = L;
  divL.m = (uint32_t)__builtin_amdgcn_readfirstlane(dp->divL_m);
  divL.s = (uint32_t)__builtin_amdgcn_readfirstlane(dp->divL_s);
  const uint32_t th_lo = __builtin_amdgcn_readfirstlane(dp->th_lo);
  const uint32_t th_hi = __builtin_amdgcn_readfirstlane(dp->th_hi);
  const uint32_t replica = __builtin_amdgcn_readfirstlane(dp->replica);
  const uint64_t soff = ((uint64_t)__builtin_amdgcn_readfirstlane(dp->spin_off_hi) << 32) |
                        __builtin_amdgcn_readfirstlane(dp->spin_off_lo);
  const uint64_t joff = ((uint64_t)__builtin_amdgcn_readfirstlane(dp->J_off_hi) << 32) |
                        __builtin_amdgcn_readfirstlane(dp->J_off_lo);
  int8_t* gs = spins + soff;
  const int8_t* gJ = J + joff;
  const uint32_t N = 2 * Nh;  // L^d, a multiple of 4 (L even)

  // Stage both planes into LDS as one byte per site: bit 0 = spin -1, bit
  // 1 + m = coupling of bond m negative (m = +x, -x, +y, -y, +z, -z), so the
  // sweep reads couplings from LDS together with the spins.
  auto nbr = [&](uint32_t c, uint32_t j, uint32_t nbi[6]) {  // in-plane neighbour indices
    const uint32_t r = fdiv(j, divR);
    const uint32_t jx = j - r * R;
    const uint32_t z = D == 3 ? fdiv(r, divL) : 0u;
    const uint32_t y = r - z * L;
    const uint32_t p = (c + y + z) & 1u;
    const uint32_t rowb = r * R;
    nbi[0] = rowb + (jx + p == R ? 0u : jx + p);
    nbi[1] = rowb + (jx + p == 0 ? R - 1 : jx + p - 1);
    const uint32_t ym = y == 0 ? L - 1 : y - 1, yp = y + 1 == L ? 0 : y + 1;
    nbi[2] = (z * L + yp) * R + jx;
    nbi[3] = (z * L + ym) * R + jx;
    nbi[4] = nbi[5] = 0;
    if (D == 3) {
      const uint32_t zm = z == 0 ? L - 1 : z - 1, zp = z + 1 == L ? 0 : z + 1;
      nbi[4] = (zp * L + y) * R + jx;
      nbi[5] = (zm * L + y) * R + jx;
    }
  };
  for (uint32_t i = threadIdx.x; i < N; i += blockDim.x) {
    const uint32_t c = i >= Nh ? 1u : 0u;
    const uint32_t j = i - c * Nh;
    uint32_t v = gs[i] < 0 ? 1u : 0u;
    if (PM) {
      uint32_t nbi[6];
      nbr(c, j, nbi);
      const int8_t* Jo = gJ + (uint64_t)c * Nh;        // J[mu][c] = gJ + (2 mu + c) Nh
      const int8_t* Jn = gJ + (uint64_t)(1 - c) * Nh;  // J[mu][1 - c]
#pragma unroll
      for (int mu = 0; mu < D; ++mu) {
        v |= (Jo[2 * (uint64_t)mu * Nh + j] < 0 ? 1u : 0u) << (1 + 2 * mu);
        v |= (Jn[2 * (uint64_t)mu * Nh + nbi[2 * mu + 1]] < 0 ? 1u : 0u) << (2 + 2 * mu);
      }
    }
    lat[i] = (int8_t)v;
  }
  __syncthreads();

  // One site: k = bonds with J s_i s_nb < 0 from the combined bytes.
  auto site_k = [&](const int8_t* own, const int8_t* oth, uint32_t c, uint32_t j,
                    uint32_t& o) -> uint32_t {
    uint32_t nbi[6];
    nbr(c, j, nbi);
    o = (uint8_t)own[j];
    uint32_t nm = 0;
#pragma unroll
    for (int m = 0; m < 2 * D; ++m) nm |= ((uint32_t)(uint8_t)oth[nbi[m]] & 1u) << m;
    const uint32_t om = (0u - (o & 1u)) & ((1u << (2 * D)) - 1u);
    return __builtin_popcount(nm ^ om ^ (PM ? (o >> 1) : 0u));
  };
  const uint32_t ngroups = (Nh + 15) / 16;
  for (uint32_t sw = 0; sw < n_sweeps; ++sw) {
    const uint32_t t = t0 + sw;
    for (uint32_t c = 0; c < 2; ++c) {
      int8_t* own = lat + c * Nh;
      const int8_t* oth = lat + (1 - c) * Nh;
      for (uint32_t g = threadIdx.x; g < ngroups; g += blockDim.x) {
        const uint32_t j0 = 16 * g;
        const Rand4 rp = philox(g, t, replica, tag(c, kIsingPrefix), key.k0, key.k1);
        const uint32_t nj = Nh - j0 < 16 ? Nh - j0 : 16u;
        auto one = [&](uint32_t jj, uint32_t word) {
          const uint32_t j = j0 + jj;
          uint32_t o;
          const uint32_t k = site_k(own, oth, c, j, o);
          const uint32_t P = (word >> (8 * (jj & 3))) & 0xFFu;
          const uint32_t Th = table_byte(th_lo, th_hi, k);
          bool accept = P < Th;
          if (P == Th) {
            const Rand4 rr = philox(j, t, replica, tag(c, kIsingRefine), key.k0, key.k1);
            accept = (rr.w[0] & 0xFFFFFFu) < dp->frac[k];  // rare: read from the table
          }
          if (accept) own[j] = (int8_t)(o ^ 1u);
        };
        if (nj == 16) {
#pragma unroll
          for (uint32_t jj = 0; jj < 16; ++jj) one(jj, rp.w[jj >> 2]);
        } else {
          for (uint32_t jj = 0; jj < nj; ++jj) {
            const uint32_t wlo = (jj & 4) ? rp.w[1] : rp.w[0];
            const uint32_t whi = (jj & 4) ? rp.w[3] : rp.w[2];
            one(jj, (jj & 8) ? whi : wlo);
          }
        }
      }
      __syncthreads();
    }
  }

  // write both planes back as +-1 bytes
  for (uint32_t i = threadIdx.x; i < N; i += blockDim.x) gs[i] = (lat[i] & 1) ? (int8_t)-1 : (int8_t)1;

  if (MEASURE) {
    // E = sum over colour-1 sites of (unsatisfied - satisfied) bonds (each
    // bond once), M = sum of the spins of both colours
    int64_t Esum = 0, Msum = 0;
    for (uint32_t j = threadIdx.x; j < Nh; j += blockDim.x) {
      uint32_t o;
      const uint32_t k = site_k(lat + Nh, lat, 1u, j, o);
      Esum += 2 * (int64_t)k - 2 * D;
      Msum += (1 - 2 * (int32_t)(o & 1u)) + (1 - 2 * (int32_t)(lat[j] & 1));
    }
    __shared__ Partial part[1];
    block_partial_int(Esum, Msum, part, 0);
    if (threadIdx.x == 0) {
      ObsOut o;
      o.E_int = part[0].Ei;
      o.M_int = part[0].Mi;
      o.E = (double)part[0].Ei * dp->J0;
      o.M[0] = (double)part[0].Mi;
      o.M[1] = 0.0;
      o.M[2] = 0.0;
      o.absM = fabs((double)part[0].Mi);
      o.sweep = (int64_t)t0 + n_sweeps;
      obs[li] = o;
    }
  }
}

hipError_t launch_batch(const BatchLaunch& a, int8_t* spins, const int8_t* J, uint32_t t0,
                        uint32_t n_sweeps, void* dev_obs, hipStream_t st) {
  const dim3 grid(a.n_lattices), block(a.threads);
  const size_t lds = a.max_sites;
#define SMC_BK(DD, PMM, MM)                                                                      \
  hipLaunchKernelGGL((batch_kernel<DD, PMM, MM>), grid, block, lds, st, a.descs, a.order, a.key, \
                     spins, J, t0, n_sweeps, (ObsOut*)dev_obs)
  const bool m = dev_obs != nullptr;
  if (a.d == 2) {
    if (a.pm) { if (m) SMC_BK(2, true, true); else SMC_BK(2, true, false); }
    else { if (m) SMC_BK(2, false, true); else SMC_BK(2, false, false); }
  } else {
    if (a.pm) { if (m) SMC_BK(3, true, true); else SMC_BK(3, true, false); }
    else { if (m) SMC_BK(3, false, true); else SMC_BK(3, false, false); }
  }
#undef SMC_BK
  return hipGetLastError();
}

// Dynamic LDS beyond the default 64 KiB needs the kernels' attribute raised.
hipError_t batch_allow_lds(size_t bytes) {
  hipError_t e = hipSuccess;
#define SMC_BA(DD, PMM, MM)                                                                     \
  if (e == hipSuccess)                                                                          \
    e = hipFuncSetAttribute((const void*)batch_kernel<DD, PMM, MM>,                             \
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes)
  SMC_BA(2, true, true); SMC_BA(2, true, false); SMC_BA(2, false, true); SMC_BA(2, false, false);
  SMC_BA(3, true, true); SMC_BA(3, true, false); SMC_BA(3, false, true); SMC_BA(3, false, false);
#undef SMC_BA
  return e;
}

}  // namespace smc

namespace smc {

const void* batch_kernel_fn(int d, bool pm, bool measure) {
  if (d == 2) {
    if (pm) return measure ? (const void*)batch_kernel<2, true, true> : (const void*)batch_kernel<2, true, false>;
    return measure ? (const void*)batch_kernel<2, false, true> : (const void*)batch_kernel<2, false, false>;
  }
  if (pm) return measure ? (const void*)batch_kernel<3, true, true> : (const void*)batch_kernel<3, true, false>;
  return measure ? (const void*)batch_kernel<3, false, true> : (const void*)batch_kernel<3, false, false>;
}

}  // namespace smc
