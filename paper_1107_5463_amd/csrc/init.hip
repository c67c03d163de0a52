// init.hip -- initial spins and couplings drawn from the Philox contract.
//
// Draws are keyed by the natural site index i = x + L*y + L*L*z (so the
// result does not depend on the storage layout) with counter word 1 = 0 for
// spins and = mu for couplings:
//   Ising hot start   s_i = +1 if bit (i&31) of word (i>>5)&3 of block i>>7 is 0, else -1
//   XY                theta = 2 pi u(w0) of block i;  s = (cos theta, sin theta)
//   Heisenberg        z = 2 u(w0) - 1, phi = 2 pi u(w1) of block i
//   +-1 couplings     bit (i&31) of word (i>>5)&3 of block i>>7, 0 -> +1
//   Gaussian          J = J0 + sigma sqrt(-2 ln u(w0)) cos(2 pi u(w1)) of block i
// Continuous values are computed in double precision and rounded to FP32.
#include "kernels.hpp"

namespace smc {

__device__ __forceinline__ uint32_t pick(const Rand4& r, uint32_t i) {
  const uint32_t a = (i & 1) ? r.w[1] : r.w[0];
  const uint32_t b = (i & 1) ? r.w[3] : r.w[2];
  return (i & 2) ? b : a;
}

__global__ __launch_bounds__(256) void init_ising_kernel(const Geom g, const RngKey key,
                                                         const int hot, int8_t* __restrict__ s) {
  const int64_t gid = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (gid >= 2 * g.Nh) return;
  const uint32_t c = gid >= g.Nh ? 1u : 0u;
  const int64_t j = gid - (int64_t)c * g.Nh;
  int8_t v = 1;
  if (hot) {
    int32_t x, y, z;
    site_coords(g, c, j, x, y, z);
    const int64_t i = natural_index(g, x, y, z);
    const Rand4 r = philox((uint32_t)(i >> 7), 0u, key.replica, tag(0, kInitSpin), key.k0, key.k1);
    const uint32_t bit = (pick(r, (uint32_t)(i >> 5) & 3u) >> (i & 31)) & 1u;
    v = bit ? (int8_t)-1 : (int8_t)1;
  }
  s[gid] = v;
}

__global__ __launch_bounds__(256) void init_cont_kernel(const Geom g, const int n, const RngKey key,
                                                        const int hot, float* __restrict__ s) {
  const int64_t gid = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int64_t Nfull = 2 * g.Nh;
  if (gid >= Nfull) return;
  double v[3] = {1.0, 0.0, 0.0};
  if (hot) {
    const uint32_t c = gid >= g.Nh ? 1u : 0u;
    const int64_t j = gid - (int64_t)c * g.Nh;
    int32_t x, y, z;
    site_coords(g, c, j, x, y, z);
    const int64_t i = natural_index(g, x, y, z);
    const Rand4 r = philox((uint32_t)i, 0u, key.replica, tag(0, kInitSpin), key.k0, key.k1);
    const double two_pi = 6.283185307179586476925286766559;
    if (n == 2) {
      const double th = two_pi * u01d(r.w[0]);
      v[0] = cos(th);
      v[1] = sin(th);
    } else {
      const double zz = 2.0 * u01d(r.w[0]) - 1.0, ph = two_pi * u01d(r.w[1]);
      const double rr = sqrt(1.0 - zz * zz);
      v[0] = rr * cos(ph);
      v[1] = rr * sin(ph);
      v[2] = zz;
    }
  }
  for (int k = 0; k < n; ++k) s[k * Nfull + gid] = (float)v[k];
}

__global__ __launch_bounds__(256) void init_couplings_kernel(const Geom g, const int J_kind,
                                                             const RngKey key, const double J0,
                                                             const double sigma, void* __restrict__ J) {
  const int64_t gid = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int64_t Nfull = 2 * g.Nh;
  if (gid >= Nfull * g.d) return;
  const int mu = (int)(gid / Nfull);
  const int64_t rest = gid - (int64_t)mu * Nfull;
  const uint32_t c = rest >= g.Nh ? 1u : 0u;
  const int64_t j = rest - (int64_t)c * g.Nh;
  int32_t x, y, z;
  site_coords(g, c, j, x, y, z);
  const int64_t i = natural_index(g, x, y, z);
  if (J_kind == 1) {
    const Rand4 r = philox((uint32_t)(i >> 7), (uint32_t)mu, key.replica, tag(0, kCoupling), key.k0,
                           key.k1);
    const uint32_t bit = (pick(r, (uint32_t)(i >> 5) & 3u) >> (i & 31)) & 1u;
    ((int8_t*)J)[gid] = bit ? (int8_t)-1 : (int8_t)1;
  } else {
    const Rand4 r = philox((uint32_t)i, (uint32_t)mu, key.replica, tag(0, kCoupling), key.k0, key.k1);
    const double two_pi = 6.283185307179586476925286766559;
    const double gss = sqrt(-2.0 * log(u01d(r.w[0]))) * cos(two_pi * u01d(r.w[1]));
    ((float*)J)[gid] = (float)(J0 + sigma * gss);
  }
}

hipError_t launch_init_ising(const Geom& g, RngKey key, int hot, int8_t* spins, hipStream_t st) {
  const dim3 grid((unsigned)((2 * g.Nh + 255) / 256));
  hipLaunchKernelGGL(init_ising_kernel, grid, dim3(256), 0, st, g, key, hot, spins);
  return hipGetLastError();
}

hipError_t launch_init_continuous(const Geom& g, int n, RngKey key, int hot, float* spins,
                                  hipStream_t st) {
  const dim3 grid((unsigned)((2 * g.Nh + 255) / 256));
  hipLaunchKernelGGL(init_cont_kernel, grid, dim3(256), 0, st, g, n, key, hot, spins);
  return hipGetLastError();
}

hipError_t launch_init_couplings(const Geom& g, int J_kind, RngKey key, double J0, double sigma,
                                 void* J, hipStream_t st) {
  const dim3 grid((unsigned)((2 * g.Nh * g.d + 255) / 256));
  hipLaunchKernelGGL(init_couplings_kernel, grid, dim3(256), 0, st, g, J_kind, key, J0, sigma, J);
  return hipGetLastError();
}

}  // namespace smc
