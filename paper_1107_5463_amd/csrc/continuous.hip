// continuous.hip -- checkerboard Metropolis half-sweeps for XY (n = 2) and
// Heisenberg (n = 3) spins stored as FP32 unit vectors (Sec. 2: spins in
// single precision, aggregates in double).
//
// Proposal: XY rotates s by Delta = delta (2u - 1); Heisenberg picks a point
// uniformly on the spherical cap of half-angle theta_max around s (cos alpha
// = 1 - u (1 - cos theta_max), azimuth 2 pi u' in the frame e1 = normalised
// (e_k - s_k s) with k the component of smallest magnitude, e2 = s x e1).
// Acceptance (Eq. (2)): dE = -(s' - s) . h, accept iff dE <= 0 or
// u_acc < exp(-beta dE).  The random words come from Philox blocks keyed by
// (seed, t, replica, colour): XY block j>>1 words 2(j&1) (accept) and
// 2(j&1)+1 (proposal); Heisenberg block j words 0 (accept), 1, 2.  An XY
// thread updates the two sites of one block.
#include "kernels.hpp"

namespace smc {

template <bool FAST>
__device__ __forceinline__ float exp_f(float x) {
  return FAST ? __expf(x) : expf(x);
}
template <bool FAST>
__device__ __forceinline__ void sincos_f(float x, float* s, float* c) {
  if (FAST) {
    *s = __sinf(x);
    *c = __cosf(x);
  } else {
    sincosf(x, s, c);
  }
}

// Local field h = sum_mu [J(i,mu) s_{i+mu} + J(i-mu,mu) s_{i-mu}] in the order
// +x, -x, +y, -y, +z, -z.
template <int D, int N, int JK>
__device__ __forceinline__ void field(const Geom& g, const float* __restrict__ s, const void* J,
                                      float J0, uint32_t c, int64_t j, int32_t x, int32_t y,
                                      int32_t z, float h[3]) {
  const int64_t Nh = g.Nh, Nfull = 2 * Nh;
  const float* oth = s + (int64_t)(1 - c) * Nh;
  h[0] = h[1] = h[2] = 0.0f;
#pragma unroll
  for (int mu = 0; mu < D; ++mu) {
    int32_t xp = x, yp = y, zp = z, xm = x, ym = y, zm = z;
    if (mu == 0) { xp = wrap(x + 1, g.L); xm = wrap(x - 1, g.L); }
    if (mu == 1) { yp = wrap(y + 1, g.L); ym = wrap(y - 1, g.L); }
    if (mu == 2) { zp = wrap(z + 1, g.L); zm = wrap(z - 1, g.L); }
    const int64_t ip = plane_index(g, xp, yp, zp);
    const int64_t im = plane_index(g, xm, ym, zm);
    float jp = J0, jm = J0;
    if (JK == 1) {
      const int8_t* Jb = (const int8_t*)J;
      jp = J0 * (float)Jb[((int64_t)mu * 2 + c) * Nh + j];
      jm = J0 * (float)Jb[((int64_t)mu * 2 + (1 - c)) * Nh + im];
    } else if (JK == 2) {
      const float* Jf = (const float*)J;
      jp = Jf[((int64_t)mu * 2 + c) * Nh + j];
      jm = Jf[((int64_t)mu * 2 + (1 - c)) * Nh + im];
    }
#pragma unroll
    for (int k = 0; k < N; ++k) h[k] += jp * oth[k * Nfull + ip];
#pragma unroll
    for (int k = 0; k < N; ++k) h[k] += jm * oth[k * Nfull + im];
  }
}

template <int D, int JK, bool FAST>
__global__ __launch_bounds__(256) void xy_kernel(const Geom g, const RngKey key,
                                                 const void* __restrict__ J, const float J0,
                                                 const float beta, const float delta,
                                                 float* __restrict__ s, const uint32_t t,
                                                 const uint32_t c) {
  const int64_t pair = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int64_t Nh = g.Nh, Nfull = 2 * Nh;
  if (2 * pair >= Nh) return;
  const Rand4 r = philox((uint32_t)pair, t, key.replica, tag(c, kContinuous), key.k0, key.k1);
  float* own = s + (int64_t)c * Nh;
#pragma unroll
  for (int half = 0; half < 2; ++half) {
    const int64_t j = 2 * pair + half;
    if (j >= Nh) break;
    int32_t x, y, z;
    site_coords(g, c, j, x, y, z);
    float h[3];
    field<D, 2, JK>(g, s, J, J0, c, j, x, y, z, h);
    const float s0 = own[j], s1 = own[Nfull + j];
    const uint32_t wacc = half ? r.w[2] : r.w[0];
    const uint32_t wprop = half ? r.w[3] : r.w[1];
    const float D_ = delta * (2.0f * u01f(wprop) - 1.0f);
    float sD, cD;
    sincos_f<FAST>(D_, &sD, &cD);
    const float n0 = s0 * cD - s1 * sD;
    const float n1 = s1 * cD + s0 * sD;
    const float dE = -((n0 - s0) * h[0] + (n1 - s1) * h[1]);
    const bool accept = dE <= 0.0f || u01f(wacc) < exp_f<FAST>(-beta * dE);
    if (accept) {
      own[j] = n0;
      own[Nfull + j] = n1;
    }
  }
}

template <int D, int JK, bool FAST>
__global__ __launch_bounds__(256) void heis_kernel(const Geom g, const RngKey key,
                                                   const void* __restrict__ J, const float J0,
                                                   const float beta, const float omc,
                                                   float* __restrict__ s, const uint32_t t,
                                                   const uint32_t c) {
  const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int64_t Nh = g.Nh, Nfull = 2 * Nh;
  if (j >= Nh) return;
  const Rand4 r = philox((uint32_t)j, t, key.replica, tag(c, kContinuous), key.k0, key.k1);
  float* own = s + (int64_t)c * Nh;
  int32_t x, y, z;
  site_coords(g, c, j, x, y, z);
  float h[3];
  field<D, 3, JK>(g, s, J, J0, c, j, x, y, z, h);
  const float sv[3] = {own[j], own[Nfull + j], own[2 * Nfull + j]};
  const float ca = 1.0f - u01f(r.w[1]) * omc;
  const float sa = sqrtf(fmaxf(0.0f, 1.0f - ca * ca));
  const float ph = 6.28318530717958647692f * u01f(r.w[2]);
  // frame axis: smallest |s_k|, lowest k on ties
  const float a0 = fabsf(sv[0]), a1 = fabsf(sv[1]), a2 = fabsf(sv[2]);
  int k = 0;
  float am = a0;
  if (a1 < am) { k = 1; am = a1; }
  if (a2 < am) { k = 2; }
  const float sk = k == 0 ? sv[0] : (k == 1 ? sv[1] : sv[2]);
  float e1[3] = {-sk * sv[0], -sk * sv[1], -sk * sv[2]};
  if (k == 0) e1[0] += 1.0f;
  if (k == 1) e1[1] += 1.0f;
  if (k == 2) e1[2] += 1.0f;
  const float inv = 1.0f / sqrtf(e1[0] * e1[0] + e1[1] * e1[1] + e1[2] * e1[2]);
  e1[0] *= inv; e1[1] *= inv; e1[2] *= inv;
  const float e2[3] = {sv[1] * e1[2] - sv[2] * e1[1], sv[2] * e1[0] - sv[0] * e1[2],
                       sv[0] * e1[1] - sv[1] * e1[0]};
  float sph, cph;
  sincos_f<FAST>(ph, &sph, &cph);
  float nv[3];
#pragma unroll
  for (int q = 0; q < 3; ++q) nv[q] = ca * sv[q] + sa * (cph * e1[q] + sph * e2[q]);
  const float dE = -((nv[0] - sv[0]) * h[0] + (nv[1] - sv[1]) * h[1] + (nv[2] - sv[2]) * h[2]);
  const bool accept = dE <= 0.0f || u01f(r.w[0]) < exp_f<FAST>(-beta * dE);
  if (accept) {
    own[j] = nv[0];
    own[Nfull + j] = nv[1];
    own[2 * Nfull + j] = nv[2];
  }
}

template <int D, int JK>
static hipError_t launch_cont_dj(const ContLaunch& a, float* s, uint32_t t, uint32_t c,
                                 hipStream_t st) {
  if (a.n == 2) {
    const int64_t pairs = (a.g.Nh + 1) / 2;
    const dim3 grid((unsigned)((pairs + 255) / 256));
    if (a.fast_math)
      hipLaunchKernelGGL((xy_kernel<D, JK, true>), grid, dim3(256), 0, st, a.g, a.key, a.J, a.J0,
                         a.beta, a.delta, s, t, c);
    else
      hipLaunchKernelGGL((xy_kernel<D, JK, false>), grid, dim3(256), 0, st, a.g, a.key, a.J,
                         a.J0, a.beta, a.delta, s, t, c);
  } else {
    const dim3 grid((unsigned)((a.g.Nh + 255) / 256));
    if (a.fast_math)
      hipLaunchKernelGGL((heis_kernel<D, JK, true>), grid, dim3(256), 0, st, a.g, a.key, a.J,
                         a.J0, a.beta, a.one_minus_cos_cap, s, t, c);
    else
      hipLaunchKernelGGL((heis_kernel<D, JK, false>), grid, dim3(256), 0, st, a.g, a.key, a.J,
                         a.J0, a.beta, a.one_minus_cos_cap, s, t, c);
  }
  return hipGetLastError();
}

template <int D>
static hipError_t launch_cont_d(const ContLaunch& a, float* s, uint32_t t, uint32_t c,
                                hipStream_t st) {
  switch (a.J_kind) {
    case 0: return launch_cont_dj<D, 0>(a, s, t, c, st);
    case 1: return launch_cont_dj<D, 1>(a, s, t, c, st);
    default: return launch_cont_dj<D, 2>(a, s, t, c, st);
  }
}

hipError_t launch_cont_half_sweep(const ContLaunch& a, float* spins, uint32_t t, uint32_t colour,
                                  hipStream_t st) {
  return a.g.d == 2 ? launch_cont_d<2>(a, spins, t, colour, st)
                    : launch_cont_d<3>(a, spins, t, colour, st);
}

template <int N>
__global__ __launch_bounds__(256) void renorm_kernel(const int64_t Nfull, float* __restrict__ s) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= Nfull) return;
  float v[N];
  float q = 0.0f;
#pragma unroll
  for (int k = 0; k < N; ++k) {
    v[k] = s[k * Nfull + i];
    q += v[k] * v[k];
  }
  const float inv = 1.0f / sqrtf(q);
#pragma unroll
  for (int k = 0; k < N; ++k) s[k * Nfull + i] = v[k] * inv;
}

hipError_t launch_renormalize(const Geom& g, int n, float* spins, hipStream_t st) {
  const int64_t Nfull = 2 * g.Nh;
  const dim3 grid((unsigned)((Nfull + 255) / 256));
  if (n == 2)
    hipLaunchKernelGGL(renorm_kernel<2>, grid, dim3(256), 0, st, Nfull, spins);
  else
    hipLaunchKernelGGL(renorm_kernel<3>, grid, dim3(256), 0, st, Nfull, spins);
  return hipGetLastError();
}

}  // namespace smc
