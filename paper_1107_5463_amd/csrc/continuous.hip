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
#include "chunk.hpp"

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

// Site geometry of a row-based launch: block -> (plane row r = y + L z,
// segment), lane -> in-row index jx.  The row decomposition is a scalar
// division per block; neighbours are row offsets plus jx or jx +- 1.
struct RowSite {
  int64_t j;          // in-colour index of the site
  int64_t row_ym, row_yp, row_zm, row_zp;  // plane offsets of the neighbour rows (+ jx)
  int64_t xp, xm;     // plane offsets of the x+1 / x-1 neighbours
  int32_t jx;
};

template <int D>
__device__ __forceinline__ RowSite row_site(const Geom& g, uint32_t c, uint32_t r, int32_t jx) {
  const int32_t L = g.L, R = g.R;
  const int32_t y = (int32_t)(r % (uint32_t)L), z = (int32_t)(r / (uint32_t)L);  // uniform
  const int32_t p = (int32_t)((c + (uint32_t)y + (uint32_t)z) & 1u);
  RowSite s;
  s.jx = jx;
  const int64_t rowoff = (int64_t)r * R;
  s.j = rowoff + jx;
  // x+1 / x-1 neighbours: in-row indices jx + p and jx + p - 1 (periodic)
  const int32_t jxp = jx + p == R ? 0 : jx + p;
  const int32_t jxm = jx + p - 1 < 0 ? R - 1 : jx + p - 1;
  s.xp = rowoff + jxp;
  s.xm = rowoff + jxm;
  const int32_t ym = y == 0 ? L - 1 : y - 1, yp = y + 1 == L ? 0 : y + 1;
  s.row_ym = ((int64_t)z * L + ym) * R + jx;
  s.row_yp = ((int64_t)z * L + yp) * R + jx;
  s.row_zm = s.row_zp = 0;
  if (D == 3) {
    const int32_t zm = z == 0 ? L - 1 : z - 1, zp = z + 1 == L ? 0 : z + 1;
    s.row_zm = ((int64_t)zm * L + y) * R + jx;
    s.row_zp = ((int64_t)zp * L + y) * R + jx;
  }
  return s;
}

// Coupling of the bond from site (cc, jj) to its +mu neighbour.
template <int JK>
__device__ __forceinline__ float bond(const void* J, float J0, int64_t Nh, int mu, uint32_t cc,
                                      int64_t jj) {
  if (JK == 1) return J0 * (float)((const int8_t*)J)[((int64_t)mu * 2 + cc) * Nh + jj];
  if (JK == 2) return ((const float*)J)[((int64_t)mu * 2 + cc) * Nh + jj];
  return J0;
}

// Local field h = sum_mu [J(i,mu) s_{i+mu} + J(i-mu,mu) s_{i-mu}] in the order
// +x, -x, +y, -y, +z, -z.
template <int D, int N, int JK>
__device__ __forceinline__ void field_row(const Geom& g, const float* __restrict__ s, const void* J,
                                          float J0, uint32_t c, const RowSite& st, float h[3]) {
  const int64_t Nh = g.Nh, Nfull = 2 * Nh;
  const float* oth = s + (int64_t)(1 - c) * Nh;
  const int64_t ip[3] = {st.xp, st.row_yp, st.row_zp};
  const int64_t im[3] = {st.xm, st.row_ym, st.row_zm};
  h[0] = h[1] = h[2] = 0.0f;
#pragma unroll
  for (int mu = 0; mu < D; ++mu) {
    const float jp = bond<JK>(J, J0, Nh, mu, c, st.j);
    const float jm = bond<JK>(J, J0, Nh, mu, 1 - c, im[mu]);
#pragma unroll
    for (int k = 0; k < N; ++k) h[k] += jp * oth[k * Nfull + ip[mu]];
#pragma unroll
    for (int k = 0; k < N; ++k) h[k] += jm * oth[k * Nfull + im[mu]];
  }
}

// Blocks of 256 lanes over (row, segment); segments per row = ceil(R / (256 spt)).
__device__ __forceinline__ void row_block(uint32_t segs, uint32_t& r, uint32_t& seg) {
  const uint32_t b = xcd_remap(blockIdx.x, gridDim.x);
  r = b / segs;  // wave-uniform: scalar division
  seg = b - r * segs;
}

// XY.  PAIRED (L/2 even): a lane updates the two in-row sites (jx, jx + 1)
// that share Philox block j >> 1; otherwise one site per lane, drawing its
// words 2(j&1), 2(j&1)+1 of block j >> 1.
template <int D, int JK, bool FAST, bool PAIRED>
__global__ __launch_bounds__(256) void xy_kernel(const Geom g, const RngKey key,
                                                 const void* __restrict__ J, const float J0,
                                                 const float beta, const float delta,
                                                 const uint32_t segs, float* __restrict__ s,
                                                 const uint32_t t, const uint32_t c) {
  uint32_t r, seg;
  row_block(segs, r, seg);
  constexpr int SPL = PAIRED ? 2 : 1;  // sites per lane
  const int32_t jx0 = (int32_t)(seg * 256 * SPL + SPL * threadIdx.x);
  if (jx0 >= g.R) return;
  const int64_t Nh = g.Nh, Nfull = 2 * Nh;
  float* own = s + (int64_t)c * Nh;
  const int64_t j0 = (int64_t)r * g.R + jx0;
  const Rand4 rnd = philox((uint32_t)(j0 >> 1), t, key.replica, tag(c, kContinuous), key.k0,
                           key.k1);
#pragma unroll
  for (int half = 0; half < SPL; ++half) {
    const RowSite st = row_site<D>(g, c, r, jx0 + half);
    float h[3];
    field_row<D, 2, JK>(g, s, J, J0, c, st, h);
    const float s0 = own[st.j], s1 = own[Nfull + st.j];
    const bool odd = PAIRED ? half == 1 : (st.j & 1) != 0;
    const uint32_t wacc = odd ? rnd.w[2] : rnd.w[0];
    const uint32_t wprop = odd ? rnd.w[3] : rnd.w[1];
    const float D_ = delta * (2.0f * u01f(wprop) - 1.0f);
    float sD, cD;
    sincos_f<FAST>(D_, &sD, &cD);
    const float n0 = s0 * cD - s1 * sD;
    const float n1 = s1 * cD + s0 * sD;
    const float dE = -((n0 - s0) * h[0] + (n1 - s1) * h[1]);
    const bool accept = dE <= 0.0f || u01f(wacc) < exp_f<FAST>(-beta * dE);
    if (accept) {
      own[st.j] = n0;
      own[Nfull + st.j] = n1;
    }
  }
}

template <int D, int JK, bool FAST>
__global__ __launch_bounds__(256) void heis_kernel(const Geom g, const RngKey key,
                                                   const void* __restrict__ J, const float J0,
                                                   const float beta, const float omc,
                                                   const uint32_t segs, float* __restrict__ s,
                                                   const uint32_t t, const uint32_t c) {
  uint32_t r, seg;
  row_block(segs, r, seg);
  const int32_t jx = (int32_t)(seg * 256 + threadIdx.x);
  if (jx >= g.R) return;
  const int64_t Nh = g.Nh, Nfull = 2 * Nh;
  float* own = s + (int64_t)c * Nh;
  const RowSite st = row_site<D>(g, c, r, jx);
  const Rand4 rnd = philox((uint32_t)st.j, t, key.replica, tag(c, kContinuous), key.k0, key.k1);
  float h[3];
  field_row<D, 3, JK>(g, s, J, J0, c, st, h);
  const float sv[3] = {own[st.j], own[Nfull + st.j], own[2 * Nfull + st.j]};
  const float ca = 1.0f - u01f(rnd.w[1]) * omc;
  const float sa = sqrtf(fmaxf(0.0f, 1.0f - ca * ca));
  const float ph = 6.28318530717958647692f * u01f(rnd.w[2]);
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
  const bool accept = dE <= 0.0f || u01f(rnd.w[0]) < exp_f<FAST>(-beta * dE);
  if (accept) {
    own[st.j] = nv[0];
    own[Nfull + st.j] = nv[1];
    own[2 * Nfull + st.j] = nv[2];
  }
}

template <int D, int JK>
static hipError_t launch_cont_dj(const ContLaunch& a, float* s, uint32_t t, uint32_t c,
                                 hipStream_t st) {
  const bool paired = a.n == 2 && (a.g.R % 2) == 0;
  const uint32_t per_block = paired ? 512u : 256u;  // sites per block
  const uint32_t segs = ((uint32_t)a.g.R + per_block - 1) / per_block;
  const dim3 grid((unsigned)((uint64_t)a.g.rows * segs));
#define SMC_XY(F, P)                                                                        \
  hipLaunchKernelGGL((xy_kernel<D, JK, F, P>), grid, dim3(256), 0, st, a.g, a.key, a.J, a.J0, \
                     a.beta, a.delta, segs, s, t, c)
  if (a.n == 2) {
    if (a.fast_math) {
      if (paired) SMC_XY(true, true); else SMC_XY(true, false);
    } else {
      if (paired) SMC_XY(false, true); else SMC_XY(false, false);
    }
  } else {
    if (a.fast_math)
      hipLaunchKernelGGL((heis_kernel<D, JK, true>), grid, dim3(256), 0, st, a.g, a.key, a.J,
                         a.J0, a.beta, a.one_minus_cos_cap, segs, s, t, c);
    else
      hipLaunchKernelGGL((heis_kernel<D, JK, false>), grid, dim3(256), 0, st, a.g, a.key, a.J,
                         a.J0, a.beta, a.one_minus_cos_cap, segs, s, t, c);
  }
#undef SMC_XY
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
