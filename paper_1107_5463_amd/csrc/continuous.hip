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
#include "reduce.hpp"

namespace smc {

// Metropolis acceptance of a continuous-spin move (Eq. (2)): the accurate
// path is metropolis_fp32; fast math takes the library's __expf.
template <bool FAST>
__device__ __forceinline__ bool cont_accept(float dE, uint32_t wacc, float beta, float bl2e) {
  if (FAST) return (dE <= 0.0f) | (u01f(wacc) < __expf(-beta * dE));
  return metropolis_fp32(dE, u01f(wacc), bl2e);
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

// sin and cos of the angle 2 pi f (f in turns).  Exact quadrant reduction
// f = q/4 + r with q = rint(4 f) and |r| <= 1/8, then the Taylor series of sin
// (to x^9) and cos (to x^10) at x = 2 pi r, |x| <= pi/4, whose truncation
// errors (x^11/11! < 2e-9, x^12/12! < 2e-10) lie below FP32 rounding.
__device__ __forceinline__ void sincos_turns(float f, float* s, float* c) {
  const float q = rintf(4.0f * f);
  const float r = fmaf(-0.25f, q, f);
  const float x = 6.28318530717958647692f * r;
  const float x2 = x * x;
  float ps = fmaf(x2, 1.0f / 362880.0f, -1.0f / 5040.0f);
  ps = fmaf(x2, ps, 1.0f / 120.0f);
  ps = fmaf(x2, ps, -1.0f / 6.0f);
  const float sx = fmaf(x * x2, ps, x);
  float pc = fmaf(x2, -1.0f / 3628800.0f, 1.0f / 40320.0f);
  pc = fmaf(x2, pc, -1.0f / 720.0f);
  pc = fmaf(x2, pc, 1.0f / 24.0f);
  pc = fmaf(x2, pc, -0.5f);
  const float cx = fmaf(x2, pc, 1.0f);
  // angle = q pi/2 + x
  const int qi = (int)q & 3;
  const float a = (qi & 1) ? cx : sx;
  const float b = (qi & 1) ? sx : cx;
  *s = (qi & 2) ? -a : a;
  *c = (qi == 1 || qi == 2) ? -b : b;
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

// One XY Metropolis attempt at a site with spin (s0, s1) in field h: rotate
// by delta (2 u_prop - 1), accept iff dE <= 0 or u_acc < exp(-beta dE).
template <bool FAST>
__device__ __forceinline__ bool xy_update(float& s0, float& s1, const float h[3],
                                          const uint32_t wacc, const uint32_t wprop,
                                          const float beta, const float bl2e,
                                          const float delta) {
  // rotation angle delta (2u - 1): in radians for the hardware sin / cos of
  // the fast path, in turns for the series otherwise
  float sD, cD;
  if (FAST)
    sincos_f<true>(delta * (2.0f * u01f(wprop) - 1.0f), &sD, &cD);
  else
    sincos_turns((delta * 0.159154943091895335769f) * (2.0f * u01f(wprop) - 1.0f), &sD, &cD);
  const float n0 = s0 * cD - s1 * sD;
  const float n1 = s1 * cD + s0 * sD;
  const float dE = -((n0 - s0) * h[0] + (n1 - s1) * h[1]);
  const bool accept = cont_accept<FAST>(dE, wacc, beta, bl2e);
  if (accept) {
    s0 = n0;
    s1 = n1;
  }
  return accept;
}

// One Heisenberg Metropolis attempt: a point uniform on the cap of
// 1 - cos(theta_max) = omc around sv (w1: cos alpha, w2: azimuth), accepted
// with u_acc = u(w0).
template <bool FAST>
__device__ __forceinline__ bool heis_update(float sv[3], const float h[3], const uint32_t w0,
                                            const uint32_t w1, const uint32_t w2,
                                            const float beta, const float bl2e,
                                            const float omc) {
  // sin alpha from 1 - cos alpha directly: (1 - c)(1 + c) keeps its relative
  // precision for small caps, where 1 - c^2 would cancel.  The argument is at
  // least omc 2^-24 (a normal number), so the hardware square root (about one
  // ulp) needs no denormal scaling.
  const float omca = u01f(w1) * omc;
  const float ca = 1.0f - omca;
  const float sa = __builtin_amdgcn_sqrtf(omca * (2.0f - omca));
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
  const float inv = rsqrtf(e1[0] * e1[0] + e1[1] * e1[1] + e1[2] * e1[2]);
  e1[0] *= inv; e1[1] *= inv; e1[2] *= inv;
  const float e2[3] = {sv[1] * e1[2] - sv[2] * e1[1], sv[2] * e1[0] - sv[0] * e1[2],
                       sv[0] * e1[1] - sv[1] * e1[0]};
  // azimuth 2 pi u(w2)
  float sph, cph;
  if (FAST)
    sincos_f<true>(6.28318530717958647692f * u01f(w2), &sph, &cph);
  else
    sincos_turns(u01f(w2), &sph, &cph);
  float nv[3];
#pragma unroll
  for (int q = 0; q < 3; ++q) nv[q] = ca * sv[q] + sa * (cph * e1[q] + sph * e2[q]);
  const float dE = -((nv[0] - sv[0]) * h[0] + (nv[1] - sv[1]) * h[1] + (nv[2] - sv[2]) * h[2]);
  const bool accept = cont_accept<FAST>(dE, w0, beta, bl2e);
  if (accept) {
    sv[0] = nv[0];
    sv[1] = nv[1];
    sv[2] = nv[2];
  }
  return accept;
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
    float s0 = own[st.j], s1 = own[Nfull + st.j];
    const bool odd = PAIRED ? half == 1 : (st.j & 1) != 0;
    if (xy_update<FAST>(s0, s1, h, odd ? rnd.w[2] : rnd.w[0], odd ? rnd.w[3] : rnd.w[1], beta,
                        beta_log2e(beta), delta)) {
      own[st.j] = s0;
      own[Nfull + st.j] = s1;
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
  float sv[3] = {own[st.j], own[Nfull + st.j], own[2 * Nfull + st.j]};
  if (heis_update<FAST>(sv, h, rnd.w[0], rnd.w[1], rnd.w[2], beta, beta_log2e(beta), omc)) {
    own[st.j] = sv[0];
    own[Nfull + st.j] = sv[1];
    own[2 * Nfull + st.j] = sv[2];
  }
}

// Streaming variant (the layout of the int8 streaming kernel with FP32
// components): a lane owns V consecutive in-row sites of one colour and walks
// a band of H plane rows at fixed z, keeping the other colour's rows y - 1,
// y, y + 1 (and the z-neighbour rows) in registers, so each row of either
// plane crosses HBM about once per half-sweep.  The x-neighbour beyond the
// lane's V sites (the "edge" element: the next group's first site for row
// parity 1, the previous group's last for parity 0) is one extra element per
// row and component.  Field order, random words and update arithmetic are
// those of the row kernels.  Requires R % V == 0, H % 4 == 0, L % H == 0.
// Plane accesses take a wave-uniform plane base and a 32-bit byte offset
// (planes below 4 GiB), which maps onto the scalar-base + vector-offset
// addressing of global loads and stores.
__device__ __forceinline__ const float* at(const float* base, uint32_t idx) {
  return reinterpret_cast<const float*>(reinterpret_cast<const char*>(base) + (idx << 2));
}
__device__ __forceinline__ float* at(float* base, uint32_t idx) {
  return reinterpret_cast<float*>(reinterpret_cast<char*>(base) + (idx << 2));
}
template <int V>
__device__ __forceinline__ void ldv(const float* base, uint32_t idx, float* o) {
  if (V == 4) {
    const float4 v = *reinterpret_cast<const float4*>(at(base, idx));
    o[0] = v.x; o[1] = v.y; o[2] = v.z; o[3] = v.w;
  } else if (V == 1) {
    o[0] = *at(base, idx);
  } else {
    const float2 v = *reinterpret_cast<const float2*>(at(base, idx));
    o[0] = v.x; o[1] = v.y;
  }
}
template <int V>
__device__ __forceinline__ void stv(float* base, uint32_t idx, const float* o) {
  if (V == 4)
    *reinterpret_cast<float4*>(at(base, idx)) = make_float4(o[0], o[1], o[2], o[3]);
  else if (V == 1)
    *at(base, idx) = o[0];
  else
    *reinterpret_cast<float2*>(at(base, idx)) = make_float2(o[0], o[1]);
}

// MEASURE (colour 1 only): each lane also sums, in FP64, the energy of the
// bonds of its updated sites and the magnetisation of its sites plus the
// colour-0 sites at the same positions (the per-site formula of the
// measurement kernel); block sums go to parts[block].
// V sites per lane: XY 4 or 2 (a lane holds whole Philox blocks of two
// sites), Heisenberg 2 or 1.
template <int D, int N, int JK, bool FAST, bool MEASURE, int V>
__global__ __launch_bounds__(256) void cont_stream_kernel(
    const Geom g, const RngKey key, const void* __restrict__ J, const float J0, const float beta,
    const float param, const FastDiv divQ, const FastDiv divL, const uint32_t H,
    const uint32_t nbands, float* __restrict__ s, const uint32_t t, const uint32_t c,
    const double J0d, Partial* __restrict__ parts) {
  static_assert(N == 2 ? (V == 2 || V == 4) : (V == 1 || V == 2), "sites per lane");
  const float bl2e = beta_log2e(beta);
  const uint32_t tid = xcd_remap(blockIdx.x, gridDim.x) * 256u + threadIdx.x;
  const uint32_t band = fdiv(tid, divQ);
  double Esum = 0.0, Msum[3] = {0.0, 0.0, 0.0};
  if (band < nbands) {
  const uint32_t Q = divQ.d;
  const uint32_t q = tid - band * Q;
  const uint32_t L = (uint32_t)g.L, R = (uint32_t)g.R;
  const uint32_t r0 = band * H;
  uint32_t z = 0, y0 = r0;
  if (D == 3) {
    z = fdiv(r0, divL);
    y0 = r0 - z * L;
  }
  const int64_t Nh = g.Nh, Nfull = 2 * Nh;
  float* own[N];
  const float* oth[N];
#pragma unroll
  for (int m = 0; m < N; ++m) {
    own[m] = s + (int64_t)m * Nfull + (int64_t)c * Nh;
    oth[m] = s + (int64_t)m * Nfull + (int64_t)(1 - c) * Nh;
  }
  const uint32_t col = V * q;
  const uint32_t zrow = L * z;
  const uint32_t pz = (c + z) & 1u;  // row parity of y even
  const uint32_t e_next = q + 1 == Q ? 0u : col + V;
  const uint32_t e_prev = q == 0 ? R - 1 : col - 1;
  const uint32_t edge_even = pz ? e_next : e_prev;
  const uint32_t edge_odd = pz ? e_prev : e_next;
  auto roff = [&](uint32_t y) -> uint32_t { return (zrow + (y >= L ? y - L : y)) * R; };
  uint32_t zm_row = 0, zp_row = 0;
  if (D == 3) {
    zm_row = L * (z == 0 ? L - 1 : z - 1);
    zp_row = L * (z + 1 == L ? 0 : z + 1);
  }
  auto zoff = [&](uint32_t zr, uint32_t y) -> uint32_t {
    return (zr + (y >= L ? y - L : y)) * R + col;
  };
  // ring buffers as in the int8 streaming kernel: Ro[y & 3] other row y,
  // Ow / Ed / Fz / Bz [y & 1] own row y, its edge element, its z-neighbours
  float Ro[4][N][V], Ow[2][N][V], Ed[2][N], Fz[2][N][V], Bz[2][N][V];
  const uint32_t ym1 = y0 == 0 ? L - 1 : y0 - 1;
#pragma unroll
  for (int m = 0; m < N; ++m) {
    ldv<V>(oth[m], roff(ym1) + col, Ro[3][m]);
    ldv<V>(oth[m], roff(y0) + col, Ro[0][m]);
    ldv<V>(oth[m], roff(y0 + 1) + col, Ro[1][m]);
    ldv<V>(oth[m], roff(y0 + 2) + col, Ro[2][m]);
    ldv<V>(own[m], roff(y0) + col, Ow[0][m]);
    ldv<V>(own[m], roff(y0 + 1) + col, Ow[1][m]);
    Ed[0][m] = *at(oth[m], roff(y0) + edge_even);
    Ed[1][m] = *at(oth[m], roff(y0 + 1) + edge_odd);
    if (D == 3) {
      ldv<V>(oth[m], zoff(zm_row, y0), Fz[0][m]);
      ldv<V>(oth[m], zoff(zm_row, y0 + 1), Fz[1][m]);
      ldv<V>(oth[m], zoff(zp_row, y0), Bz[0][m]);
      ldv<V>(oth[m], zoff(zp_row, y0 + 1), Bz[1][m]);
    }
  }
  // 3D: plane offsets of the rows the loop touches, stepped by R per row (a
  // row past L - 1 wraps to row 0 of its z-plane) -- row y, y - 1, y + 2,
  // y + 3, and the z - 1 / z + 1 planes' rows y and y + 2 -- instead of a
  // multiply per row and stream (in 2D the running offsets cost more
  // registers than the multiplies cost issue slots)
  constexpr bool STEP = D == 3;
  const uint32_t zR = zrow * R, zmR = zm_row * R, zpR = zp_row * R;
  auto step = [&](uint32_t off, uint32_t yy, uint32_t base) -> uint32_t {
    return yy + 1 == L ? base : off + R;
  };
  uint32_t ry = roff(y0), rym = roff(ym1), ry2 = roff(y0 + 2), ry3 = roff(y0 + 3);
  uint32_t zm0 = zoff(zm_row, y0) - col, zm2 = zoff(zm_row, y0 + 2) - col;
  uint32_t zp2 = zoff(zp_row, y0 + 2) - col;
  for (uint32_t i = 0; i < H; i += 4) {
#pragma unroll
    for (int ph = 0; ph < 4; ++ph) {
      const uint32_t y = y0 + i + ph;  // y0 and i are multiples of 4
      const bool p = ((pz + (uint32_t)ph) & 1u) != 0;
      const uint32_t rowoff = STEP ? ry : roff(y);
      const uint32_t jrow = rowoff + col;
      const int up = (ph + 3) & 3, ct = ph, dn = (ph + 1) & 3, b = ph & 1;
      Rand4 rnd[N == 2 ? V / 2 : V];
#pragma unroll
      for (int k = 0; k < (N == 2 ? V / 2 : V); ++k)
        rnd[k] = philox(N == 2 ? (jrow >> 1) + k : jrow + k, t, key.replica, tag(c, kContinuous),
                        key.k0, key.k1);
#pragma unroll
      for (int k = 0; k < V; ++k) {
        const uint32_t j = jrow + k;
        float h[3] = {0.0f, 0.0f, 0.0f};
        float jp = J0, jm = J0;
        // +x, -x
        if (JK != 0) {
          const uint32_t xm = p ? col + k : (k > 0 ? col + k - 1 : e_prev);
          jp = bond<JK>(J, J0, Nh, 0, c, j);
          jm = bond<JK>(J, J0, Nh, 0, 1 - c, rowoff + xm);
        }
#pragma unroll
        for (int m = 0; m < N; ++m) {
          const float vp = p ? (k + 1 < V ? Ro[ct][m][(k + 1) % V] : Ed[b][m]) : Ro[ct][m][k];
          h[m] += jp * vp;
        }
#pragma unroll
        for (int m = 0; m < N; ++m) {
          const float vm = p ? Ro[ct][m][k] : (k > 0 ? Ro[ct][m][(k + V - 1) % V] : Ed[b][m]);
          h[m] += jm * vm;
        }
        // +y, -y
        if (JK != 0) {
          jp = bond<JK>(J, J0, Nh, 1, c, j);
          jm = bond<JK>(J, J0, Nh, 1, 1 - c, (STEP ? rym : roff(y + L - 1)) + col + k);
        }
#pragma unroll
        for (int m = 0; m < N; ++m) h[m] += jp * Ro[dn][m][k];
#pragma unroll
        for (int m = 0; m < N; ++m) h[m] += jm * Ro[up][m][k];
        if (D == 3) {
          if (JK != 0) {
            jp = bond<JK>(J, J0, Nh, 2, c, j);
            jm = bond<JK>(J, J0, Nh, 2, 1 - c, zm0 + col + k);
          }
#pragma unroll
          for (int m = 0; m < N; ++m) h[m] += jp * Bz[b][m][k];
#pragma unroll
          for (int m = 0; m < N; ++m) h[m] += jm * Fz[b][m][k];
        }
        if (N == 2) {
          const Rand4& rw = rnd[k >> 1];
          xy_update<FAST>(Ow[b][0][k], Ow[b][1][k], h, (k & 1) ? rw.w[2] : rw.w[0],
                          (k & 1) ? rw.w[3] : rw.w[1], beta, bl2e, param);
        } else {
          float sv[3] = {Ow[b][0][k], Ow[b][1][k], Ow[b][2][k]};
          heis_update<FAST>(sv, h, rnd[k].w[0], rnd[k].w[1], rnd[k].w[2], beta, bl2e, param);
          Ow[b][0][k] = sv[0];
          Ow[b][1][k] = sv[1];
          Ow[b][2][k] = sv[2];
        }
      }
#pragma unroll
      for (int m = 0; m < N; ++m) stv<V>(own[m], jrow, Ow[b][m]);
      if (MEASURE) {
#pragma unroll
        for (int k = 0; k < V; ++k) {
          const uint32_t j = jrow + k;
          double si[3] = {0.0, 0.0, 0.0};
#pragma unroll
          for (int m = 0; m < N; ++m) si[m] = (double)Ow[b][m][k];
          double e = 0.0;
#pragma unroll
          for (int mu = 0; mu < D; ++mu) {
            double dp = 0.0, dm = 0.0;
#pragma unroll
            for (int m = 0; m < N; ++m) {
              float vp, vm;
              if (mu == 0) {
                vp = p ? (k + 1 < V ? Ro[ct][m][(k + 1) % V] : Ed[b][m]) : Ro[ct][m][k];
                vm = p ? Ro[ct][m][k] : (k > 0 ? Ro[ct][m][(k + V - 1) % V] : Ed[b][m]);
              } else if (mu == 1) {
                vp = Ro[dn][m][k];
                vm = Ro[up][m][k];
              } else {
                vp = Bz[b][m][k];
                vm = Fz[b][m][k];
              }
              dp += si[m] * (double)vp;
              dm += si[m] * (double)vm;
            }
            double jp = J0d, jm = J0d;
            if (JK != 0) {
              uint32_t im;
              if (mu == 0) im = rowoff + (p ? col + k : (k > 0 ? col + k - 1 : e_prev));
              else if (mu == 1) im = (STEP ? rym : roff(y + L - 1)) + col + k;
              else im = zm0 + col + k;
              if (JK == 1) {
                const int8_t* Jb = (const int8_t*)J;
                jp = J0d * Jb[((int64_t)mu * 2 + 1) * Nh + j];
                jm = J0d * Jb[((int64_t)mu * 2 + 0) * Nh + im];
              } else {
                const float* Jf = (const float*)J;
                jp = Jf[((int64_t)mu * 2 + 1) * Nh + j];
                jm = Jf[((int64_t)mu * 2 + 0) * Nh + im];
              }
            }
            e -= jp * dp + jm * dm;
          }
          Esum += e;
#pragma unroll
          for (int m = 0; m < N; ++m) Msum[m] += si[m] + (double)Ro[ct][m][k];
        }
      }
      // refill the dead slots: other row y + 3, own row y + 2 with its edge
      // element and z-neighbours (rows past the band are read, never used)
#pragma unroll
      for (int m = 0; m < N; ++m) {
        const uint32_t r3 = STEP ? ry3 : roff(y + 3), r2 = STEP ? ry2 : roff(y + 2);
        ldv<V>(oth[m], r3 + col, Ro[up][m]);
        ldv<V>(own[m], r2 + col, Ow[b][m]);
        Ed[b][m] = *at(oth[m], r2 + (b ? edge_odd : edge_even));
        if (D == 3) {
          ldv<V>(oth[m], zm2 + col, Fz[b][m]);
          ldv<V>(oth[m], zp2 + col, Bz[b][m]);
        }
      }
      rym = ry;
      ry = step(ry, y, zR);
      ry2 = ry3;
      ry3 = step(ry3, y + 3, zR);
      zm0 = step(zm0, y, zmR);
      zm2 = step(zm2, y + 2, zmR);
      zp2 = step(zp2, y + 2, zpR);
    }
  }
  }
  if (MEASURE) {
    Partial v{0, 0, Esum, {Msum[0], Msum[1], Msum[2]}};
    block_partial(v, parts);
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

template <int D, int JK>
static hipError_t launch_cont_stream(const ContLaunch& a, float* s, uint32_t t, uint32_t c,
                                     hipStream_t st, void* partials = nullptr,
                                     int64_t* nparts = nullptr) {
  const uint32_t H = a.rows_per_band;
  const uint32_t nbands = (uint32_t)a.g.rows / H;
  const uint64_t threads = (uint64_t)nbands * a.divQ.d;
  const dim3 grid((unsigned)((threads + 255) / 256));
  const float param = a.n == 2 ? a.delta : a.one_minus_cos_cap;
  const bool meas = partials != nullptr;
  if (meas && nparts) *nparts = grid.x;
#define SMC_CS(N, F, M, V)                                                                         \
  hipLaunchKernelGGL((cont_stream_kernel<D, N, JK, F, M, V>), grid, dim3(256), 0, st, a.g, a.key,  \
                     a.J, a.J0, a.beta, param, a.divQ, a.divL, H, nbands, s, t, c, a.J0d,           \
                     (Partial*)partials)
#define SMC_CSV(N, V)                                                 \
  do {                                                                \
    if (meas) { if (a.fast_math) SMC_CS(N, true, true, V); else SMC_CS(N, false, true, V); } \
    else { if (a.fast_math) SMC_CS(N, true, false, V); else SMC_CS(N, false, false, V); }   \
  } while (0)
  if (a.n == 2) {
    if (a.sites_per_lane == 2) SMC_CSV(2, 2); else SMC_CSV(2, 4);
  } else {
    if (a.sites_per_lane == 1) SMC_CSV(3, 1); else SMC_CSV(3, 2);
  }
#undef SMC_CSV
#undef SMC_CS
  return hipGetLastError();
}

uint32_t cont_default_sites_per_lane(int n) { return n == 2 ? 4u : 2u; }

bool cont_sites_per_lane_ok(int n, uint32_t V) {
  return n == 2 ? (V == 2 || V == 4) : (V == 1 || V == 2);
}

bool cont_stream_supported(const Geom& g, uint32_t V, uint32_t H) {
  return V >= 1 && (uint32_t)g.R % V == 0 && H >= 4 && H % 4 == 0 && (uint32_t)g.L % H == 0 &&
         g.Nh < ((int64_t)1 << 30);  // 32-bit byte offsets within a plane
}

// Band height of the streaming kernel: the largest divisor of L up to 64 that
// still gives at least `min_waves` waves.
uint32_t cont_rows_per_band(const Geom& g, uint32_t V, uint32_t min_waves) {
  const uint32_t Q = (uint32_t)g.R / V;
  uint32_t best = 4;
  for (uint32_t H = 4; H <= 64; H *= 2) {
    if (g.L % H) break;
    const uint64_t waves = (uint64_t)Q * (uint64_t)(g.rows / H) / 64;
    if (waves >= min_waves) best = H;
  }
  return best;
}

int cont_variant_used(const ContLaunch& a) {
  if (a.variant == kContRow) return kContRow;
  return cont_stream_supported(a.g, a.sites_per_lane, a.rows_per_band) ? kContStream : kContRow;
}

template <int D>
static hipError_t launch_cont_d(const ContLaunch& a, float* s, uint32_t t, uint32_t c,
                                hipStream_t st) {
  const bool stream = cont_variant_used(a) == kContStream;
  switch (a.J_kind) {
    case 0: return stream ? launch_cont_stream<D, 0>(a, s, t, c, st) : launch_cont_dj<D, 0>(a, s, t, c, st);
    case 1: return stream ? launch_cont_stream<D, 1>(a, s, t, c, st) : launch_cont_dj<D, 1>(a, s, t, c, st);
    default: return stream ? launch_cont_stream<D, 2>(a, s, t, c, st) : launch_cont_dj<D, 2>(a, s, t, c, st);
  }
}

hipError_t launch_cont_half_sweep(const ContLaunch& a, float* spins, uint32_t t, uint32_t colour,
                                  hipStream_t st) {
  return a.g.d == 2 ? launch_cont_d<2>(a, spins, t, colour, st)
                    : launch_cont_d<3>(a, spins, t, colour, st);
}

bool cont_half_sweep_measured(const ContLaunch& a, float* spins, uint32_t t, void* partials,
                              int64_t* nparts, hipStream_t st, hipError_t* err) {
  if (cont_variant_used(a) != kContStream) return false;
  if (a.g.d == 2) {
    *err = a.J_kind == 0 ? launch_cont_stream<2, 0>(a, spins, t, 1u, st, partials, nparts)
         : a.J_kind == 1 ? launch_cont_stream<2, 1>(a, spins, t, 1u, st, partials, nparts)
                         : launch_cont_stream<2, 2>(a, spins, t, 1u, st, partials, nparts);
  } else {
    *err = a.J_kind == 0 ? launch_cont_stream<3, 0>(a, spins, t, 1u, st, partials, nparts)
         : a.J_kind == 1 ? launch_cont_stream<3, 1>(a, spins, t, 1u, st, partials, nparts)
                         : launch_cont_stream<3, 2>(a, spins, t, 1u, st, partials, nparts);
  }
  return true;
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
