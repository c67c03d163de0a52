// chunk.hpp -- 16-byte chunks of same-colour int8 Ising spins (internal).
// A chunk holds 16 consecutive sites of one plane row; four sites per 32-bit
// word, site 4w+b in byte b of word w.
#pragma once

#include "kernels.hpp"

namespace smc {

__device__ __forceinline__ uint32_t fdiv(uint32_t n, const FastDiv& f) {
  if (f.d == 1) return n;
  const uint32_t hi = __umulhi(f.m, n);
  return (hi + ((n - hi) >> 1)) >> f.s;
}

struct Chunk {
  uint32_t w[4];
};

__device__ __forceinline__ Chunk ld16(const int8_t* p) {
  const uint4 v = *reinterpret_cast<const uint4*>(p);
  Chunk c;
  c.w[0] = v.x; c.w[1] = v.y; c.w[2] = v.z; c.w[3] = v.w;
  return c;
}

__device__ __forceinline__ void st16(int8_t* p, const uint32_t w[4]) {
  *reinterpret_cast<uint4*>(p) = make_uint4(w[0], w[1], w[2], w[3]);
}

// chunk of the neighbours at jx + 1: byte b <- byte b+1, byte 15 <- edge byte 0
__device__ __forceinline__ Chunk shift_next(const Chunk& c, uint32_t edge) {
  Chunk o;
  o.w[0] = __builtin_amdgcn_alignbyte(c.w[1], c.w[0], 1);
  o.w[1] = __builtin_amdgcn_alignbyte(c.w[2], c.w[1], 1);
  o.w[2] = __builtin_amdgcn_alignbyte(c.w[3], c.w[2], 1);
  o.w[3] = __builtin_amdgcn_alignbyte(edge, c.w[3], 1);
  return o;
}

// chunk of the neighbours at jx - 1: byte b <- byte b-1, byte 0 <- edge byte 3
__device__ __forceinline__ Chunk shift_prev(const Chunk& c, uint32_t edge) {
  Chunk o;
  o.w[0] = __builtin_amdgcn_alignbyte(c.w[0], edge, 3);
  o.w[1] = __builtin_amdgcn_alignbyte(c.w[1], c.w[0], 3);
  o.w[2] = __builtin_amdgcn_alignbyte(c.w[2], c.w[1], 3);
  o.w[3] = __builtin_amdgcn_alignbyte(c.w[3], c.w[2], 3);
  return o;
}

constexpr uint32_t kBit1 = 0x02020202u;  // bit 1 of a +-1 byte: set for -1
constexpr uint32_t kHigh = 0x80808080u;
constexpr uint32_t kOnes = 0x01010101u;


// Unsatisfied-bond counts of the 16 sites of chunk gid of colour c: byte b of
// kk[w] = number of bonds of site 4w+b with J_b s_i s_b < 0.  Also returns the
// chunk's plane offset, its spins and the other colour's chunk at the same
// position (the colour-0 partner used by the measurement).
template <int D, bool PM>
__device__ __forceinline__ void chunk_counts(const Geom& g, const int8_t* __restrict__ s,
                                             const int8_t* __restrict__ J, const FastDiv& divQ,
                                             const FastDiv& divL, uint32_t c, uint32_t gid,
                                             int64_t& base, Chunk& o, Chunk& ctr, uint32_t kk[4]) {
  const uint32_t Q = divQ.d;
  const uint32_t L = (uint32_t)g.L;
  const uint32_t r = fdiv(gid, divQ);
  const uint32_t q = gid - r * Q;
  uint32_t y = r, z = 0;
  if (D == 3) {
    z = fdiv(r, divL);
    y = r - z * L;
  }
  const uint32_t p = (c + y + z) & 1u;
  const int64_t Nh = g.Nh;
  const int64_t R = g.R;
  const int8_t* own = s + (int64_t)c * Nh;
  const int8_t* oth = s + (int64_t)(1 - c) * Nh;
  base = (int64_t)r * R + 16 * (int64_t)q;
  const uint32_t qe = p ? (q + 1 == Q ? 0u : q + 1) : (q == 0 ? Q - 1 : q - 1);
  const int64_t edge_off = (int64_t)r * R + 16 * (int64_t)qe + (p ? 0 : 12);

  o = ld16(own + base);
  ctr = ld16(oth + base);
  const uint32_t e = *reinterpret_cast<const uint32_t*>(oth + edge_off);
  const Chunk sh = p ? shift_next(ctr, e) : shift_prev(ctr, e);
  const uint32_t ym = y == 0 ? L - 1 : y - 1, yp = y + 1 == L ? 0 : y + 1;
  const int64_t off_ym = ((int64_t)ym + (int64_t)L * z) * R + 16 * (int64_t)q;
  const int64_t off_yp = ((int64_t)yp + (int64_t)L * z) * R + 16 * (int64_t)q;
  const Chunk nym = ld16(oth + off_ym);
  const Chunk nyp = ld16(oth + off_yp);
  Chunk nzm{}, nzp{};
  int64_t off_zm = 0;
  if (D == 3) {
    const uint32_t zm = z == 0 ? L - 1 : z - 1, zp = z + 1 == L ? 0 : z + 1;
    off_zm = ((int64_t)y + (int64_t)L * zm) * R + 16 * (int64_t)q;
    const int64_t off_zp = ((int64_t)y + (int64_t)L * zp) * R + 16 * (int64_t)q;
    nzm = ld16(oth + off_zm);
    nzp = ld16(oth + off_zp);
  }
  // neighbours at x+1 / x-1
  const Chunk& nxp = p ? sh : ctr;
  const Chunk& nxm = p ? ctr : sh;

  Chunk jxp{}, jxm{}, jyp{}, jym{}, jzp{}, jzm{};
  if (PM) {
    const int8_t* Jo = J + (int64_t)c * Nh;        // J[mu][c] = J + (2 mu + c) Nh
    const int8_t* Jn = J + (int64_t)(1 - c) * Nh;  // J[mu][1-c]
    jxp = ld16(Jo + base);
    const Chunk jc = ld16(Jn + base);
    if (p) {
      jxm = jc;
    } else {
      const uint32_t je = *reinterpret_cast<const uint32_t*>(Jn + edge_off);
      jxm = shift_prev(jc, je);
    }
    jyp = ld16(Jo + 2 * Nh + base);
    jym = ld16(Jn + 2 * Nh + off_ym);
    if (D == 3) {
      jzp = ld16(Jo + 4 * Nh + base);
      jzm = ld16(Jn + 4 * Nh + off_zm);
    }
  }
#pragma unroll
  for (int w = 0; w < 4; ++w) {
    const uint32_t ow = o.w[w];
    uint32_t k2;
    if (PM) {
      k2 = ((ow ^ nxp.w[w] ^ jxp.w[w]) & kBit1) + ((ow ^ nxm.w[w] ^ jxm.w[w]) & kBit1) +
           ((ow ^ nyp.w[w] ^ jyp.w[w]) & kBit1) + ((ow ^ nym.w[w] ^ jym.w[w]) & kBit1);
      if (D == 3)
        k2 += ((ow ^ nzp.w[w] ^ jzp.w[w]) & kBit1) + ((ow ^ nzm.w[w] ^ jzm.w[w]) & kBit1);
    } else {
      k2 = ((ow ^ nxp.w[w]) & kBit1) + ((ow ^ nxm.w[w]) & kBit1) + ((ow ^ nyp.w[w]) & kBit1) +
           ((ow ^ nym.w[w]) & kBit1);
      if (D == 3) k2 += ((ow ^ nzp.w[w]) & kBit1) + ((ow ^ nzm.w[w]) & kBit1);
    }
    kk[w] = k2 >> 1;
  }
}

}  // namespace smc
