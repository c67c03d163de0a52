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

// Blocks are dealt to the 8 XCDs round-robin (block b runs on XCD b % 8).
// Renumber them so that each XCD receives a contiguous range of logical
// blocks, i.e. neighbouring rows of the lattice share one L2.
__device__ __forceinline__ uint32_t xcd_remap(uint32_t b, uint32_t nb) {
  const uint32_t q = nb >> 3, rem = nb & 7u, x = b & 7u, k = b >> 3;
  return x * q + (x < rem ? x : rem) + k;
}

constexpr uint32_t kBit1 = 0x02020202u;  // bit 1 of a +-1 byte: set for -1
constexpr uint32_t kHigh = 0x80808080u;
constexpr uint32_t kOnes = 0x01010101u;


__device__ __forceinline__ uint32_t pick4(const Rand4& r, uint32_t i) {
  const uint32_t a = (i & 1) ? r.w[1] : r.w[0];
  const uint32_t b = (i & 1) ? r.w[3] : r.w[2];
  return (i & 2) ? b : a;
}

__device__ __forceinline__ uint32_t table_byte(uint32_t lo, uint32_t hi, uint32_t k) {
  return ((k < 4 ? lo : hi) >> (8 * (k & 3))) & 0xFFu;
}

__device__ __forceinline__ uint32_t frac_of(const IsingTable& tab, uint32_t k) {
  uint32_t v = tab.frac[0];
  v = k == 1 ? tab.frac[1] : v;
  v = k == 2 ? tab.frac[2] : v;
  v = k == 3 ? tab.frac[3] : v;
  v = k == 4 ? tab.frac[4] : v;
  v = k == 5 ? tab.frac[5] : v;
  v = k == 6 ? tab.frac[6] : v;
  return v;
}

// Unsatisfied-bond counts of a chunk of 2D sites from its four neighbour
// chunks (x+1 / x-1 as centre and shifted chunk, y-1, y+1): byte b of kk[w].
__device__ __forceinline__ void counts2d(const Chunk& o, const Chunk& ctr, const Chunk& sh,
                                         const Chunk& up, const Chunk& dn, uint32_t kk[4]) {
#pragma unroll
  for (int w = 0; w < 4; ++w) {
    const uint32_t ow = o.w[w];
    const uint32_t k2 = ((ow ^ ctr.w[w]) & kBit1) + ((ow ^ sh.w[w]) & kBit1) +
                        ((ow ^ up.w[w]) & kBit1) + ((ow ^ dn.w[w]) & kBit1);
    kk[w] = k2 >> 1;
  }
}

// The refinement fractions of the 7 classes held in scalar registers, as
// named scalars: with an array the compiler turns the select chain back into
// an indexed memory load.
struct FracRegs {
  uint32_t f0, f1, f2, f3, f4, f5, f6;
};

__device__ __forceinline__ FracRegs frac_regs(const IsingTable& tab) {
  FracRegs r;
  r.f0 = __builtin_amdgcn_readfirstlane(tab.frac[0]);
  r.f1 = __builtin_amdgcn_readfirstlane(tab.frac[1]);
  r.f2 = __builtin_amdgcn_readfirstlane(tab.frac[2]);
  r.f3 = __builtin_amdgcn_readfirstlane(tab.frac[3]);
  r.f4 = __builtin_amdgcn_readfirstlane(tab.frac[4]);
  r.f5 = __builtin_amdgcn_readfirstlane(tab.frac[5]);
  r.f6 = __builtin_amdgcn_readfirstlane(tab.frac[6]);
  return r;
}

// Selections below are written as masks, not conditionals: a select of two
// fields of a register-held aggregate can be rewritten into one load through
// a selected pointer, which puts the aggregate in scratch memory.
__device__ __forceinline__ uint32_t mask_sel(uint32_t a, uint32_t b, uint32_t bit) {
  return a ^ ((a ^ b) & (0u - bit));  // bit ? b : a (bit is 0 or 1)
}

__device__ __forceinline__ uint32_t frac_sel(const FracRegs& r, uint32_t k) {
  const uint32_t b0 = k & 1u, b1 = (k >> 1) & 1u, b2 = (k >> 2) & 1u;
  const uint32_t lo = mask_sel(mask_sel(r.f0, r.f1, b0), mask_sel(r.f2, r.f3, b0), b1);
  const uint32_t hi = mask_sel(mask_sel(r.f4, r.f5, b0), r.f6, b1);
  return mask_sel(lo, hi, b2);
}

// Threshold bytes, always-accept flags and refinement fractions pinned in
// scalar registers.
struct TabRegs {
  uint32_t th_lo, th_hi, al_lo, al_hi;
  FracRegs fr;
};

__device__ __forceinline__ TabRegs tab_regs(const IsingTable& tab) {
  TabRegs r;
  r.th_lo = __builtin_amdgcn_readfirstlane(tab.th_lo);
  r.th_hi = __builtin_amdgcn_readfirstlane(tab.th_hi);
  r.al_lo = __builtin_amdgcn_readfirstlane(tab.al_lo);
  r.al_hi = __builtin_amdgcn_readfirstlane(tab.al_hi);
  r.fr = frac_regs(tab);
  return r;
}

// Per-byte decision for 4 sites on the threshold byte alone.  Classes that
// always accept are flagged in Al (bytes 0xFF): they flip whatever the prefix.
// Returns the spin word after the flips the prefix bytes decide; a prefix
// equal to the threshold byte of a refusable class is a tie (probability
// 2^-8), left unflipped here and flagged in bit 7 of the bytes of `tie`
// (the other bits of `tie` are garbage).
__device__ __forceinline__ uint32_t decide4_tie(const TabRegs& tab, uint32_t own, uint32_t k,
                                                uint32_t P, uint32_t& tie) {
  const uint32_t Th = __builtin_amdgcn_perm(tab.th_hi, tab.th_lo, k);
  const uint32_t Al = __builtin_amdgcn_perm(tab.al_hi, tab.al_lo, k);
  const uint32_t x = P ^ Th;
  const uint32_t dlow = (P | kHigh) - (Th & ~kHigh);
  const uint32_t ge = (x & P) | (~x & dlow);  // bit 7 of each byte: P >= Th
  // 0xFF in every byte whose bit 7 of ge is set (sign-replicating selectors)
  const uint32_t rej = __builtin_amdgcn_perm(ge, ge << 8, 0x0B090A08u);
  // bit 7 of z: the low 7 bits of the byte of x are not all zero
  const uint32_t z = (x & 0x7F7F7F7Fu) + 0x7F7F7F7Fu;
  tie = ~(z | x | Al);  // bit 7: x byte == 0 and the class is refusable
  return own ^ ((~rej | Al) & 0xFEFEFEFEu);
}

// 16-bit mask (bit 4w + b) of the tie flags of a chunk.
__device__ __forceinline__ uint32_t tie_mask16(const uint32_t tie[4]) {
  uint32_t m = 0;
#pragma unroll
  for (int w = 0; w < 4; ++w) {
    const uint32_t t7 = tie[w] & kHigh;
    m |= (((t7 >> 7) | (t7 >> 14) | (t7 >> 21) | (t7 >> 28)) & 0xFu) << (4 * w);
  }
  return m;
}

__device__ __forceinline__ uint32_t word_of(const uint32_t v[4], uint32_t w) {
  const uint32_t b0 = w & 1u, b1 = (w >> 1) & 1u;
  return mask_sel(mask_sel(v[0], v[1], b0), mask_sel(v[2], v[3], b0), b1);
}

// Metropolis update of one chunk with its ties resolved on the spot by the
// sites' refinement draws (used where the new spins are read again within
// the same launch).
// `hit` (k-hit schedules) goes to bits 8.. of the counter's last word.
__device__ __forceinline__ Chunk update_chunk_now(const TabRegs& tab, const RngKey& key,
                                                  uint32_t t, uint32_t c, uint32_t jbase,
                                                  const Chunk& o, const uint32_t kk[4],
                                                  uint32_t hit = 0) {
  const Rand4 rp = philox(jbase >> 4, t, key.replica, tag(c, kIsingPrefix) | (hit << 8), key.k0,
                          key.k1);
  uint32_t nw[4], tie[4];
#pragma unroll
  for (int w = 0; w < 4; ++w) nw[w] = decide4_tie(tab, o.w[w], kk[w], rp.w[w], tie[w]);
  if ((tie[0] | tie[1] | tie[2] | tie[3]) & kHigh) {
    uint32_t m = tie_mask16(tie);
    do {
      const uint32_t idx = __builtin_ctz(m);
      m &= m - 1;
      const uint32_t w = idx >> 2, sh = 8 * (idx & 3u);
      const uint32_t k = (word_of(kk, w) >> sh) & 0xFu;
      const Rand4 rr = philox(jbase + idx, t, key.replica, tag(c, kIsingRefine) | (hit << 8),
                              key.k0, key.k1);
      if ((rr.w[0] & 0xFFFFFFu) < frac_sel(tab.fr, k)) {
        const uint32_t f = 0xFEu << sh;
        nw[0] ^= w == 0 ? f : 0u;
        nw[1] ^= w == 1 ? f : 0u;
        nw[2] ^= w == 2 ? f : 0u;
        nw[3] ^= w == 3 ? f : 0u;
      }
    } while (m);
  }
  Chunk n;
  n.w[0] = nw[0]; n.w[1] = nw[1]; n.w[2] = nw[2]; n.w[3] = nw[3];
  return n;
}

// Ties of one lane deferred to the end of its band: 16-bit entries in LDS
// (slot i of lane l at slot[i * stride]), each holding the row within the
// band (6 bits), the site within the chunk (4 bits), the class k (3 bits) and
// whether the spin was -1 (1 bit).  Site of an entry: base + row * R + site.
// Deferring is exact because no update of the same colour reads the site.
constexpr uint32_t kTieSlots = 32;

struct TieQueue {
  uint16_t* slot;   // this lane's first slot
  uint32_t stride;  // slots of one lane are `stride` entries apart
  uint32_t n;       // queued entries
  uint32_t base;    // plane offset of the lane's chunk in row 0 of the band
  uint32_t R;       // plane row length
  int64_t dE;       // change of the unsatisfied-bond sum by resolved flips
  int64_t dM;       // change of the spin sum
};

// Draw the refinement of every queued tie and flip the accepted sites in the
// plane `own` (bytes only this lane touches in this launch).
template <int D>
__device__ __forceinline__ void tie_flush(TieQueue& q, const TabRegs& tab, const RngKey& key,
                                       uint32_t t, uint32_t c, int8_t* own) {
  for (uint32_t i = 0; i < q.n; ++i) {
    const uint32_t e = q.slot[i * q.stride];
    const uint32_t js = q.base + (e >> 4 & 63u) * q.R + (e & 15u);
    const uint32_t k = e >> 10 & 7u;
    const Rand4 rr = philox(js, t, key.replica, tag(c, kIsingRefine), key.k0, key.k1);
    if ((rr.w[0] & 0xFFFFFFu) < frac_sel(tab.fr, k)) {
      const int v = (e >> 13 & 1u) ? -1 : 1;
      own[js] = (int8_t)(-v);
      q.dE += 4 * (int64_t)(D - (int)k);  // all 2d bonds of the site change sign
      q.dM -= 2 * (int64_t)v;
    }
  }
  q.n = 0;
}

// Metropolis update of one chunk (plane row `row` of the band) with its ties
// queued.  A queue without room for the chunk's ties (at most 16, fewer than
// the slots) is flushed before any of them is queued: a flush writes its
// flips to the plane, so it must only hold ties of chunks already stored.
template <int D>
__device__ __forceinline__ Chunk update_chunk_deferred(const TabRegs& tab, const RngKey& key,
                                                       uint32_t t, uint32_t c, uint32_t jbase,
                                                       uint32_t row, const Chunk& o,
                                                       const uint32_t kk[4], TieQueue& q,
                                                       int8_t* own) {
  const Rand4 rp = philox(jbase >> 4, t, key.replica, tag(c, kIsingPrefix), key.k0, key.k1);
  Chunk n;
  uint32_t tie[4];
#pragma unroll
  for (int w = 0; w < 4; ++w) n.w[w] = decide4_tie(tab, o.w[w], kk[w], rp.w[w], tie[w]);
  if ((tie[0] | tie[1] | tie[2] | tie[3]) & kHigh) {
    uint32_t m = tie_mask16(tie);
    if (q.n + (uint32_t)__builtin_popcount(m) > kTieSlots) tie_flush<D>(q, tab, key, t, c, own);
    do {
      const uint32_t idx = __builtin_ctz(m);
      m &= m - 1;
      const uint32_t w = idx >> 2, sh = 8 * (idx & 3u);
      const uint32_t k = (word_of(kk, w) >> sh) & 7u;
      const uint32_t neg = (word_of(o.w, w) >> (sh + 1)) & 1u;  // bit 1 set for -1
      q.slot[q.n * q.stride] = (uint16_t)((row << 4) | idx | (k << 10) | (neg << 13));
      q.n += 1;
    } while (m);
  }
  return n;
}

// Sum of the +-1 spins of a chunk.
__device__ __forceinline__ int32_t chunk_spin_sum(const Chunk& o) {
  uint32_t down2 = 0;
#pragma unroll
  for (int w = 0; w < 4; ++w) down2 = __builtin_amdgcn_sad_u8(o.w[w] & kBit1, 0u, down2);
  return 16 - (int32_t)down2;  // down2 counts 2 per -1 spin
}

// Sum of the per-site unsatisfied-bond counts of a chunk.
__device__ __forceinline__ int32_t chunk_count_sum(const uint32_t kk[4]) {
  uint32_t s = 0;
#pragma unroll
  for (int w = 0; w < 4; ++w) s = __builtin_amdgcn_sad_u8(kk[w], 0u, s);
  return (int32_t)s;
}

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
  // (by value through masks: a conditional reference would put the chunks
  // in scratch memory)
  Chunk nxp, nxm;
#pragma unroll
  for (int w = 0; w < 4; ++w) {
    nxp.w[w] = mask_sel(ctr.w[w], sh.w[w], p);
    nxm.w[w] = mask_sel(sh.w[w], ctr.w[w], p);
  }

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
