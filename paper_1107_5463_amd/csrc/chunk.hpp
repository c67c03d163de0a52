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

// Per-byte decision for 4 sites: k = unsatisfied-bond counts (bytes), P = 4
// prefix bytes.  Returns the spin word after the accepted flips, and the tie
// mask candidates (bit 7 of bytes that may need the refinement draw).
__device__ __forceinline__ uint32_t decide4(const IsingTable& tab, uint32_t own, uint32_t k,
                                            uint32_t P, uint32_t& tie) {
  const uint32_t Th = __builtin_amdgcn_perm(tab.th_hi, tab.th_lo, k);
  const uint32_t Al = __builtin_amdgcn_perm(tab.al_hi, tab.al_lo, k);
  // bit 7 of each byte: P >= Th (unsigned bytes)
  const uint32_t dlow = (P | kHigh) - (Th & ~kHigh);
  const uint32_t x = P ^ Th;
  const uint32_t ge = (x & P) | (~x & dlow);
  const uint32_t acc = (~ge | Al) & kHigh;
  // candidate exact ties P == Th on classes that are not always accepted
  const uint32_t zz = x | Al;
  tie = (zz - kOnes) & ~zz & kHigh;
  return own ^ ((acc - (acc >> 7)) << 1);  // 0xFE flips +1 <-> -1
}

// Exact per-byte tie mask: bit 7 of each byte where P == Th and the class is
// not always accepted (no carries cross bytes).
__device__ __forceinline__ uint32_t tie_bytes(const IsingTable& tab, uint32_t k, uint32_t P) {
  const uint32_t Th = __builtin_amdgcn_perm(tab.th_hi, tab.th_lo, k);
  const uint32_t Al = __builtin_amdgcn_perm(tab.al_hi, tab.al_lo, k);
  const uint32_t z = (P ^ Th) | Al;
  const uint32_t nz = (((z & 0x7F7F7F7Fu) + 0x7F7F7F7Fu) | z) & kHigh;
  return ~nz & kHigh;
}

// 16-bit mask (bit 4w+b) of sites whose prefix byte ties its threshold byte.
__device__ __forceinline__ uint32_t tie_mask16(const IsingTable& tab, const uint32_t kk[4],
                                               const Rand4& rp) {
  uint32_t m = 0;
#pragma unroll
  for (int w = 0; w < 4; ++w) {
    const uint32_t t7 = tie_bytes(tab, kk[w], rp.w[w]);
    const uint32_t nib = ((t7 >> 7) | (t7 >> 14) | (t7 >> 21) | (t7 >> 28)) & 0xFu;
    m |= nib << (4 * w);
  }
  return m;
}

// Resolve the rare ties with each site's 24-bit refinement draw.
__device__ __forceinline__ void resolve_ties(const IsingTable& tab, const RngKey& key, uint32_t t,
                                             uint32_t c, uint32_t jbase, const uint32_t kk[4],
                                             uint32_t mask, uint32_t nw[4]) {
  while (mask) {
    const uint32_t idx = __builtin_ctz(mask);
    mask &= mask - 1;
    const uint32_t w = idx >> 2, b = idx & 3u;
    const uint32_t kw = w == 0 ? kk[0] : (w == 1 ? kk[1] : (w == 2 ? kk[2] : kk[3]));
    const uint32_t k = (kw >> (8 * b)) & 0xFFu;
    const Rand4 rr = philox(jbase + idx, t, key.replica, tag(c, kIsingRefine), key.k0, key.k1);
    if ((rr.w[0] & 0xFFFFFFu) < frac_of(tab, k)) {
      const uint32_t f = 0xFEu << (8 * b);
      nw[0] ^= w == 0 ? f : 0u;
      nw[1] ^= w == 1 ? f : 0u;
      nw[2] ^= w == 2 ? f : 0u;
      nw[3] ^= w == 3 ? f : 0u;
    }
  }
}

// Per-byte decision for 4 sites testing the threshold byte only.  Classes
// that always accept carry threshold byte 0xFF and refinement fraction 2^24,
// and are also flagged in Al: they flip whatever the prefix.  Returns the spin
// word after the flips decided by the prefix bytes; tie7 flags (bit 7) the
// bytes of refusable classes whose prefix may equal the threshold byte -- every
// exact tie (2^-8 of the uphill attempts) plus occasional false alarms directly
// above one, which the slow path re-checks.
__device__ __forceinline__ uint32_t decide4_fast(uint32_t th_lo, uint32_t th_hi, uint32_t al_lo,
                                                 uint32_t al_hi, uint32_t own, uint32_t k,
                                                 uint32_t P, uint32_t& tie7) {
  const uint32_t Th = __builtin_amdgcn_perm(th_hi, th_lo, k);
  const uint32_t Al = __builtin_amdgcn_perm(al_hi, al_lo, k);
  const uint32_t x = P ^ Th;
  const uint32_t dlow = (P | kHigh) - (Th & ~kHigh);
  const uint32_t ge = (x & P) | (~x & dlow);  // bit 7 of each byte: P >= Th
  // 0xFF in every byte whose bit 7 of ge is set (sign-replicating selectors)
  const uint32_t rej = __builtin_amdgcn_perm(ge, ge << 8, 0x0B090A08u);
  tie7 = (x - kOnes) & ~x & ~Al & kHigh;
  return own ^ ((~rej | Al) & 0xFEFEFEFEu);
}

// Deferred tie resolutions of one lane (at most 4 held; more are resolved on
// the spot by the caller).
struct PendingTies {
  uint32_t j[4];
  uint32_t k;  // nibble p = class of entry p
  uint32_t n;
};

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

__device__ __forceinline__ uint32_t frac_sel(const FracRegs& r, uint32_t k) {
  const uint32_t a = (k & 1) ? r.f1 : r.f0;
  const uint32_t b = (k & 1) ? r.f3 : r.f2;
  const uint32_t c = (k & 1) ? r.f5 : r.f4;
  const uint32_t lo = (k & 2) ? b : a;
  const uint32_t hi = (k & 2) ? r.f6 : c;
  return (k & 4) ? hi : lo;
}

// Exact 16-bit mask (bit 4w+b) of sites whose prefix byte equals the threshold
// byte of their class.
__device__ __forceinline__ uint32_t exact_ties16(uint32_t th_lo, uint32_t th_hi,
                                                 const uint32_t kk[4], const Rand4& rp) {
  uint32_t m = 0;
#pragma unroll
  for (int w = 0; w < 4; ++w) {
    const uint32_t z7 = rp.w[w] ^ __builtin_amdgcn_perm(th_hi, th_lo, kk[w]);
    const uint32_t t7 = ~((((z7 & 0x7F7F7F7Fu) + 0x7F7F7F7Fu) | z7)) & kHigh;
    m |= (((t7 >> 7) | (t7 >> 14) | (t7 >> 21) | (t7 >> 28)) & 0xFu) << (4 * w);
  }
  return m;
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

// Flip byte b of word w of a chunk's new spins (static register indices).
__device__ __forceinline__ void flip_byte(uint32_t nw[4], uint32_t w, uint32_t b) {
  const uint32_t f = 0xFEu << (8 * b);
  nw[0] ^= w == 0 ? f : 0u;
  nw[1] ^= w == 1 ? f : 0u;
  nw[2] ^= w == 2 ? f : 0u;
  nw[3] ^= w == 3 ? f : 0u;
}

// Queue an exact tie for the end of the band, or resolve it now if the queue
// is full.  Returns true if it was resolved now and the move accepted.
__device__ __forceinline__ bool queue_tie(PendingTies& pend, const TabRegs& tab, const RngKey& key,
                                          uint32_t t, uint32_t c, uint32_t js, uint32_t k) {
  if (pend.n < 4) {
    pend.j[0] = pend.n == 0 ? js : pend.j[0];
    pend.j[1] = pend.n == 1 ? js : pend.j[1];
    pend.j[2] = pend.n == 2 ? js : pend.j[2];
    pend.j[3] = pend.n == 3 ? js : pend.j[3];
    pend.k |= k << (4 * pend.n);
    pend.n += 1;
    return false;
  }
  const Rand4 rr = philox(js, t, key.replica, tag(c, kIsingRefine), key.k0, key.k1);
  return (rr.w[0] & 0xFFFFFFu) < frac_sel(tab.fr, k);
}

// Visit the tie candidates of one chunk: exact ties (prefix byte == threshold
// byte of the site's class) are resolved at once (DEFER = false) or queued.
template <bool DEFER>
__device__ __forceinline__ void handle_ties(const TabRegs& tab, const RngKey& key, uint32_t t,
                                            uint32_t c, uint32_t jbase, const uint32_t kk[4],
                                            const Rand4& rp, const uint32_t tie7[4],
                                            uint32_t nw[4], PendingTies& pend) {
#pragma unroll
  for (uint32_t w = 0; w < 4; ++w) {
    uint32_t m = tie7[w];
    while (m) {
      const uint32_t b = __builtin_ctz(m) >> 3;
      m &= m - 1;
      const uint32_t k = (kk[w] >> (8 * b)) & 0xFu;
      if (((rp.w[w] >> (8 * b)) & 0xFFu) != table_byte(tab.th_lo, tab.th_hi, k)) continue;
      const uint32_t js = jbase + 4 * w + b;
      bool acc;
      if (DEFER) {
        acc = queue_tie(pend, tab, key, t, c, js, k);
      } else {
        const Rand4 rr = philox(js, t, key.replica, tag(c, kIsingRefine), key.k0, key.k1);
        acc = (rr.w[0] & 0xFFFFFFu) < frac_sel(tab.fr, k);
      }
      if (acc) flip_byte(nw, w, b);
    }
  }
}

// Metropolis update of one chunk given its unsatisfied-bond counts: one
// Philox block for the 16 prefix bytes; the refinement draw only for the rare
// exact ties, resolved on the spot (DEFER = false) or queued in pend.
template <bool DEFER>
__device__ __forceinline__ Chunk update_chunk(const TabRegs& tab, const RngKey& key, uint32_t t,
                                              uint32_t c, uint32_t jbase, const Chunk& o,
                                              const uint32_t kk[4], PendingTies& pend) {
  const Rand4 rp = philox(jbase >> 4, t, key.replica, tag(c, kIsingPrefix), key.k0, key.k1);
  uint32_t nw[4], tie7[4], anytie = 0;
#pragma unroll
  for (int w = 0; w < 4; ++w) {
    nw[w] = decide4_fast(tab.th_lo, tab.th_hi, tab.al_lo, tab.al_hi, o.w[w], kk[w], rp.w[w], tie7[w]);
    anytie |= tie7[w];
  }
  if (anytie) handle_ties<DEFER>(tab, key, t, c, jbase, kk, rp, tie7, nw, pend);
  Chunk n;
  n.w[0] = nw[0]; n.w[1] = nw[1]; n.w[2] = nw[2]; n.w[3] = nw[3];
  return n;
}

// Resolve a lane's queued ties against its own colour plane (bytes of plane
// `own` that no other lane of the launch touches).  Returns the change of the
// unsatisfied-bond sum of the flipped sites' energy and of their spin sum
// through dE / dM (for a fused measurement).
template <int D>
__device__ __forceinline__ void resolve_pending(const PendingTies& pend, const TabRegs& tab,
                                                const RngKey& key, uint32_t t, uint32_t c,
                                                int8_t* own, int64_t& dE, int64_t& dM) {
  for (uint32_t e = 0; e < pend.n; ++e) {
    const uint32_t js = e == 0 ? pend.j[0] : (e == 1 ? pend.j[1] : (e == 2 ? pend.j[2] : pend.j[3]));
    const uint32_t k = (pend.k >> (4 * e)) & 0xFu;
    const Rand4 rr = philox(js, t, key.replica, tag(c, kIsingRefine), key.k0, key.k1);
    if ((rr.w[0] & 0xFFFFFFu) < frac_sel(tab.fr, k)) {
      const int8_t v = own[js];
      own[js] = (int8_t)(-v);
      dE += 4 * (int64_t)(D - (int)k);  // all 2d bonds of the site change sign
      dM -= 2 * (int64_t)v;
    }
  }
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
