// packed.hpp -- bit-sliced Ising decisions for 32 same-colour sites held one
// bit per site in a 32-bit word (multi-spin coding, Sec. 2): the prefix bytes
// of the word's two Philox blocks as bit planes, the unsatisfied-bond count
// planes, and the threshold compare with its exact ties.  Shared by the
// single-lattice packed kernel and the packed path of the batched kernel.
#pragma once

#include <type_traits>

#include "chunk.hpp"

namespace smc {

// bit 7 of each byte of v -> bits 0..3 (byte b -> bit b): the four flag bits
// land on bits 28..31 of the product without carries.
__device__ __forceinline__ uint32_t gather7(uint32_t v) {
  return ((v & 0x80808080u) * 0x00204081u) >> 28;
}

// Bit-sliced equality of the 3-bit count (k2 k1 k0) with a constant K.
template <int K>
__device__ __forceinline__ uint32_t class_mask(uint32_t k0, uint32_t k1, uint32_t k2) {
  const uint32_t a = (K & 1) ? k0 : ~k0;
  const uint32_t b = (K & 2) ? k1 : ~k1;
  const uint32_t c = (K & 4) ? k2 : ~k2;
  return a & b & c;
}

// Exchange of a word-index bit with bit k of the bit position (d = 2^k,
// m = the positions whose bit k is 0) between the words a (index bit 0) and
// b (index bit 1): afterwards a holds the bits whose position bit k was 0, b
// those whose bit k was 1, and position bit k tells which word a bit came
// from.  One rotation serves both outputs: with b' = b rotated left by d, a
// takes b' where m is 0 (b' equals b << d there), and b comes out rotated
// left by d as the select of b' where m is 1 and a elsewhere (a position p
// with bit k set of the rotated word is position p - d, bit k clear, of the
// plain one, whose bits are a's at p and b's at p - d).  Words that carry a
// rotation by r go through later exchanges unchanged as long as the later
// masks repeat with a period dividing r.  (v_bitop3 with the table 0xE4
// selects its first operand where the third is 1 and its second elsewhere;
// the builtin keeps the compiler from splitting the selects into separate
// masks.)
template <int D>
__device__ __forceinline__ void cross_swap_rot(uint32_t& a, uint32_t& b, uint32_t m) {
  const uint32_t br = __builtin_amdgcn_alignbit(b, b, 32 - D);  // b rotated left by D
  const uint32_t na = __builtin_amdgcn_bitop3_b32(a, br, m, 0xE4);
  const uint32_t nb = __builtin_amdgcn_bitop3_b32(br, a, m, 0xE4);
  a = na;
  b = nb;
}

// The 32 prefix bytes of a word's sites (site s in byte s & 3 of P[s >> 2])
// as 8 bit planes: bit s of B[b] = bit b of site s's byte.  With site
// s = 4w + i (word w, byte i) and the bit b of a byte, a byte of P sits at
// word (w2 w1 w0), byte (i1 i0); a bit of the planes must end at word
// (b2 b1 b0), position (w2 w1 w0 i1 i0).  A 4x4 byte transpose (v_perm)
// among the words of equal w0 trades (w2 w1) for (i1 i0); three cross-word
// bit swaps then trade the word bits (w0, i1, i0) for the bit-in-byte bits
// (b2, b1, b0), which leaves every bit at its site's position -- plane b
// rotated left by b (4 b2 + 2 b1 + b0, the rotations its swaps left on it),
// which one rotation per plane takes back.  The masks 0x33333333 and
// 0x55555555 repeat every 4 and 2 bits, so the rotations by 4 and 2 that
// the earlier swaps leave do not disturb the later ones.
__device__ __forceinline__ void prefix_planes(const uint32_t P[8], uint32_t B[8]) {
  uint32_t Q[2][4];  // Q[w0][i]: byte k = byte i of P[2k + w0]
#pragma unroll
  for (int w0 = 0; w0 < 2; ++w0) {
    const uint32_t g0 = P[w0], g1 = P[2 + w0], g2 = P[4 + w0], g3 = P[6 + w0];
    const uint32_t t0 = __builtin_amdgcn_perm(g1, g0, 0x06020400u);  // g0.0 g1.0 g0.2 g1.2
    const uint32_t t1 = __builtin_amdgcn_perm(g1, g0, 0x07030501u);  // g0.1 g1.1 g0.3 g1.3
    const uint32_t t2 = __builtin_amdgcn_perm(g3, g2, 0x06020400u);
    const uint32_t t3 = __builtin_amdgcn_perm(g3, g2, 0x07030501u);
    Q[w0][0] = __builtin_amdgcn_perm(t2, t0, 0x05040100u);  // byte 0 of g0 .. g3
    Q[w0][2] = __builtin_amdgcn_perm(t2, t0, 0x07060302u);
    Q[w0][1] = __builtin_amdgcn_perm(t3, t1, 0x05040100u);
    Q[w0][3] = __builtin_amdgcn_perm(t3, t1, 0x07060302u);
  }
  // w0 <-> b2 (position bit 2), i1 <-> b1, i0 <-> b0
#pragma unroll
  for (int i = 0; i < 4; ++i) cross_swap_rot<4>(Q[0][i], Q[1][i], 0x0F0F0F0Fu);
#pragma unroll
  for (int c2 = 0; c2 < 2; ++c2) {
    cross_swap_rot<2>(Q[c2][0], Q[c2][2], 0x33333333u);
    cross_swap_rot<2>(Q[c2][1], Q[c2][3], 0x33333333u);
    // Q[c2][2 c1 + i0] now holds bit b2 = c2, b1 = c1 of the sites' bytes
#pragma unroll
    for (int c1 = 0; c1 < 2; ++c1) cross_swap_rot<1>(Q[c2][2 * c1], Q[c2][2 * c1 + 1], 0x55555555u);
  }
  B[0] = Q[0][0];
#pragma unroll
  for (int b = 1; b < 8; ++b) {
    const uint32_t v = Q[b >> 2][b & 3];
    B[b] = __builtin_amdgcn_alignbit(v, v, b);  // rotated right by b
  }
}

// Threshold bits of the refusable classes for the fast decision: class 0
// (and class 2 in 3D) as all-ones / zero masks held in vector registers,
// class 1 as all-ones / zero masks in scalar registers (one scalar operand
// per instruction).
struct FastTab {
  uint32_t v0[8], v2[8];
  uint32_t s1[8];
};

__device__ __forceinline__ uint32_t vgpr_copy(uint32_t s) {
  uint32_t v;
  asm volatile("v_mov_b32 %0, %1" : "=v"(v) : "s"(s));
  return v;
}

template <int D>
__device__ __forceinline__ FastTab fast_tab(const TabRegs& tab) {
  FastTab f;
  const uint32_t t0 = table_byte(tab.th_lo, tab.th_hi, 0), t2 = table_byte(tab.th_lo, tab.th_hi, 2);
#pragma unroll
  for (int b = 0; b < 8; ++b) {
    f.v0[b] = vgpr_copy(0u - ((t0 >> b) & 1u));
    f.v2[b] = D == 3 ? vgpr_copy(0u - ((t2 >> b) & 1u)) : 0u;
  }
  const uint32_t t1 = table_byte(tab.th_lo, tab.th_hi, 1);
#pragma unroll
  for (int b = 0; b < 8; ++b) f.s1[b] = __builtin_amdgcn_readfirstlane(0u - ((t1 >> b) & 1u));
  return f;
}

// The 32 prefix bytes of a word's sites as bit planes B[0..7] (bit b of each
// site's byte), from the word's two Philox blocks (hit h of the tiled
// schedule: h in bits 8.. of the counter's last word).
__device__ __forceinline__ void word_prefix(const RngKey& key, uint32_t t, uint32_t c, uint32_t wi,
                                            uint32_t B[8], uint32_t hit = 0) {
  const uint32_t blk = wi * 2u;  // Philox blocks of sites 32 wi .. 32 wi + 31
  const uint32_t tg = tag(c, kIsingPrefix) | (hit << 8);
  const Rand4 ra = philox(blk, t, key.replica, tg, key.k0, key.k1);
  const Rand4 rb = philox(blk + 1u, t, key.replica, tg, key.k0, key.k1);
  const uint32_t P[8] = {ra.w[0], ra.w[1], ra.w[2], ra.w[3], rb.w[0], rb.w[1], rb.w[2], rb.w[3]};
  prefix_planes(P, B);
}

// Decision when only the classes k < d can refuse a move (J0 > 0, where
// Delta E = 4 J0 (d - k)); classes whose threshold reaches 2^32 keep the
// table's threshold byte 0xFF with a full refinement fraction, so they accept
// on every draw here too (a prefix of 0xFF is a tie whose refinement always
// accepts).  Per site the threshold bit X_b of its class is a select by the
// count planes; the compare runs from the least significant bit up,
// lt = [prefix < threshold] by its borrow, eq = [prefix == threshold].
template <int D>
__device__ __forceinline__ uint32_t packed_compare_fast(const FastTab& ft, const uint32_t B[8],
                                                        uint32_t k0, uint32_t k1, uint32_t k2,
                                                        uint32_t& ties) {
  // v_bitop3 truth tables (operands a, b, c): 0xCA = a ? b : c;
  // 0x8E = (~a & b) | (~(a ^ b) & c), the borrow of a - b into c;
  // 0x82 = c & ~(a ^ b)
  uint32_t lt = 0, eq = ~0u;
#pragma unroll
  for (int b = 0; b < 8; ++b) {
    uint32_t X = __builtin_amdgcn_bitop3_b32(k0, ft.s1[b], ft.v0[b], 0xCA);
    if (D == 3) X = __builtin_amdgcn_bitop3_b32(k1, ft.v2[b], X, 0xCA);
    lt = __builtin_amdgcn_bitop3_b32(B[b], X, lt, 0x8E);
    eq = __builtin_amdgcn_bitop3_b32(B[b], X, eq, 0x82);
  }
  // refusable: k < d (2D: k1 = k2 = 0; 3D: k2 = 0 and not k = 3)
  const uint32_t refus = D == 2 ? ~(k1 | k2) : ~(k2 | (k1 & k0));
  ties = refus & eq;
  return ~(refus & ~lt);  // ties are refused here and resolved by their refinement draws
}

// The fast decision for the 32 sites of word wi of a plane (prefix bytes from
// the word's two Philox blocks).
template <int D>
__device__ __forceinline__ uint32_t packed_decide_fast(const FastTab& ft, const RngKey& key,
                                                       uint32_t t, uint32_t c, uint32_t wi,
                                                       uint32_t k0, uint32_t k1, uint32_t k2,
                                                       uint32_t& ties, uint32_t hit = 0) {
  uint32_t B[8];
  word_prefix(key, t, c, wi, B, hit);
  return packed_compare_fast<D>(ft, B, k0, k1, k2, ties);
}

// Decision for the 32 sites of one word from the count planes k0, k1, k2:
// returns the flip mask, with the exact ties (in `ties`) refused.
template <int D>
__device__ __forceinline__ uint32_t packed_compare(const TabRegs& tab, const uint32_t B[8],
                                                   uint32_t k0, uint32_t k1, uint32_t k2,
                                                   uint32_t& ties) {
  // Per-site threshold bit planes: T[b] holds bit b of the threshold byte of
  // each site's class, then one bit-sliced compare of the prefix planes
  // against them.  With J0 > 0 only the classes k < d (Delta E = 4 J0 (d - k)
  // > 0) can refuse a move: they are added without branches, a class whose
  // threshold reaches 2^32 (the table's always-accept flag, also every k < d
  // when J0 <= 0) masked out by a wave-uniform mask.  The classes k > d refuse
  // only when J0 < 0 and are added behind wave-uniform branches, as is class
  // d (Delta E = 0, always accepted; under the heat-bath rule, whose classes
  // count up neighbours, the class of a zero field).
  uint32_t T[8];
  uint32_t refus = 0;
  auto add_class = [&](auto kv) {
    constexpr int KV = decltype(kv)::value;
    const uint32_t live =
        __builtin_amdgcn_readfirstlane(table_byte(tab.al_lo, tab.al_hi, KV) == 0u ? ~0u : 0u);
    const uint32_t m = class_mask<KV>(k0, k1, k2) & live;
    const uint32_t th = table_byte(tab.th_lo, tab.th_hi, KV);
    refus |= m;
#pragma unroll
    for (int b = 0; b < 8; ++b) {
      const uint32_t tb = m & __builtin_amdgcn_readfirstlane(0u - ((th >> b) & 1u));
      T[b] = KV == 0 ? tb : (T[b] | tb);
    }
  };
  auto add_class_if = [&](auto kv) {
    constexpr int KV = decltype(kv)::value;
    if (table_byte(tab.al_lo, tab.al_hi, KV) == 0u) {
      const uint32_t m = class_mask<KV>(k0, k1, k2);
      const uint32_t th = table_byte(tab.th_lo, tab.th_hi, KV);
      refus |= m;
#pragma unroll
      for (int b = 0; b < 8; ++b) T[b] |= m & __builtin_amdgcn_readfirstlane(0u - ((th >> b) & 1u));
    }
  };
  add_class(std::integral_constant<int, 0>());
  add_class(std::integral_constant<int, 1>());
  if constexpr (D == 3) add_class(std::integral_constant<int, 2>());
  add_class_if(std::integral_constant<int, D>());
  add_class_if(std::integral_constant<int, D + 1>());
  add_class_if(std::integral_constant<int, D + 2>());
  if constexpr (D == 3) add_class_if(std::integral_constant<int, 6>());
  // most significant bit first: eq = equal so far, lt = prefix below threshold
  uint32_t eq = ~0u, lt = 0u;
#pragma unroll
  for (int b = 7; b >= 0; --b) {
    lt |= eq & ~B[b] & T[b];
    eq &= ~(B[b] ^ T[b]);
  }
  const uint32_t rej = refus & ~lt;  // prefix >= threshold (ties included)
  ties = refus & eq;
  return ~rej;  // ties are refused here; the caller queues them once the word is stored
}

// The general decision for the 32 sites of word wi of a plane.
template <int D>
__device__ __forceinline__ uint32_t packed_decide(const TabRegs& tab, const RngKey& key,
                                                  uint32_t t, uint32_t c, uint32_t wi,
                                                  uint32_t k0, uint32_t k1, uint32_t k2,
                                                  uint32_t& ties, uint32_t hit = 0) {
  uint32_t B[8];
  word_prefix(key, t, c, wi, B, hit);
  return packed_compare<D>(tab, B, k0, k1, k2, ties);
}

// Unsatisfied-bond count planes of 32 sites from their 2d neighbour words
// (xor of the spin bits, and of the coupling bits with +-1 couplings).
template <int D>
__device__ __forceinline__ void count_planes(const uint32_t u[6], uint32_t& k0, uint32_t& k1,
                                             uint32_t& k2) {
  // full adder of u0, u1, u2
  const uint32_t s1 = u[0] ^ u[1] ^ u[2];
  const uint32_t c1 = (u[0] & u[1]) | (u[2] & (u[0] ^ u[1]));
  if (D == 2) {
    k0 = s1 ^ u[3];
    const uint32_t c2 = s1 & u[3];
    k1 = c1 ^ c2;
    k2 = c1 & c2;
  } else {
    const uint32_t s2 = u[3] ^ u[4] ^ u[5];
    const uint32_t c2 = (u[3] & u[4]) | (u[5] & (u[3] ^ u[4]));
    k0 = s1 ^ s2;
    const uint32_t c3 = s1 & s2;
    // twos: c1 + c2 + c3
    k1 = c1 ^ c2 ^ c3;
    k2 = (c1 & c2) | (c3 & (c1 ^ c2));
  }
}

}  // namespace smc
