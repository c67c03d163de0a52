// device.hpp -- device-side building blocks shared by the libsmc kernels:
// Philox4x32-10, the counter layout of the random-number contract, lattice
// geometry in the colour-split layout, and small wave-level helpers.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace smc {

// ---------------------------------------------------------------------------
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): ten rounds of two
// 32x32->64 multiplies (counter words 0 and 2) whose high halves are xored
// with the other counter words and the round key; the round key advances by
// the Weyl increments.  The key is wave-uniform (the seed), so its schedule
// lives in scalar registers.
// ---------------------------------------------------------------------------
struct Rand4 {
  uint32_t w[4];
};

__device__ __forceinline__ Rand4 philox(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                        uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    // one 32x32 -> 64-bit product per multiplier (a single v_mad_u64_u32)
    const uint64_t p0 = (uint64_t)0xD2511F53u * c0, p1 = (uint64_t)0xCD9E8D57u * c2;
    const uint32_t lo0 = (uint32_t)p0, hi0 = (uint32_t)(p0 >> 32);
    const uint32_t lo1 = (uint32_t)p1, hi1 = (uint32_t)(p1 >> 32);
    // three-way xors as single v_bitop3_b32 (truth table 0x96 = a ^ b ^ c)
    const uint32_t n0 = __builtin_amdgcn_bitop3_b32(hi1, c1, k0, 0x96);
    const uint32_t n2 = __builtin_amdgcn_bitop3_b32(hi0, c3, k1, 0x96);
    c0 = n0;
    c1 = lo1;
    c2 = n2;
    c3 = lo0;
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
  Rand4 o;
  o.w[0] = c0; o.w[1] = c1; o.w[2] = c2; o.w[3] = c3;
  return o;
}

// Random-number contract: counter = (block, t, replica, colour | purpose<<1).
enum Purpose : uint32_t {
  kIsingPrefix = 0,  // one byte per Ising site: byte j&3 of word (j>>2)&3 of block j>>4
  kIsingRefine = 1,  // low 24 bits of word 0 of block j, drawn only on a prefix tie
  kContinuous = 2,   // XY: block j>>1, words 2(j&1), 2(j&1)+1; Heisenberg: block j;
                     // Ising with FP32 couplings: word j&3 of block j>>2
  kInitSpin = 3,     // block from the natural site index i, counter word 1 = 0
  kCoupling = 4      // counter word 1 = axis mu
};

__device__ __forceinline__ uint32_t tag(uint32_t colour, uint32_t purpose) {
  return colour | (purpose << 1);
}

// Uniform in (0,1): (2k+1)/2^24 with k the top 23 bits of w (exact in FP32,
// symmetric about 1/2).
__device__ __forceinline__ float u01f(uint32_t w) {
  return __uint2float_rn((w >> 9) * 2u + 1u) * 5.9604644775390625e-8f;  // 2^-24
}
__device__ __forceinline__ double u01d(uint32_t w) {
  return (double)((w >> 9) * 2u + 1u) * 5.9604644775390625e-8;
}

// Metropolis acceptance of a move with an FP32 energy change (Eq. (2)):
// dE <= 0, or u < exp(-beta dE).  exp(-beta dE) is taken as 2^(-b dE) with
// b = beta log2(e) rounded once from FP64 (`beta_log2e`) and the hardware
// base-2 exponential: the argument carries two FP32 roundings (relative
// 2^-23) and the exponential about one ulp, so p is off by less than
// p (x ln2 2^-23 + 2^-23) <= 2e-7 -- below the FP32 rounding of dE itself.
// Both sides are evaluated and or-ed, with no branch.
__device__ __forceinline__ float beta_log2e(float beta) {
  return (float)((double)beta * 1.44269504088896340736);
}
__device__ __forceinline__ bool metropolis_fp32(float dE, float u, float bl2e) {
  return (dE <= 0.0f) | (u < __builtin_amdgcn_exp2f(-bl2e * dE));
}

// ---------------------------------------------------------------------------
// Geometry of the colour-split layout.  Site i = x + L*y + L*L*z has colour
// c = (x+y+z)&1 and index j = i>>1 in plane c.  Plane rows: row r = y + L*z
// holds the L/2 same-colour sites of that (y, z) line, j = r*(L/2) + (x>>1).
// ---------------------------------------------------------------------------
struct Geom {
  int32_t L;        // edge
  int32_t d;        // 2 or 3
  int32_t R;        // L/2: sites per plane row
  int32_t rows;     // L^(d-1)
  int64_t Nh;       // N/2 sites per colour
};

// Coordinates of site (c, j): returns x, y, z.
__device__ __forceinline__ void site_coords(const Geom& g, uint32_t c, int64_t j, int32_t& x,
                                            int32_t& y, int32_t& z) {
  // plane indices are below N/2 < 2^31: 32-bit divisions
  const uint32_t ju = (uint32_t)j, R = (uint32_t)g.R, L = (uint32_t)g.L;
  const uint32_t r = ju / R;
  const int32_t jx = (int32_t)(ju - r * R);
  z = (int32_t)(r / L);
  y = (int32_t)(r - (uint32_t)z * L);
  const int32_t p = (int32_t)((c + (uint32_t)y + (uint32_t)z) & 1u);
  x = 2 * jx + p;
}

// Index within its plane of the site at (x, y, z) (any colour).
__device__ __forceinline__ int64_t plane_index(const Geom& g, int32_t x, int32_t y, int32_t z) {
  return ((int64_t)z * g.L + y) * g.R + (x >> 1);
}

__device__ __forceinline__ int32_t wrap(int32_t v, int32_t L) {
  return v < 0 ? v + L : (v >= L ? v - L : v);
}

// Natural site index (used only by the init draws).
__device__ __forceinline__ int64_t natural_index(const Geom& g, int32_t x, int32_t y, int32_t z) {
  return ((int64_t)z * g.L + y) * g.L + x;
}

// Ising threshold table, per number k of unsatisfied bonds (k = 0..2d):
// bytes of T[k] >> 24, bytes of the always-accept flag, and the low 24 bits.
struct IsingTable {
  uint32_t th_lo, th_hi;   // byte k of (th_hi:th_lo) = T[k] >> 24 (k < 8)
  uint32_t al_lo, al_hi;   // byte k = 0xFF if class k is always accepted
  uint32_t frac[8];        // T[k] & 0xFFFFFF
};

}  // namespace smc
