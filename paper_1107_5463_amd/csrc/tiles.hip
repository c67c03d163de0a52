// tiles.hip -- the paper's two-level ("double") checkerboard with k hits per
// tile load (Sec. 2), for Ising spins with uniform couplings, under the
// Metropolis or the heat-bath rule.
//
// The lattice is cut into tiles of edge T (T = 16 or T % 32 == 0, L / T even), coloured
// by (tx + ty + tz) mod 2.  One launch treats every tile of one colour: a
// workgroup stages its tile plus a one-site boundary layer in LDS (both colour
// planes, rows of T/2 sites with 16 bytes of padding on each side so that
// every 16-site chunk is an aligned 16-byte LDS access and the in-row halo
// bytes sit next to the row), then k times updates the tile's colour-0 sites,
// barrier, colour-1 sites, barrier, and finally writes the tile back.  The
// boundary layer belongs to tiles of the other colour, which no workgroup of
// the launch modifies.  A lane updates one 16-site chunk of a tile row at a
// time with the SWAR decision of the streaming kernel; hit h draws its bytes
// with h in bits 8.. of the counter's last word, so hit 0 of a sweep uses the
// plain sweep's counters.
//
// Heat bath: the new spin is +1 iff u32 < T_hb[npos], npos = number of
// neighbours with sign(J) s_nb = +1 (= 2d - k for s = +1, k for s = -1, with
// k the unsatisfied bonds), with the same prefix-byte / 24-bit refinement
// draw as the Metropolis rule.
//
// 2D Metropolis tiles of edge 16, 64 or 128 take the bit-packed kernels at the
// end of this file, which hold the tile at one bit per site in LDS and make
// the same decisions bit for bit.
#include "chunk.hpp"
#include "packed.hpp"

namespace smc {

__device__ __forceinline__ Chunk lds16(const int8_t* p) {
  const uint4 v = *reinterpret_cast<const uint4*>(p);
  Chunk c;
  c.w[0] = v.x; c.w[1] = v.y; c.w[2] = v.z; c.w[3] = v.w;
  return c;
}

// Heat-bath update of a 16-site chunk: class npos per site, new spin from
// the prefix byte against the class's threshold byte, exact ties refined.
__device__ __forceinline__ Chunk heatbath_chunk(const TabRegs& tab, const RngKey& key, uint32_t t,
                                                uint32_t c, uint32_t jbase, const Chunk& o,
                                                const uint32_t kk[4], uint32_t two_d,
                                                uint32_t hit) {
  const Rand4 rp = philox(jbase >> 4, t, key.replica, tag(c, kIsingPrefix) | (hit << 8), key.k0,
                          key.k1);
  Chunk n;
  uint32_t tie[4], idx[4];
#pragma unroll
  for (int w = 0; w < 4; ++w) {
    const uint32_t negm = __builtin_amdgcn_perm(o.w[w], o.w[w] << 8, 0x0B090A08u);  // 0xFF: s = -1
    idx[w] = (kk[w] & negm) | ((two_d * kOnes - kk[w]) & ~negm);
    const uint32_t Th = __builtin_amdgcn_perm(tab.th_hi, tab.th_lo, idx[w]);
    const uint32_t P = rp.w[w];
    const uint32_t x = P ^ Th;
    const uint32_t dlow = (P | kHigh) - (Th & ~kHigh);
    const uint32_t ge = (x & P) | (~x & dlow);  // bit 7: P >= Th -> spin -1
    n.w[w] = __builtin_amdgcn_perm(ge, ge << 8, 0x0B090A08u) | kOnes;
    const uint32_t z = (x & 0x7F7F7F7Fu) + 0x7F7F7F7Fu;
    tie[w] = ~(z | x) & kHigh;
  }
  if (tie[0] | tie[1] | tie[2] | tie[3]) {
    uint32_t m = tie_mask16(tie);
    do {
      const uint32_t b = __builtin_ctz(m);
      m &= m - 1;
      const uint32_t w = b >> 2, sh = 8 * (b & 3u);
      const uint32_t cls = (word_of(idx, w) >> sh) & 0xFu;
      const Rand4 rr = philox(jbase + b, t, key.replica, tag(c, kIsingRefine) | (hit << 8),
                              key.k0, key.k1);
      // tie: the new spin is +1 iff the 24-bit refinement is below the class's fraction
      const uint32_t up = (rr.w[0] & 0xFFFFFFu) < frac_sel(tab.fr, cls) ? 1u : 0u;
      const uint32_t clear = ~(0xFFu << sh);
      const uint32_t val = (up ? 0x01u : 0xFFu) << sh;
      n.w[0] = w == 0 ? (n.w[0] & clear) | val : n.w[0];
      n.w[1] = w == 1 ? (n.w[1] & clear) | val : n.w[1];
      n.w[2] = w == 2 ? (n.w[2] & clear) | val : n.w[2];
      n.w[3] = w == 3 ? (n.w[3] & clear) | val : n.w[3];
    } while (m);
  }
  return n;
}

template <int D, bool HB>
__global__ __launch_bounds__(256) void tile_kernel(const Geom g, const RngKey key,
                                                   const IsingTable table, const uint32_t T,
                                                   const uint32_t hits, const uint32_t t,
                                                   const uint32_t tc, int8_t* __restrict__ s) {
  extern __shared__ __align__(16) int8_t lds[];
  const uint32_t L = (uint32_t)g.L, R = (uint32_t)g.R;
  const uint32_t nt = L / T, half = nt / 2;
  uint32_t tx, ty, tz = 0;
  {
    const uint32_t b = blockIdx.x;
    uint32_t rem = b;
    if (D == 3) {
      tz = b / (nt * half);
      rem = b - tz * nt * half;
    }
    ty = rem / half;
    tx = 2 * (rem - ty * half) + ((ty + tz + tc) & 1u);
  }
  const uint32_t X0 = tx * T, Y0 = ty * T, Z0 = tz * T;
  const uint32_t RS = T / 2 + 32;                        // LDS row stride (bytes)
  const uint32_t TR = T + 2;                             // rows per axis incl. halo
  const uint32_t NR = D == 3 ? TR * TR : TR;             // rows per colour plane
  const uint32_t words = T / 8;                          // 4-byte words of a tile row
  const uint64_t Nh = (uint64_t)g.Nh;
  auto grow = [&](uint32_t r) -> uint64_t {  // global plane row of LDS row r
    const uint32_t ry = r % TR, rz = r / TR;
    const uint32_t y = (Y0 + L - 1 + ry) % L;
    const uint32_t z = D == 3 ? (Z0 + L - 1 + rz) % L : 0u;
    return ((uint64_t)z * L + y) * R;
  };
  // stage both planes: T/8 words per row plus the two halo bytes
  const uint32_t per_row = words + 2;
  for (uint32_t it = threadIdx.x; it < 2 * NR * per_row; it += blockDim.x) {
    const uint32_t cc = it / (NR * per_row);
    const uint32_t rest = it - cc * NR * per_row;
    const uint32_t r = rest / per_row, wv = rest - r * per_row;
    const int8_t* src = s + cc * Nh + grow(r);
    int8_t* dst = lds + (cc * NR + r) * RS;
    if (wv < words) {
      *reinterpret_cast<uint32_t*>(dst + 16 + 4 * wv) =
          *reinterpret_cast<const uint32_t*>(src + X0 / 2 + 4 * wv);
    } else if (wv == words) {
      dst[15] = src[X0 == 0 ? R - 1 : X0 / 2 - 1];
    } else {
      const uint32_t xr = X0 / 2 + T / 2;
      dst[16 + T / 2] = src[xr == R ? 0 : xr];
    }
  }
  __syncthreads();

  const TabRegs tab = tab_regs(table);
  const uint32_t cpr = T / 32;                            // chunks per tile row
  const uint32_t nchunks = (D == 3 ? T * T : T) * cpr;    // per colour
  for (uint32_t h = 0; h < hits; ++h) {
    for (uint32_t c = 0; c < 2; ++c) {
      int8_t* own = lds + c * NR * RS;
      const int8_t* oth = lds + (1 - c) * NR * RS;
      for (uint32_t ci = threadIdx.x; ci < nchunks; ci += blockDim.x) {
        const uint32_t m = ci % cpr, rowi = ci / cpr;
        const uint32_t ry = 1 + rowi % T, rz = D == 3 ? 1 + rowi / T : 0u;
        const uint32_t y = Y0 + ry - 1, z = D == 3 ? Z0 + rz - 1 : 0u;
        const uint32_t p = (c + y + z) & 1u;
        const uint32_t r = ry + TR * rz;
        const uint32_t off = 16 + 16 * m;
        const Chunk o = lds16(own + r * RS + off);
        const Chunk ct = lds16(oth + r * RS + off);
        const Chunk up = lds16(oth + (r - 1) * RS + off);
        const Chunk dn = lds16(oth + (r + 1) * RS + off);
        const uint32_t e = *reinterpret_cast<const uint32_t*>(oth + r * RS + (p ? off + 16 : off - 4));
        const Chunk sh = p ? shift_next(ct, e) : shift_prev(ct, e);
        Chunk fz{}, bz{};
        if (D == 3) {
          fz = lds16(oth + (r - TR) * RS + off);
          bz = lds16(oth + (r + TR) * RS + off);
        }
        uint32_t kk[4];
#pragma unroll
        for (int w = 0; w < 4; ++w) {
          const uint32_t ow = o.w[w];
          uint32_t k2 = ((ow ^ ct.w[w]) & kBit1) + ((ow ^ sh.w[w]) & kBit1) +
                        ((ow ^ up.w[w]) & kBit1) + ((ow ^ dn.w[w]) & kBit1);
          if (D == 3) k2 += ((ow ^ fz.w[w]) & kBit1) + ((ow ^ bz.w[w]) & kBit1);
          kk[w] = k2 >> 1;
        }
        const uint32_t jbase = (uint32_t)(((uint64_t)z * L + y) * R + X0 / 2 + 16 * m);
        const Chunk nw = HB ? heatbath_chunk(tab, key, t, c, jbase, o, kk, 2 * D, h)
                            : update_chunk_now(tab, key, t, c, jbase, o, kk, h);
        *reinterpret_cast<uint4*>(own + r * RS + off) = make_uint4(nw.w[0], nw.w[1], nw.w[2], nw.w[3]);
      }
      __syncthreads();
    }
  }

  // write back the tile's own rows of both colours
  const uint32_t trows = D == 3 ? T * T : T;
  for (uint32_t it = threadIdx.x; it < 2 * trows * words; it += blockDim.x) {
    const uint32_t cc = it / (trows * words);
    const uint32_t rest = it - cc * trows * words;
    const uint32_t rowi = rest / words, wv = rest - rowi * words;
    const uint32_t ry = 1 + rowi % T, rz = D == 3 ? 1 + rowi / T : 0u;
    const uint32_t r = ry + TR * rz;
    const uint32_t y = Y0 + ry - 1, z = D == 3 ? Z0 + rz - 1 : 0u;
    int8_t* dst = s + cc * Nh + ((uint64_t)z * L + y) * R + X0 / 2 + 4 * wv;
    *reinterpret_cast<uint32_t*>(dst) =
        *reinterpret_cast<const uint32_t*>(lds + (cc * NR + r) * RS + 16 + 4 * wv);
  }
}

// The 8 sites of a 16-wide tile row: words h0 and h0 + 1 (h0 = 0 or 2) of
// their 16-site chunk, whose Philox block (base jbase) gives the words h0,
// h0 + 1 of prefix bytes.  Metropolis with the ties resolved on the spot.
__device__ __forceinline__ uint2 update_half_now(const TabRegs& tab, const RngKey& key,
                                                 uint32_t t, uint32_t c, uint32_t jbase,
                                                 uint32_t h0, uint32_t o0, uint32_t o1,
                                                 uint32_t k0, uint32_t k1, uint32_t hit) {
  const Rand4 rp = philox(jbase >> 4, t, key.replica, tag(c, kIsingPrefix) | (hit << 8), key.k0,
                          key.k1);
  const uint32_t P0 = h0 ? rp.w[2] : rp.w[0], P1 = h0 ? rp.w[3] : rp.w[1];
  uint32_t tie[4] = {0u, 0u, 0u, 0u};
  uint32_t n0 = decide4_tie(tab, o0, k0, P0, tie[0]);
  uint32_t n1 = decide4_tie(tab, o1, k1, P1, tie[1]);
  if ((tie[0] | tie[1]) & kHigh) {
    uint32_t m = tie_mask16(tie);  // bits 0..7: sites 4 h0 .. 4 h0 + 7 of the chunk
    do {
      const uint32_t idx = __builtin_ctz(m);
      m &= m - 1;
      const uint32_t w = idx >> 2, sh = 8 * (idx & 3u);
      const uint32_t k = ((w ? k1 : k0) >> sh) & 0xFu;
      const Rand4 rr = philox(jbase + 4 * h0 + idx, t, key.replica,
                              tag(c, kIsingRefine) | (hit << 8), key.k0, key.k1);
      if ((rr.w[0] & 0xFFFFFFu) < frac_sel(tab.fr, k)) {
        const uint32_t f = 0xFEu << sh;
        n0 ^= w == 0 ? f : 0u;
        n1 ^= w == 1 ? f : 0u;
      }
    } while (m);
  }
  return make_uint2(n0, n1);
}

// The heat-bath update of the same 8 sites (cf. heatbath_chunk).
__device__ __forceinline__ uint2 heatbath_half(const TabRegs& tab, const RngKey& key, uint32_t t,
                                               uint32_t c, uint32_t jbase, uint32_t h0,
                                               uint32_t o0, uint32_t o1, uint32_t k0,
                                               uint32_t k1, uint32_t two_d, uint32_t hit) {
  const Rand4 rp = philox(jbase >> 4, t, key.replica, tag(c, kIsingPrefix) | (hit << 8), key.k0,
                          key.k1);
  const uint32_t o[2] = {o0, o1}, kk[2] = {k0, k1};
  const uint32_t P[2] = {h0 ? rp.w[2] : rp.w[0], h0 ? rp.w[3] : rp.w[1]};
  uint32_t n[2], idx[2], tie[4] = {0u, 0u, 0u, 0u};
#pragma unroll
  for (int w = 0; w < 2; ++w) {
    const uint32_t negm = __builtin_amdgcn_perm(o[w], o[w] << 8, 0x0B090A08u);  // 0xFF: s = -1
    idx[w] = (kk[w] & negm) | ((two_d * kOnes - kk[w]) & ~negm);
    const uint32_t Th = __builtin_amdgcn_perm(tab.th_hi, tab.th_lo, idx[w]);
    const uint32_t x = P[w] ^ Th;
    const uint32_t dlow = (P[w] | kHigh) - (Th & ~kHigh);
    const uint32_t ge = (x & P[w]) | (~x & dlow);  // bit 7: P >= Th -> spin -1
    n[w] = __builtin_amdgcn_perm(ge, ge << 8, 0x0B090A08u) | kOnes;
    const uint32_t z = (x & 0x7F7F7F7Fu) + 0x7F7F7F7Fu;
    tie[w] = ~(z | x) & kHigh;
  }
  if (tie[0] | tie[1]) {
    uint32_t m = tie_mask16(tie);
    do {
      const uint32_t b = __builtin_ctz(m);
      m &= m - 1;
      const uint32_t w = b >> 2, sh = 8 * (b & 3u);
      const uint32_t cls = ((w ? idx[1] : idx[0]) >> sh) & 0xFu;
      const Rand4 rr = philox(jbase + 4 * h0 + b, t, key.replica,
                              tag(c, kIsingRefine) | (hit << 8), key.k0, key.k1);
      const uint32_t up = (rr.w[0] & 0xFFFFFFu) < frac_sel(tab.fr, cls) ? 1u : 0u;
      const uint32_t clear = ~(0xFFu << sh);
      const uint32_t val = (up ? 0x01u : 0xFFu) << sh;
      n[0] = w == 0 ? (n[0] & clear) | val : n[0];
      n[1] = w == 1 ? (n[1] & clear) | val : n[1];
    } while (m);
  }
  return make_uint2(n[0], n[1]);
}

// Tiles of edge 16 (the tile size of the paper's measurements): a tile row
// holds 8 sites of a colour, half of a 16-site chunk and of its Philox block.
// A lane updates its 8 sites as words h0, h0 + 1 of their 16-site chunk
// (h0 = 0 for even tx, 2 for odd), drawing the chunk's Philox block: in its
// 48-byte LDS row the tile's sites sit where those words of the chunk would
// (byte 16 or 24), the halo bytes next to them.
// The workgroup's 256 lanes take one tile row each: 16 tiles per workgroup in
// 2D, one in 3D.
template <int D, bool HB>
__global__ __launch_bounds__(256) void tile16_kernel(const Geom g, const RngKey key,
                                                     const IsingTable table, const uint32_t hits,
                                                     const uint32_t t, const uint32_t tc,
                                                     const uint32_t ntiles, int8_t* __restrict__ s) {
  constexpr uint32_t T = 16, TR = T + 2, RS = 48;
  constexpr uint32_t NR = D == 3 ? TR * TR : TR;  // LDS rows per colour plane of a tile
  constexpr uint32_t TROWS = D == 3 ? T * T : T;  // tile rows per colour
  constexpr uint32_t G = 256 / TROWS;             // tiles per workgroup
  constexpr uint32_t TB = 2 * NR * RS;            // LDS bytes per tile
  extern __shared__ __align__(16) int8_t lds[];
  const uint32_t L = (uint32_t)g.L, R = (uint32_t)g.R;
  const uint32_t nt = L / T, half = nt / 2;
  const uint64_t Nh = (uint64_t)g.Nh;
  auto coords = [&](uint32_t b, uint32_t& tx, uint32_t& ty, uint32_t& tz) {
    uint32_t rem = b;
    tz = 0;
    if (D == 3) {
      tz = b / (nt * half);
      rem = b - tz * nt * half;
    }
    ty = rem / half;
    tx = 2 * (rem - ty * half) + ((ty + tz + tc) & 1u);
  };
  // stage both planes of each tile: 2 words per row plus the two halo bytes
  for (uint32_t it = threadIdx.x; it < G * 2 * NR * 4; it += 256) {
    const uint32_t gi = it / (2 * NR * 4);
    const uint32_t b = blockIdx.x * G + gi;
    if (b >= ntiles) continue;
    uint32_t rest = it - gi * 2 * NR * 4;
    const uint32_t cc = rest / (NR * 4);
    rest -= cc * NR * 4;
    const uint32_t r = rest / 4, wv = rest - r * 4;
    uint32_t tx, ty, tz;
    coords(b, tx, ty, tz);
    const uint32_t ry = r % TR, rz = r / TR;
    const uint32_t y = (ty * T + L - 1 + ry) % L;
    const uint32_t z = D == 3 ? (tz * T + L - 1 + rz) % L : 0u;
    const int8_t* src = s + cc * Nh + ((uint64_t)z * L + y) * R;
    int8_t* dst = lds + gi * TB + (cc * NR + r) * RS + 16 + 8 * (tx & 1u);
    const uint32_t x0 = tx * (T / 2);  // first in-colour index of the tile row
    if (wv < 2) {
      *reinterpret_cast<uint32_t*>(dst + 4 * wv) = *reinterpret_cast<const uint32_t*>(src + x0 + 4 * wv);
    } else if (wv == 2) {
      dst[-1] = src[x0 == 0 ? R - 1 : x0 - 1];
    } else {
      const uint32_t xr = x0 + T / 2;
      dst[T / 2] = src[xr == R ? 0 : xr];
    }
  }
  __syncthreads();

  const TabRegs tab = tab_regs(table);
  const uint32_t gi = threadIdx.x / TROWS, rowi = threadIdx.x - gi * TROWS;
  const uint32_t b = blockIdx.x * G + gi;
  const bool valid = b < ntiles;
  uint32_t tx = 0, ty = 0, tz = 0;
  if (valid) coords(b, tx, ty, tz);
  const uint32_t odd = tx & 1u;
  const uint32_t ry = 1 + rowi % T, rz = D == 3 ? 1 + rowi / T : 0u;
  const uint32_t y = ty * T + ry - 1, z = D == 3 ? tz * T + rz - 1 : 0u;
  const uint32_t r = ry + TR * rz;
  // the chunk holding the tile row: LDS bytes 16..31, global in-colour index
  const uint32_t jbase = (uint32_t)(((uint64_t)z * L + y) * R + tx * (T / 2) - 8 * odd);
  for (uint32_t h = 0; h < hits; ++h) {
    for (uint32_t c = 0; c < 2; ++c) {
      if (valid) {
        int8_t* own = lds + gi * TB + c * NR * RS;
        const int8_t* oth = lds + gi * TB + (1 - c) * NR * RS;
        const uint32_t p = (c + y + z) & 1u;
        const uint32_t base = 16 + 8 * odd;  // the tile row's 8 bytes
        auto ld2 = [&](const int8_t* q) { return *reinterpret_cast<const uint2*>(q); };
        const uint2 o = ld2(own + r * RS + base);
        const uint2 ct = ld2(oth + r * RS + base);
        const uint2 up = ld2(oth + (r - 1) * RS + base);
        const uint2 dn = ld2(oth + (r + 1) * RS + base);
        // the in-row neighbours: next site (p = 1) or previous (p = 0), with
        // the halo byte beyond the row's 8 bytes
        const uint32_t e = *reinterpret_cast<const uint32_t*>(oth + r * RS + (p ? base + 8 : base - 4));
        const uint32_t s0 = p ? __builtin_amdgcn_alignbyte(ct.y, ct.x, 1) : __builtin_amdgcn_alignbyte(ct.x, e, 3);
        const uint32_t s1 = p ? __builtin_amdgcn_alignbyte(e, ct.y, 1) : __builtin_amdgcn_alignbyte(ct.y, ct.x, 3);
        uint2 fz = make_uint2(0u, 0u), bz = make_uint2(0u, 0u);
        if (D == 3) {
          fz = ld2(oth + (r - TR) * RS + base);
          bz = ld2(oth + (r + TR) * RS + base);
        }
        auto count = [&](uint32_t ow, uint32_t c0, uint32_t sh, uint32_t u, uint32_t d,
                         uint32_t f, uint32_t bk) {
          uint32_t k2 = ((ow ^ c0) & kBit1) + ((ow ^ sh) & kBit1) + ((ow ^ u) & kBit1) +
                        ((ow ^ d) & kBit1);
          if (D == 3) k2 += ((ow ^ f) & kBit1) + ((ow ^ bk) & kBit1);
          return k2 >> 1;
        };
        const uint32_t k0 = count(o.x, ct.x, s0, up.x, dn.x, fz.x, bz.x);
        const uint32_t k1 = count(o.y, ct.y, s1, up.y, dn.y, fz.y, bz.y);
        const uint2 nw = HB ? heatbath_half(tab, key, t, c, jbase, 2 * odd, o.x, o.y, k0, k1, 2 * D, h)
                            : update_half_now(tab, key, t, c, jbase, 2 * odd, o.x, o.y, k0, k1, h);
        *reinterpret_cast<uint2*>(own + r * RS + base) = nw;
      }
      __syncthreads();
    }
  }

  // write back the tiles' own rows of both colours
  for (uint32_t it = threadIdx.x; it < G * 2 * TROWS * 2; it += 256) {
    const uint32_t gw = it / (2 * TROWS * 2);
    const uint32_t bw = blockIdx.x * G + gw;
    if (bw >= ntiles) continue;
    uint32_t rest = it - gw * 2 * TROWS * 2;
    const uint32_t cc = rest / (TROWS * 2);
    rest -= cc * TROWS * 2;
    const uint32_t ri = rest / 2, wv = rest - ri * 2;
    uint32_t wx, wy, wz;
    coords(bw, wx, wy, wz);
    const uint32_t wry = 1 + ri % T, wrz = D == 3 ? 1 + ri / T : 0u;
    const uint32_t wr = wry + TR * wrz;
    const uint32_t yy = wy * T + wry - 1, zz = D == 3 ? wz * T + wrz - 1 : 0u;
    int8_t* dst = s + cc * Nh + ((uint64_t)zz * L + yy) * R + wx * (T / 2) + 4 * wv;
    *reinterpret_cast<uint32_t*>(dst) = *reinterpret_cast<const uint32_t*>(
        lds + gw * TB + (cc * NR + wr) * RS + 16 + 8 * (wx & 1u) + 4 * wv);
  }
}

// ---------------------------------------------------------------------------
// Exact ties of a bit-packed tile pass, resolved by the workgroup instead of
// by each lane: ballot prefix sums of the lanes' counts of tied sites number
// the sites within each wave, the four waves' totals go through LDS, thread
// i draws the refinement of tied site i and toggles the site in its owner's
// LDS word (an LDS atomic xor) if the move is accepted after all -- the
// owner stored the word with its ties refused (Metropolis: left as they
// were; heat bath: down).  A pass leaves about 30 tied sites a workgroup, so
// one wave draws where every wave did (a lane's own ties cost its wave one
// draw each, and some lane of a wave almost always has one).  A workgroup
// with a lane holding 8 or more tied sites, or more than `cap` in all (at
// most kTileTieCap; 0 takes this path always), lets each lane draw its own.
// Every thread of the 256-thread workgroup calls this once per pass, after
// storing its word; the caller's barrier after the pass orders the flips
// before the next reads.
// ---------------------------------------------------------------------------
constexpr uint32_t kTileTieCap = 512;  // entries of the workgroup's list of tied sites

struct TileTies {
  uint4 ent[256];             // per thread: k0, k1, first site, LDS index of its word
  uint32_t k2[256];           // per thread: k2 (classes of 4 or more, K2)
  uint16_t idx[kTileTieCap];  // thread | bit << 8
  uint32_t wsum[4];           // the waves' counts of tied sites
};

// ROWS8: bit b of a word is site base + (b >> 3) R + (b & 7) (four tile rows
// of 8 sites), else site base + b.  K2: a tied site's class can reach 4 (the
// general decision), else it is k0 + 2 k1 (the fast decision: only k < 2
// refuses).
template <bool ROWS8, bool K2>
__device__ __forceinline__ void tile_ties_group(TileTies& tt, uint32_t ties, uint32_t k0,
                                                uint32_t k1, uint32_t k2, uint32_t base, uint32_t R,
                                                uint32_t* words, uint32_t off, const TabRegs& tab,
                                                const RngKey& key, uint32_t t, uint32_t c,
                                                uint32_t h, uint32_t cap) {
  auto accepts = [&](uint32_t bs, uint32_t b, uint32_t kc) -> bool {
    const uint32_t js = ROWS8 ? bs + (b >> 3) * R + (b & 7u) : bs + b;
    const Rand4 rr = philox(js, t, key.replica, tag(c, kIsingRefine) | (h << 8), key.k0, key.k1);
    return (rr.w[0] & 0xFFFFFFu) < frac_sel(tab.fr, kc);
  };
  auto below = [](uint64_t b) -> uint32_t {
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(b >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)b, 0u));
  };
  const uint32_t lane = __lane_id(), wave = threadIdx.x >> 6;
  const uint32_t ns = (uint32_t)__builtin_popcount(ties);
  tt.ent[threadIdx.x] = make_uint4(k0, k1, base, off);
  if (K2) tt.k2[threadIdx.x] = k2;
  const bool few = __ballot(ns >= 8u) == 0;  // every lane's count fits three bits
  uint32_t wtotal = 0, first = 0;
  if (few) {
    const uint64_t b0 = __ballot(ns & 1u), b1 = __ballot(ns & 2u), b2 = __ballot(ns & 4u);
    wtotal = (uint32_t)__popcll(b0) + 2u * (uint32_t)__popcll(b1) + 4u * (uint32_t)__popcll(b2);
    first = below(b0) + 2u * below(b1) + 4u * below(b2);
  }
  if (lane == 0) tt.wsum[wave] = few ? wtotal : kTileTieCap + 1u;
  __syncthreads();
  const uint32_t s0 = tt.wsum[0], s1 = tt.wsum[1], s2 = tt.wsum[2], s3 = tt.wsum[3];
  const uint32_t total = s0 + s1 + s2 + s3;  // above kTileTieCap if any wave could not number
  if (total == 0u) return;  // the same for every thread
  if (total <= cap) {
    uint32_t k = first + (wave > 0 ? s0 : 0u) + (wave > 1 ? s1 : 0u) + (wave > 2 ? s2 : 0u);
    for (uint32_t m = ties; m; m &= m - 1)
      tt.idx[k++] = (uint16_t)(threadIdx.x | ((uint32_t)__builtin_ctz(m) << 8));
    __syncthreads();
    for (uint32_t r0 = 0; r0 < total; r0 += 256u) {
      const uint32_t i = r0 + threadIdx.x;
      if (i < total) {
        const uint32_t id = tt.idx[i], b = id >> 8;
        const uint4 en = tt.ent[id & 255u];
        const uint32_t kc = ((en.x >> b) & 1u) | (((en.y >> b) & 1u) << 1) |
                            (K2 ? ((tt.k2[id & 255u] >> b) & 1u) << 2 : 0u);
        if (accepts(en.z, b, kc)) atomicXor(words + en.w, 1u << b);
      }
    }
  } else {
    uint32_t flips = 0;
    for (uint32_t m = ties; m; m &= m - 1) {
      const uint32_t b = (uint32_t)__builtin_ctz(m);
      const uint32_t kc = ((k0 >> b) & 1u) | (((k1 >> b) & 1u) << 1) | (K2 ? ((k2 >> b) & 1u) << 2 : 0u);
      if (accepts(base, b, kc)) flips |= 1u << b;
    }
    if (flips) words[off] ^= flips;  // the lane's own word
  }
}

// ---------------------------------------------------------------------------
// Bit-packed tiles (2D, T % 64 == 0, uniform couplings, Metropolis or heat
// bath): a tile and its boundary layer sit in LDS at one bit per site.  Per
// colour, LDS row r (0 .. T + 1; rows 0 and T + 1 are the boundary rows)
// holds the T / 64 words of the tile row's T / 2 same-colour sites (site
// 32 i + b of the row in bit b of word i, bit 1 = spin -1), framed by a word
// with the site before the row in bit 31 and one with the site after it in
// bit 0, so the in-row neighbours are funnel shifts, as in the packed
// streaming kernel.  A lane owns one word of a tile row of each colour for
// all k hits and decides its 32 sites with that kernel's bit-sliced decision,
// drawing the same prefix bytes (the hit in the counter): Metropolis by the
// count of unsatisfied bonds, heat bath (HB) by the count of up neighbours,
// whose class threshold the prefix must stay below for the spin to come out
// up.  Exact ties take their refinement draws before the pass ends (shared
// by the workgroup, tile_ties_group).  Every site
// makes the int8 tile kernel's decision, so the chain is the same bit for
// bit.  T = 64 (a tile is one wave, four to a workgroup) or T = 128 (a tile
// is one 256-lane workgroup).
// ---------------------------------------------------------------------------
template <bool FAST, bool HB>
__global__ __launch_bounds__(256) void tile_packed_kernel(const Geom g, const RngKey key,
                                                          const IsingTable table, const uint32_t T,
                                                          const uint32_t hits, const uint32_t t,
                                                          const uint32_t tc, const uint32_t ntiles,
                                                          const uint32_t tie_cap,
                                                          int8_t* __restrict__ s) {
  extern __shared__ __align__(16) int8_t lds_raw[];
  const uint32_t L = (uint32_t)g.L, R = (uint32_t)g.R;
  const uint32_t WT = T / 64;            // tile words per row and colour
  const uint32_t RW = WT + 2;            // LDS words per row: frame, tile words, frame
  const uint32_t TR = T + 2;             // rows with the boundary rows
  const uint32_t PL = TR * RW;           // LDS words per colour
  const uint32_t items = T * WT;         // words a colour of one tile
  const uint32_t G = blockDim.x / items; // tiles of the workgroup (>= 1)
  const uint32_t gi = threadIdx.x / items, li = threadIdx.x - gi * items;
  const uint32_t bt = blockIdx.x * G + gi;  // tile of this lane among the colour's tiles
  const bool valid = bt < ntiles;
  uint32_t* lw = reinterpret_cast<uint32_t*>(lds_raw) + gi * 2u * PL;
  const uint32_t nt = L / T, half = nt / 2;
  const uint32_t bv = valid ? bt : 0u;
  const uint32_t ty = bv / half;
  const uint32_t tx = 2 * (bv - ty * half) + ((ty + tc) & 1u);
  const uint32_t X0 = tx * T, Y0 = ty * T;
  const uint32_t xw0 = X0 / 2;           // in-row index of the tile row's first site
  const uint64_t Nh = (uint64_t)g.Nh;
  auto prow = [&](uint32_t r) -> uint32_t { return (Y0 + L - 1 + r) % L; };  // plane row of LDS row r

  // stage: the tile words of every row (boundary rows included) and the frames
  if (valid) {
    for (uint32_t it = li; it < 2u * PL; it += items) {
      const uint32_t cc = it / PL, rest = it - cc * PL;
      const uint32_t r = rest / RW, i = rest - r * RW;
      const int8_t* src = s + cc * Nh + (uint64_t)prow(r) * R;
      uint32_t v = 0;
      if (i == 0) {
        v = src[xw0 == 0 ? R - 1 : xw0 - 1] < 0 ? 0x80000000u : 0u;
      } else if (i == RW - 1) {
        const uint32_t xr = xw0 + T / 2;
        v = src[xr == R ? 0 : xr] < 0 ? 1u : 0u;
      } else {
        const uint32_t* q = reinterpret_cast<const uint32_t*>(src + xw0 + 32u * (i - 1));
#pragma unroll
        for (int k = 0; k < 8; ++k) v |= gather7(q[k]) << (4 * k);
      }
      lw[it] = v;
    }
  }
  __syncthreads();

  const TabRegs tab = tab_regs(table);
  FastTab ft;
  if (FAST) ft = fast_tab<2>(tab);
  const uint32_t ry = 1 + li / WT, i = 1 + li % WT;  // the lane's LDS row and word
  const uint32_t y = Y0 + ry - 1;
  const uint32_t rb = ry * RW + i;
  const uint32_t wi = (y * R + xw0) / 32u + (i - 1);  // global word index (R % 32 == 0)
  __shared__ TileTies tt;
  uint32_t* const words = reinterpret_cast<uint32_t*>(lds_raw);
  for (uint32_t h = 0; h < hits; ++h) {
#pragma unroll
    for (uint32_t c = 0; c < 2; ++c) {
      uint32_t ties = 0, k0 = 0, k1 = 0, k2 = 0, off = 0;
      if (valid) {
        uint32_t* own = lw + c * PL;
        const uint32_t* oth = lw + (1 - c) * PL;
        const uint32_t p = (c + y) & 1u;
        const uint32_t o = own[rb], ct = oth[rb], en = oth[rb + 1], ep = oth[rb - 1];
        const uint32_t up = oth[rb - RW], dn = oth[rb + RW];
        // x + 1 neighbours (p = 1: next in-row site) and x - 1 (p = 0: previous)
        const uint32_t sh_next = __builtin_amdgcn_alignbit(en, ct, 1u);
        const uint32_t sh_prev = __builtin_amdgcn_alignbit(ct, ep, 31u);
        const uint32_t nxp = mask_sel(ct, sh_next, p), nxm = mask_sel(sh_prev, ct, p);
        // Metropolis: the unsatisfied bonds (class k = their count); heat
        // bath: the up neighbours (bit 0; class = their number), whose
        // table's threshold is that of the spin coming out up
        const uint32_t u[6] = {HB ? ~nxp : o ^ nxp, HB ? ~nxm : o ^ nxm, HB ? ~dn : o ^ dn,
                               HB ? ~up : o ^ up, 0u, 0u};
        count_planes<2>(u, k0, k1, k2);
        // `flip`: Metropolis, the accepted flips; heat bath, the sites coming
        // out up -- exact ties refused, resolved below
        const uint32_t flip = FAST ? packed_decide_fast<2>(ft, key, t, c, wi, k0, k1, k2, ties, h)
                                   : packed_decide<2>(tab, key, t, c, wi, k0, k1, k2, ties, h);
        own[rb] = HB ? ~flip : o ^ flip;
        off = (uint32_t)(own - words) + rb;
      }
      tile_ties_group<false, !FAST>(tt, ties, k0, k1, k2, wi * 32u, R, words, off, tab, key, t, c, h,
                                    tie_cap);
      __syncthreads();
    }
  }

  // write back the tile rows of both colours as +-1 bytes
  if (valid) {
    for (uint32_t it = li; it < 2u * items; it += items) {
      const uint32_t cc = it / items, rest = it - cc * items;
      const uint32_t r = 1 + rest / WT, w = 1 + rest % WT;
      const uint32_t v = lw[cc * PL + r * RW + w];
      uint32_t* dst = reinterpret_cast<uint32_t*>(s + cc * Nh + (uint64_t)(Y0 + r - 1) * R + xw0 +
                                                  32u * (w - 1));
#pragma unroll
      for (int k = 0; k < 8; ++k) {
        const uint32_t spread = (((v >> (4 * k)) & 0xFu) * 0x00204081u) & kOnes;
        dst[k] = kOnes | (spread * 0xFEu);
      }
    }
  }
}

// ---------------------------------------------------------------------------
// Bit-packed 16 x 16 tiles (2D, Metropolis or heat bath): a tile row holds 8 sites of a
// colour, so a word packs four tile rows -- word i of a tile's colour holds
// rows 4i .. 4i + 3 of the tile, site s of row r in bit 8 r + s (bit 1 = spin
// -1).  Per tile and colour, LDS holds the column [above, w0, w1, w2, w3,
// below] (the boundary row above the tile in bits 24..31 of `above`, the one
// below in bits 0..7 of `below`, so the y neighbours of word i are 8-bit
// funnel shifts of its column) and per word the sites left and right of its
// rows (bit 8 r and bit 8 r + 7), which complete the in-row neighbours, a
// shift by one within each byte.  Row r of a word has parity (c + r) & 1
// (tiles start at even rows), a per-byte mask.  A row's 8 prefix bytes are
// words 2 h0, 2 h0 + 1 of its 16-site Philox block, as in the int8 16 x 16
// kernel, so a word takes four blocks; the transpose to bit planes and the
// compare are the packed kernel's.  Exact ties take their refinement draws
// before the pass ends, as in the tiles of 64.  Four lanes a tile, 64 tiles a
// workgroup.
// ---------------------------------------------------------------------------
constexpr uint32_t kT16Words = 14;  // per tile and colour: column (6), left (4), right (4)

template <bool FAST, bool HB>
__global__ __launch_bounds__(256) void tile16_packed_kernel(const Geom g, const RngKey key,
                                                            const IsingTable table,
                                                            const uint32_t hits, const uint32_t t,
                                                            const uint32_t tc, const uint32_t ntiles,
                                                            const uint32_t tie_cap,
                                                            int8_t* __restrict__ s) {
  __shared__ uint32_t lw[64 * 2 * kT16Words];
  const uint32_t L = (uint32_t)g.L, R = (uint32_t)g.R;
  const uint32_t gi = threadIdx.x >> 2, i = threadIdx.x & 3u;  // tile of the workgroup, word
  const uint32_t bt = blockIdx.x * 64u + gi;
  const bool valid = bt < ntiles;
  const uint32_t half = L / 32;  // tiles of one colour per tile row
  const uint32_t bv = valid ? bt : 0u;
  const uint32_t ty = bv / half;
  const uint32_t tx = 2 * (bv - ty * half) + ((ty + tc) & 1u);
  const uint32_t Y0 = ty * 16, x0 = tx * 8;  // first row; in-row index of the tile row's first site
  const uint64_t Nh = (uint64_t)g.Nh;
  uint32_t* tw = lw + gi * 2u * kT16Words;   // colour c at tw + c * kT16Words
  auto bits8 = [&](const int8_t* row) -> uint32_t {  // sign bits of 8 sites
    const uint2 v = *reinterpret_cast<const uint2*>(row);
    return gather7(v.x) | (gather7(v.y) << 4);
  };
  // stage: lane i of the tile fills word i of both colours, its left and right
  // sites, and (lanes 0 and 3) the boundary rows
  if (valid) {
#pragma unroll
    for (uint32_t cc = 0; cc < 2; ++cc) {
      uint32_t* col = tw + cc * kT16Words;
      const int8_t* pl = s + cc * Nh;
      uint32_t w = 0, lh = 0, rh = 0;
      const uint32_t xl = x0 == 0 ? R - 1 : x0 - 1, xr = x0 + 8 == R ? 0 : x0 + 8;
#pragma unroll
      for (uint32_t r = 0; r < 4; ++r) {
        const int8_t* row = pl + (uint64_t)(Y0 + 4 * i + r) * R;
        w |= bits8(row + x0) << (8 * r);
        lh |= (row[xl] < 0 ? 1u : 0u) << (8 * r);
        rh |= (row[xr] < 0 ? 0x80u : 0u) << (8 * r);
      }
      col[1 + i] = w;
      col[6 + i] = lh;
      col[10 + i] = rh;
      if (i == 0) col[0] = bits8(pl + (uint64_t)(Y0 == 0 ? L - 1 : Y0 - 1) * R + x0) << 24;
      if (i == 3) col[5] = bits8(pl + (uint64_t)(Y0 + 16 == L ? 0 : Y0 + 16) * R + x0);
    }
  }
  __syncthreads();

  const TabRegs tab = tab_regs(table);
  FastTab ft;
  if (FAST) ft = fast_tab<2>(tab);
  const uint32_t j0 = (Y0 + 4 * i) * R + x0;  // in-colour index of the word's first site
  __shared__ TileTies tt;
  for (uint32_t h = 0; h < hits; ++h) {
#pragma unroll
    for (uint32_t c = 0; c < 2; ++c) {
      uint32_t ties = 0, k0 = 0, k1 = 0, k2 = 0;
      if (valid) {
        uint32_t* own = tw + c * kT16Words;
        const uint32_t* oth = tw + (1 - c) * kT16Words;
        const uint32_t o = own[1 + i], ct = oth[1 + i];
        const uint32_t up = __builtin_amdgcn_alignbit(ct, oth[i], 24u);    // rows r - 1
        const uint32_t dn = __builtin_amdgcn_alignbit(oth[2 + i], ct, 8u);  // rows r + 1
        const uint32_t sh_next = ((ct >> 1) & 0x7F7F7F7Fu) | oth[10 + i];   // site + 1 in its row
        const uint32_t sh_prev = ((ct << 1) & 0xFEFEFEFEu) | oth[6 + i];    // site - 1
        // rows of parity 1 (x + 1 = next site): rows 1, 3 for colour 0, rows 0, 2 for colour 1
        constexpr uint32_t P1[2] = {0xFF00FF00u, 0x00FF00FFu};
        const uint32_t pm = P1[c];
        const uint32_t nxp = (ct & ~pm) | (sh_next & pm);
        const uint32_t nxm = (sh_prev & ~pm) | (ct & pm);
        // Metropolis: the unsatisfied bonds; heat bath: the up neighbours
        const uint32_t u[6] = {HB ? ~nxp : o ^ nxp, HB ? ~nxm : o ^ nxm, HB ? ~dn : o ^ dn,
                               HB ? ~up : o ^ up, 0u, 0u};
        count_planes<2>(u, k0, k1, k2);
        // prefix bytes: row r's 8 sites are words 2 h0, 2 h0 + 1 of block j >> 4
        uint32_t P[8];
#pragma unroll
        for (uint32_t r = 0; r < 4; ++r) {
          const uint32_t jr = j0 + r * R;
          const Rand4 rb = philox(jr >> 4, t, key.replica, tag(c, kIsingPrefix) | (h << 8), key.k0,
                                  key.k1);
          const bool h0 = ((jr >> 3) & 1u) != 0;
          P[2 * r] = h0 ? rb.w[2] : rb.w[0];
          P[2 * r + 1] = h0 ? rb.w[3] : rb.w[1];
        }
        uint32_t B[8];
        prefix_planes(P, B);
        // exact ties refused, resolved below
        const uint32_t flip = FAST ? packed_compare_fast<2>(ft, B, k0, k1, k2, ties)
                                   : packed_compare<2>(tab, B, k0, k1, k2, ties);
        own[1 + i] = HB ? ~flip : o ^ flip;
      }
      tile_ties_group<true, !FAST>(tt, ties, k0, k1, k2, j0, R, lw,
                                   gi * 2u * kT16Words + c * kT16Words + 1u + i, tab, key, t, c,
                                   h, tie_cap);
      __syncthreads();
    }
  }

  // write back word i of both colours: four rows of 8 sites as +-1 bytes
  if (valid) {
#pragma unroll
    for (uint32_t cc = 0; cc < 2; ++cc) {
      const uint32_t v = tw[cc * kT16Words + 1 + i];
#pragma unroll
      for (uint32_t r = 0; r < 4; ++r) {
        const uint32_t byte = (v >> (8 * r)) & 0xFFu;
        uint32_t q[2];
#pragma unroll
        for (int k = 0; k < 2; ++k) {
          const uint32_t spread = (((byte >> (4 * k)) & 0xFu) * 0x00204081u) & kOnes;
          q[k] = kOnes | (spread * 0xFEu);
        }
        *reinterpret_cast<uint2*>(s + cc * Nh + (uint64_t)(Y0 + 4 * i + r) * R + x0) =
            make_uint2(q[0], q[1]);
      }
    }
  }
}

// ---------------------------------------------------------------------------
// Bit-packed 16^3 tiles (3D, Metropolis or heat bath): each of the tile's 16
// z-planes is laid out as a 16 x 16 tile of the 2D kernel above -- per colour
// the column [above, w0, w1, w2, w3, below] and the left and right sites of
// each word's four rows -- plus the words w0 .. w3 of the boundary planes
// below and above the tile.  A lane owns word i of plane z (rows 4 i .. 4 i +
// 3 of that plane); its z-neighbours are the other colour's words at the same
// place in planes z - 1 and z + 1 (the in-row index of a site's z-neighbour
// is its own), its y- and in-row neighbours those of the 2D kernel, with the
// rows' parity (c + r + z) mod 2 (tiles start at even rows and planes).  A
// tile is one wave (16 planes x 4 words), four tiles a workgroup.
// ---------------------------------------------------------------------------
constexpr uint32_t kT3Planes = 18;  // the tile's 16 planes and the two boundary planes

template <bool FAST, bool HB>
__global__ __launch_bounds__(256) void tile16_packed3d_kernel(const Geom g, const RngKey key,
                                                              const IsingTable table,
                                                              const uint32_t hits, const uint32_t t,
                                                              const uint32_t tc,
                                                              const uint32_t ntiles,
                                                              const uint32_t tie_cap,
                                                              int8_t* __restrict__ s) {
  constexpr uint32_t CW = kT3Planes * kT16Words;  // words of a colour of one tile
  __shared__ uint32_t lw[4 * 2 * CW];
  const uint32_t L = (uint32_t)g.L, R = (uint32_t)g.R;
  const uint32_t gi = threadIdx.x >> 6, z = (threadIdx.x >> 2) & 15u, i = threadIdx.x & 3u;
  const uint32_t bt = blockIdx.x * 4u + gi;
  const bool valid = bt < ntiles;
  const uint32_t nt = L / 16, half = nt / 2;
  const uint32_t bv = valid ? bt : 0u;
  const uint32_t tz = bv / (nt * half), rem = bv - tz * nt * half;
  const uint32_t ty = rem / half;
  const uint32_t tx = 2 * (rem - ty * half) + ((ty + tz + tc) & 1u);
  const uint32_t Z0 = tz * 16, Y0 = ty * 16, x0 = tx * 8;
  const uint32_t Zg = Z0 + z;  // the lane's plane
  const uint64_t Nh = (uint64_t)g.Nh;
  uint32_t* tw = lw + gi * 2u * CW;  // colour c, plane zz (0: below the tile) at tw + c CW + zz 14
  auto bits8 = [&](const int8_t* row) -> uint32_t {  // sign bits of 8 sites
    const uint2 v = *reinterpret_cast<const uint2*>(row);
    return gather7(v.x) | (gather7(v.y) << 4);
  };
  auto rowp = [&](const int8_t* pl, uint32_t zg, uint32_t y) -> const int8_t* {
    return pl + ((uint64_t)zg * L + y) * R;
  };
  // stage: lane (z, i) fills word i of plane z of both colours, its left and
  // right sites, the boundary rows (i = 0 and 3) and the boundary planes'
  // word i (z = 0 and 15)
  if (valid) {
#pragma unroll
    for (uint32_t cc = 0; cc < 2; ++cc) {
      uint32_t* col = tw + cc * CW + (z + 1) * kT16Words;
      const int8_t* pl = s + cc * Nh;
      uint32_t w = 0, lh = 0, rh = 0;
      const uint32_t xl = x0 == 0 ? R - 1 : x0 - 1, xr = x0 + 8 == R ? 0 : x0 + 8;
#pragma unroll
      for (uint32_t r = 0; r < 4; ++r) {
        const int8_t* row = rowp(pl, Zg, Y0 + 4 * i + r);
        w |= bits8(row + x0) << (8 * r);
        lh |= (row[xl] < 0 ? 1u : 0u) << (8 * r);
        rh |= (row[xr] < 0 ? 0x80u : 0u) << (8 * r);
      }
      col[1 + i] = w;
      col[6 + i] = lh;
      col[10 + i] = rh;
      if (i == 0) col[0] = bits8(rowp(pl, Zg, Y0 == 0 ? L - 1 : Y0 - 1) + x0) << 24;
      if (i == 3) col[5] = bits8(rowp(pl, Zg, Y0 + 16 == L ? 0 : Y0 + 16) + x0);
      if (z == 0 || z == 15) {
        const uint32_t zb = z == 0 ? (Z0 == 0 ? L - 1 : Z0 - 1) : (Z0 + 16 == L ? 0 : Z0 + 16);
        uint32_t wb = 0;
#pragma unroll
        for (uint32_t r = 0; r < 4; ++r) wb |= bits8(rowp(pl, zb, Y0 + 4 * i + r) + x0) << (8 * r);
        tw[cc * CW + (z == 0 ? 0u : kT3Planes - 1) * kT16Words + 1 + i] = wb;
      }
    }
  }
  __syncthreads();

  const TabRegs tab = tab_regs(table);
  FastTab ft;
  if (FAST) ft = fast_tab<3>(tab);
  const uint32_t j0 = ((uint32_t)Zg * L + Y0 + 4 * i) * R + x0;  // in-colour index of the word's first site
  __shared__ TileTies tt;
  for (uint32_t h = 0; h < hits; ++h) {
#pragma unroll
    for (uint32_t c = 0; c < 2; ++c) {
      uint32_t ties = 0, k0 = 0, k1 = 0, k2 = 0;
      if (valid) {
        uint32_t* own = tw + c * CW + (z + 1) * kT16Words;
        const uint32_t* oth = tw + (1 - c) * CW + (z + 1) * kT16Words;
        const uint32_t o = own[1 + i], ct = oth[1 + i];
        const uint32_t up = __builtin_amdgcn_alignbit(ct, oth[i], 24u);    // rows r - 1
        const uint32_t dn = __builtin_amdgcn_alignbit(oth[2 + i], ct, 8u);  // rows r + 1
        const uint32_t fz = oth[1 + i - kT16Words], bz = oth[1 + i + kT16Words];  // planes z -+ 1
        const uint32_t sh_next = ((ct >> 1) & 0x7F7F7F7Fu) | oth[10 + i];   // site + 1 in its row
        const uint32_t sh_prev = ((ct << 1) & 0xFEFEFEFEu) | oth[6 + i];    // site - 1
        // rows of parity 1 (x + 1 = next site): rows 1, 3 when c + z is even, rows 0, 2 when odd
        const uint32_t pm = ((c + z) & 1u) ? 0x00FF00FFu : 0xFF00FF00u;
        const uint32_t nxp = (ct & ~pm) | (sh_next & pm);
        const uint32_t nxm = (sh_prev & ~pm) | (ct & pm);
        // Metropolis: the unsatisfied bonds; heat bath: the up neighbours
        const uint32_t u[6] = {HB ? ~nxp : o ^ nxp, HB ? ~nxm : o ^ nxm, HB ? ~dn : o ^ dn,
                               HB ? ~up : o ^ up,   HB ? ~bz : o ^ bz,   HB ? ~fz : o ^ fz};
        count_planes<3>(u, k0, k1, k2);
        // prefix bytes: row r's 8 sites are words 2 h0, 2 h0 + 1 of block j >> 4
        uint32_t P[8];
#pragma unroll
        for (uint32_t r = 0; r < 4; ++r) {
          const uint32_t jr = j0 + r * R;
          const Rand4 rb = philox(jr >> 4, t, key.replica, tag(c, kIsingPrefix) | (h << 8), key.k0,
                                  key.k1);
          const bool h0 = ((jr >> 3) & 1u) != 0;
          P[2 * r] = h0 ? rb.w[2] : rb.w[0];
          P[2 * r + 1] = h0 ? rb.w[3] : rb.w[1];
        }
        uint32_t B[8];
        prefix_planes(P, B);
        // exact ties refused, resolved below
        const uint32_t flip = FAST ? packed_compare_fast<3>(ft, B, k0, k1, k2, ties)
                                   : packed_compare<3>(tab, B, k0, k1, k2, ties);
        own[1 + i] = HB ? ~flip : o ^ flip;
      }
      tile_ties_group<true, !FAST>(tt, ties, k0, k1, k2, j0, R, lw,
                                   gi * 2u * CW + c * CW + (z + 1) * kT16Words + 1u + i, tab, key,
                                   t, c, h, tie_cap);
      __syncthreads();
    }
  }

  // write back word i of plane z of both colours: four rows of 8 sites as +-1 bytes
  if (valid) {
#pragma unroll
    for (uint32_t cc = 0; cc < 2; ++cc) {
      const uint32_t v = tw[cc * CW + (z + 1) * kT16Words + 1 + i];
#pragma unroll
      for (uint32_t r = 0; r < 4; ++r) {
        const uint32_t byte = (v >> (8 * r)) & 0xFFu;
        uint32_t q[2];
#pragma unroll
        for (int k = 0; k < 2; ++k) {
          const uint32_t spread = (((byte >> (4 * k)) & 0xFu) * 0x00204081u) & kOnes;
          q[k] = kOnes | (spread * 0xFEu);
        }
        *reinterpret_cast<uint2*>(s + cc * Nh + ((uint64_t)Zg * L + Y0 + 4 * i + r) * R + x0) =
            make_uint2(q[0], q[1]);
      }
    }
  }
}

bool tile_packed_supported(const Geom& g, uint32_t T, bool heatbath) {
  (void)heatbath;  // both rules
  const bool shape = g.d == 2 ? (T == 16 || T == 64 || T == 128) : (g.d == 3 && T == 16);
  return shape && (uint32_t)g.L % T == 0 && ((uint32_t)g.L / T) % 2 == 0;
}

// 256 lanes a workgroup: four tiles of 64 (64 words a colour each) or one of 128
static uint32_t tile_packed_group(uint32_t T) { return T == 64 ? 4u : 1u; }

static size_t tile_packed_lds_bytes(uint32_t T) {
  return (size_t)tile_packed_group(T) * 2 * (T + 2) * (T / 64 + 2) * 4;
}

size_t tile_lds_bytes(int d, uint32_t T) {
  const size_t TR = T + 2;
  if (T == 16) {  // 48-byte rows, 256 / 16^(d-1) tiles per workgroup
    const size_t G = d == 3 ? 1 : 16;
    return G * 2 * (d == 3 ? TR * TR : TR) * 48;
  }
  return 2 * (d == 3 ? TR * TR : TR) * (T / 2 + 32);
}

bool tile_supported(const Geom& g, uint32_t T) {
  return (T == 16 || (T >= 32 && T % 32 == 0)) && (uint32_t)g.L % T == 0 &&
         ((uint32_t)g.L / T) % 2 == 0 && tile_lds_bytes(g.d, T) <= 160 * 1024;
}

static const void* tile_fn(int d, bool hb, bool t16) {
  if (t16) {
    if (d == 2) return hb ? (const void*)tile16_kernel<2, true> : (const void*)tile16_kernel<2, false>;
    return hb ? (const void*)tile16_kernel<3, true> : (const void*)tile16_kernel<3, false>;
  }
  if (d == 2) return hb ? (const void*)tile_kernel<2, true> : (const void*)tile_kernel<2, false>;
  return hb ? (const void*)tile_kernel<3, true> : (const void*)tile_kernel<3, false>;
}

hipError_t tile_allow_lds(int d, size_t bytes) {
  for (int t16 = 0; t16 < 2; ++t16)
    for (int hb = 0; hb < 2; ++hb) {
      const hipError_t e = allow_dynamic_lds(tile_fn(d, hb != 0, t16 != 0), bytes);
      if (e != hipSuccess) return e;
    }
  return hipSuccess;
}

// One tile-colour pass (k hits) of the tiled schedule; `packed`: the bit-packed
// kernel where it applies.
hipError_t launch_tile_pass(const IsingLaunch& a, bool heatbath, uint32_t T, uint32_t hits,
                            int8_t* spins, uint32_t t, uint32_t tc, hipStream_t st, bool packed) {
  const uint32_t nt = (uint32_t)a.g.L / T;
  const uint32_t tiles = (a.g.d == 3 ? nt * nt * nt : nt * nt) / 2;
  if (packed && tile_packed_supported(a.g, T, heatbath)) {
    // the fast decision when every class k >= d always accepts (J0 > 0)
    bool fast = true;
    for (int k = a.g.d; k <= 2 * a.g.d; ++k)
      if ((((k < 4 ? a.tab.al_lo : a.tab.al_hi) >> (8 * (k & 3))) & 0xFFu) != 0xFFu) fast = false;
    // the workgroup's list of tied sites (packed_ties other than 0: each lane its own)
    const uint32_t tie_cap = a.packed_ties == 0 ? kTileTieCap : 0u;
    if (T == 16 && a.g.d == 3) {
      const dim3 grid((tiles + 3) / 4), block(256);
      if (heatbath)
        hipLaunchKernelGGL((tile16_packed3d_kernel<false, true>), grid, block, 0, st, a.g, a.key, a.tab,
                           hits, t, tc, tiles, tie_cap, spins);
      else if (fast)
        hipLaunchKernelGGL((tile16_packed3d_kernel<true, false>), grid, block, 0, st, a.g, a.key, a.tab,
                           hits, t, tc, tiles, tie_cap, spins);
      else
        hipLaunchKernelGGL((tile16_packed3d_kernel<false, false>), grid, block, 0, st, a.g, a.key, a.tab,
                           hits, t, tc, tiles, tie_cap, spins);
      return hipGetLastError();
    }
    if (T == 16) {
      const dim3 grid((tiles + 63) / 64), block(256);
      if (heatbath)
        hipLaunchKernelGGL((tile16_packed_kernel<false, true>), grid, block, 0, st, a.g, a.key, a.tab, hits, t,
                           tc, tiles, tie_cap, spins);
      else if (fast)
        hipLaunchKernelGGL((tile16_packed_kernel<true, false>), grid, block, 0, st, a.g, a.key, a.tab, hits, t,
                           tc, tiles, tie_cap, spins);
      else
        hipLaunchKernelGGL((tile16_packed_kernel<false, false>), grid, block, 0, st, a.g, a.key, a.tab, hits, t,
                           tc, tiles, tie_cap, spins);
      return hipGetLastError();
    }
    const uint32_t G = tile_packed_group(T);
    const dim3 grid((tiles + G - 1) / G), block(256);
    const size_t lds = tile_packed_lds_bytes(T);
    if (heatbath)
      hipLaunchKernelGGL((tile_packed_kernel<false, true>), grid, block, lds, st, a.g, a.key, a.tab, T, hits, t,
                         tc, tiles, tie_cap, spins);
    else if (fast)
      hipLaunchKernelGGL((tile_packed_kernel<true, false>), grid, block, lds, st, a.g, a.key, a.tab, T, hits, t,
                         tc, tiles, tie_cap, spins);
    else
      hipLaunchKernelGGL((tile_packed_kernel<false, false>), grid, block, lds, st, a.g, a.key, a.tab, T, hits, t,
                         tc, tiles, tie_cap, spins);
    return hipGetLastError();
  }
  if (T == 16) {
    const uint32_t G = a.g.d == 3 ? 1 : 16;
    const dim3 grid((tiles + G - 1) / G), block(256);
    const size_t lds = tile_lds_bytes(a.g.d, 16);
    if (a.g.d == 2) {
      if (heatbath)
        hipLaunchKernelGGL((tile16_kernel<2, true>), grid, block, lds, st, a.g, a.key, a.tab, hits, t, tc, tiles, spins);
      else
        hipLaunchKernelGGL((tile16_kernel<2, false>), grid, block, lds, st, a.g, a.key, a.tab, hits, t, tc, tiles, spins);
    } else {
      if (heatbath)
        hipLaunchKernelGGL((tile16_kernel<3, true>), grid, block, lds, st, a.g, a.key, a.tab, hits, t, tc, tiles, spins);
      else
        hipLaunchKernelGGL((tile16_kernel<3, false>), grid, block, lds, st, a.g, a.key, a.tab, hits, t, tc, tiles, spins);
    }
    return hipGetLastError();
  }
  const uint32_t cpr = T / 32;
  const uint32_t nchunks = (a.g.d == 3 ? T * T : T) * cpr;
  const uint32_t threads = nchunks >= 256 ? 256 : (nchunks + 63) / 64 * 64;
  const size_t lds = tile_lds_bytes(a.g.d, T);
  const dim3 grid(tiles), block(threads);
  if (a.g.d == 2) {
    if (heatbath)
      hipLaunchKernelGGL((tile_kernel<2, true>), grid, block, lds, st, a.g, a.key, a.tab, T, hits, t, tc, spins);
    else
      hipLaunchKernelGGL((tile_kernel<2, false>), grid, block, lds, st, a.g, a.key, a.tab, T, hits, t, tc, spins);
  } else {
    if (heatbath)
      hipLaunchKernelGGL((tile_kernel<3, true>), grid, block, lds, st, a.g, a.key, a.tab, T, hits, t, tc, spins);
    else
      hipLaunchKernelGGL((tile_kernel<3, false>), grid, block, lds, st, a.g, a.key, a.tab, T, hits, t, tc, spins);
  }
  return hipGetLastError();
}

}  // namespace smc
