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
#include "chunk.hpp"

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

// One tile-colour pass (k hits) of the tiled schedule.
hipError_t launch_tile_pass(const IsingLaunch& a, bool heatbath, uint32_t T, uint32_t hits,
                            int8_t* spins, uint32_t t, uint32_t tc, hipStream_t st) {
  const uint32_t nt = (uint32_t)a.g.L / T;
  const uint32_t tiles = (a.g.d == 3 ? nt * nt * nt : nt * nt) / 2;
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
