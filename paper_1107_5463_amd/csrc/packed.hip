// packed.hip -- Ising spins at one bit per site (multi-spin coding, Sec. 2:
// many spins per machine word), computing exactly the chain of the int8
// kernels.
//
// Layout: the colour-split planes of the int8 layout with 32 consecutive
// same-colour sites per 32-bit word, site j of a plane in bit j & 31 of word
// j >> 5; bit 1 = spin -1.  A plane row (L/2 sites) is W = L/64 words.  +-1
// couplings use the same layout per (mu, colour) plane, bit 1 = J = -1.
//
// Half-sweep: a lane owns one word column of its colour and walks a band of H
// rows, as the int8 streaming kernel does.  Per word (32 sites):
//  * the unsatisfied bonds of the 2d neighbours are the xor of the two spin
//    bits (and the coupling's sign bit); the x-neighbour word is the other
//    colour's word shifted by one bit with the adjacent word's edge bit
//    (v_alignbit);
//  * the count k of unsatisfied bonds is a bit-sliced sum: three bit planes
//    k0, k1, k2 for 32 sites at once (full adders as v_bitop3);
//  * the same two Philox blocks as the int8 path give the 32 prefix bytes,
//    transposed into 8 bit planes (a byte transpose with v_perm, then three
//    bit swaps between word pairs); the threshold bytes of the sites' classes
//    (those whose move can be refused: at most d of the 2d + 1) are laid out
//    as 8 bit planes too, and one bit-sliced compare against them gives the
//    refused sites and the exact ties;
//  * exact ties (prefix byte == threshold byte, 2^-8 of refusable moves) are
//    queued in LDS once their word is stored and resolved at the end of the
//    band with each site's 24-bit refinement draw, as in the int8 kernel.
#include <type_traits>

#include "chunk.hpp"
#include "packed.hpp"
#include "reduce.hpp"

namespace smc {

// Per-lane queue of the words with exact ties: a slot holds the word's tie
// mask and its count planes (for the classes of the tied sites) and the row
// in the band -- or, when only the classes k < d can refuse a move (k2 = 0 at
// every tied site, the fast decision) and WSLOT is set, the tie mask, k0, k1
// and the word's index.  A word is queued without a branch (its slot is
// written and the count advances only if it has ties); the ties are resolved
// when the queue is full and at the end of the band.
constexpr uint32_t kTieWords = 4;

__device__ __forceinline__ int32_t popc(uint32_t v) { return __builtin_popcount(v); }

struct PackedTies {
  uint4* ent;       // ent[slot * stride]: (ties, k0, k1, k2), or (ties, k0, k1, word index) with WSLOT
  uint8_t* rows;    // rows[slot * stride]: row in the band
  uint32_t stride, n, base, W;  // base: word index of the lane's column in row 0
  int64_t dE, dM;
  // wave resolution of a measured launch: flipped tied sites, their k0 and
  // k1 bits, and how many of them held s = -1 (k2 = 0 at every tied site)
  uint32_t tf, tk0, tk1, tset;
};

// Class k of tied site b of a queued word.
template <bool WSLOT>
__device__ __forceinline__ uint32_t tie_class(const uint4& en, uint32_t b) {
  return ((en.y >> b) & 1u) | (((en.z >> b) & 1u) << 1) | (WSLOT ? 0u : ((en.w >> b) & 1u) << 2);
}

template <int D, bool MEASURE, bool WSLOT = false>
__device__ __forceinline__ void packed_tie_flush(PackedTies& q, const TabRegs& tab,
                                                 const RngKey& key, uint32_t t, uint32_t c,
                                                 uint32_t* own) {
  for (uint32_t e = 0; e < q.n; ++e) {
    const uint4 en = q.ent[e * q.stride];
    const uint32_t wi = WSLOT ? en.w : q.base + (uint32_t)q.rows[e * q.stride] * q.W;
    uint32_t m = en.x;
    uint32_t word = 0, flips = 0;
    if (MEASURE) word = own[wi];
    while (m) {
      const uint32_t b = __builtin_ctz(m);
      m &= m - 1;
      const uint32_t k = tie_class<WSLOT>(en, b);
      const uint32_t js = wi * 32u + b;
      const Rand4 rr = philox(js, t, key.replica, tag(c, kIsingRefine), key.k0, key.k1);
      if ((rr.w[0] & 0xFFFFFFu) < frac_sel(tab.fr, k)) {
        flips |= 1u << b;
        if (MEASURE) {
          const int v = (word >> b) & 1u ? -1 : 1;  // a tied site was left unflipped
          q.dE += 4 * (int64_t)(D - (int)k);
          q.dM -= 2 * (int64_t)v;
        }
      }
    }
    if (flips) own[wi] ^= flips;  // the lane's own word, stored earlier by this lane
  }
  q.n = 0;
}

// Queue a stored word's exact ties: its slot is written in any case and the
// count advances only if there are ties; a full queue is resolved at once (its
// flips go to words already stored).
template <int D, bool MEASURE, bool WSLOT = false>
__device__ __forceinline__ void packed_queue_word(PackedTies& q, uint32_t ties, uint32_t row,
                                                  uint32_t wi, uint32_t k0, uint32_t k1,
                                                  uint32_t k2, const TabRegs& tab,
                                                  const RngKey& key, uint32_t t, uint32_t c,
                                                  uint32_t* own) {
  q.ent[q.n * q.stride] = make_uint4(ties, k0, k1, WSLOT ? wi : k2);
  if (!WSLOT) q.rows[q.n * q.stride] = (uint8_t)row;
  q.n += ties != 0u ? 1u : 0u;
  if (q.n == kTieWords) packed_tie_flush<D, MEASURE, WSLOT>(q, tab, key, t, c, own);
}

// End-of-band resolution shared by the workgroup (WSLOT slots): the
// workgroup's tied sites are numbered in thread order (a ballot prefix sum of
// the lanes' counts of tied sites within each wave, the waves' totals through
// LDS), thread i draws the refinement of tied site i and clears that site's
// bit in its word's slot if the move stays refused, and each lane then
// applies the flips left in the slots of its own words.  The workgroup so
// spends one round of refinement draws per 256 tied sites: a band of 4 rows
// leaves about 30 per wave, so two of the four waves draw and two wait at the
// barrier, and every spin word is still written by the lane that owns it.
// A workgroup with a lane holding 8 or more tied sites, or more than
// `cap` tied sites in all (at most 256 kTieWords; 0 takes this path always),
// resolves wave by wave instead: the wave numbers its tied words and lane i
// draws every tied site of word i.  `idx`
// is the workgroup's list of 256 kTieWords entries in LDS -- thread | slot
// << 8 | the site's bit << 10 when sites are numbered, lane | slot << 6 in a
// wave's quarter when words are -- and `wsum` four words of LDS for the
// waves' totals.  Every thread of the workgroup calls this once.  MEASURE:
// the owner adds what its words' tie flips change -- each flipped site with
// k unsatisfied bonds raises E by 4 (d - k) and moves M by -2 s.
template <int D, bool MEASURE>
__device__ __forceinline__ void packed_tie_flush_group(PackedTies& q, const TabRegs& tab,
                                                       const RngKey& key, uint32_t t, uint32_t c,
                                                       uint32_t* own, uint16_t* idx,
                                                       uint4* ent, uint32_t* wsum, uint32_t cap) {
  static_assert(kTieWords <= 4, "queue length fits the two slot bits of an index entry");
  constexpr uint32_t kCap = kTieWords * 256u;  // entries of the workgroup's list
  const uint32_t lane = __lane_id(), wave = threadIdx.x >> 6;
  const uint32_t n = q.n;
  uint32_t m[kTieWords], ns = 0;
#pragma unroll
  for (uint32_t e = 0; e < kTieWords; ++e) {
    m[e] = e < n ? q.ent[e * q.stride].x : 0u;
    ns += popc(m[e]);
  }
  auto below = [&](uint64_t b) -> uint32_t {
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(b >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)b, 0u));
  };
  // exclusive prefix sum over the wave's lanes and the wave's total of v < 8
  auto prefix = [&](uint32_t v, uint32_t& total) -> uint32_t {
    const uint64_t b0 = __ballot(v & 1u), b1 = __ballot(v & 2u), b2 = __ballot(v & 4u);
    total = (uint32_t)__popcll(b0) + 2u * (uint32_t)__popcll(b1) + 4u * (uint32_t)__popcll(b2);
    return below(b0) + 2u * below(b1) + 4u * below(b2);
  };
  uint32_t wtotal = 0, first = 0;
  const bool few = __ballot(ns >= 8u) == 0;  // every lane's count fits three bits
  if (few) first = prefix(ns, wtotal);
  if (lane == 0) wsum[wave] = few ? wtotal : kCap + 1u;
  __syncthreads();
  const uint32_t s0 = wsum[0], s1 = wsum[1], s2 = wsum[2], s3 = wsum[3];
  const uint32_t total = s0 + s1 + s2 + s3;  // above kCap if any wave could not number
  if (total == 0u) return;  // the same for every thread: no barrier follows
  if (total <= cap) {
    uint32_t k = first + (wave > 0 ? s0 : 0u) + (wave > 1 ? s1 : 0u) + (wave > 2 ? s2 : 0u);
#pragma unroll
    for (uint32_t e = 0; e < kTieWords; ++e) {
      uint32_t mm = m[e];
      while (mm) {
        const uint32_t b = __builtin_ctz(mm);
        mm &= mm - 1;
        idx[k++] = (uint16_t)(threadIdx.x | (e << 8) | (b << 10));
      }
    }
    __syncthreads();
    for (uint32_t r0 = 0; r0 < total; r0 += 256u) {
      const uint32_t i = r0 + threadIdx.x;
      if (i < total) {
        // the slot still holds the word's tie mask; only this thread changes bit b
        const uint32_t id = idx[i], b = id >> 10;
        uint4* slot = ent + ((id >> 8) & 3u) * q.stride + (id & 255u);
        const uint4 en = *slot;
        const Rand4 rr = philox(en.w * 32u + b, t, key.replica, tag(c, kIsingRefine), key.k0, key.k1);
        if (!((rr.w[0] & 0xFFFFFFu) < frac_sel(tab.fr, tie_class<true>(en, b))))
          atomicAnd(&slot->x, ~(1u << b));
      }
    }
    __syncthreads();
  } else {
    uint16_t* widx = idx + wave * 64u * kTieWords;
    uint4* went = ent + wave * 64u;
    uint32_t wt = 0;
    const uint32_t wfirst = prefix(n, wt);
    if (wt == 0u) return;  // the same for the wave's lanes; nothing else waits for them
#pragma unroll
    for (uint32_t e = 0; e < kTieWords; ++e)
      if (e < n) widx[wfirst + e] = (uint16_t)(lane | (e << 6));
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    for (uint32_t r0 = 0; r0 < wt; r0 += 64u) {
      const uint32_t i = r0 + lane;
      if (i < wt) {
        const uint32_t id = widx[i];
        uint4* slot = went + (id >> 6) * q.stride + (id & 63u);
        const uint4 en = *slot;
        uint32_t mm = en.x, flips = 0;
        while (mm) {
          const uint32_t b = __builtin_ctz(mm);
          mm &= mm - 1;
          const Rand4 rr = philox(en.w * 32u + b, t, key.replica, tag(c, kIsingRefine), key.k0, key.k1);
          if ((rr.w[0] & 0xFFFFFFu) < frac_sel(tab.fr, tie_class<true>(en, b))) flips |= 1u << b;
        }
        slot->x = flips;
      }
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  }
#pragma unroll
  for (uint32_t e = 0; e < kTieWords; ++e) {
    if (e < n) {
      const uint4 en = q.ent[e * q.stride];
      if (en.x) {  // the lane's own word, stored earlier by this lane
        const uint32_t word = own[en.w];
        own[en.w] = word ^ en.x;
        if (MEASURE) {  // counts, widened once at the end of the band
          q.tf += popc(en.x);
          q.tk0 += popc(en.x & en.y);
          q.tk1 += popc(en.x & en.z);
          q.tset += popc(en.x & word);  // a set bit is s = -1
        }
      }
    }
  }
  q.n = 0;
}

// The plain launches of a band height chosen for eight waves per SIMD ask the
// compiler for that occupancy (64 registers); the +-1-coupling 3D kernel would
// spill there and keeps the default.
// FAST: only the classes k < d can refuse a move (J0 > 0), decided by
// packed_decide_fast; otherwise packed_decide.  WAVE (with FAST): the
// end-of-band ties are resolved by the whole workgroup
// (packed_tie_flush_group).
// WM (with WAVE): kWaveBand when a plane row is a multiple of 64 words, so
// the 64 lanes of a wave share their band and the band's row arithmetic runs
// once per wave in scalar registers; kWaveParity when a row is fewer words
// that divide 64, the band height is even and a wave's bands lie in one
// z-plane, so the wave's rows still share their parity; kWaveFallback to
// resolve the ties by the workgroup resolution's fallback always (a test of
// that path).
constexpr int kWaveAny = 0, kWaveBand = 1, kWaveFallback = 2, kWaveParity = 3;
template <int D, bool PM, bool MEASURE, bool FAST, bool WAVE, int WM>
__global__ __launch_bounds__(256)
__attribute__((amdgpu_waves_per_eu((MEASURE || (D == 3 && PM)) ? 1 : 8))) void packed_stream_kernel(const Geom g, const RngKey key,
                                                            const IsingTable table,
                                                            const FastDiv divW, const FastDiv divL,
                                                            const uint32_t H, const uint32_t nbands,
                                                            uint32_t* __restrict__ s,
                                                            const uint32_t* __restrict__ J,
                                                            const uint32_t t, const uint32_t c,
                                                            Partial* __restrict__ parts) {
  constexpr bool UB = WM == kWaveBand;
  constexpr bool WP = UB || WM == kWaveParity;  // the wave's rows share their parity
  static_assert(!WAVE || FAST, "wave resolution: the fast decision's slot layout");
  static_assert(WM == kWaveAny || WAVE, "wave modes only with the workgroup's tie resolution");
  __shared__ uint4 tie_ent[kTieWords * 256];
  __shared__ uint8_t tie_rows[WAVE ? 1 : kTieWords * 256];
  __shared__ uint16_t tie_idx[WAVE ? kTieWords * 256 : 1];
  __shared__ uint32_t tie_sum[WAVE ? 4 : 1];
  const uint32_t tid = xcd_remap(blockIdx.x, gridDim.x) * 256u + threadIdx.x;
  const uint32_t band = fdiv(UB ? __builtin_amdgcn_readfirstlane(tid) : tid, divW);
  int64_t Esum = 0, Msum = 0;
  // measured launches: per-lane 32-bit counts (v_bcnt_u32_b32 adds its
  // popcount to an accumulator), widened once per band -- unsatisfied bonds
  // by weight 1, 2, 4 of the count planes, set spin bits, words measured
  uint32_t cn0 = 0, cn1 = 0, cn2 = 0, cset = 0, cwords = 0;
  const uint32_t W = divW.d;
  const uint32_t Wh = (uint32_t)(g.Nh / 32);  // words per plane
  uint32_t* own = s + (uint64_t)c * Wh;
  const TabRegs tab = tab_regs(table);
  FastTab ft;
  if (FAST) ft = fast_tab<D>(tab);
  PackedTies tq;
  tq.ent = tie_ent + threadIdx.x;
  tq.rows = tie_rows + (WAVE ? 0u : threadIdx.x);
  tq.stride = 256;
  tq.n = 0;
  tq.base = 0;
  tq.W = W;
  tq.dE = 0;
  tq.dM = 0;
  tq.tf = tq.tk0 = tq.tk1 = tq.tset = 0;
  if (band < nbands) {
    // the band's index arithmetic in 24-bit multiplies (full rate): every
    // factor is below 2^24 -- a plane has at most 2^24 rows (packed_supported)
    auto mul = [](uint32_t a, uint32_t b) -> uint32_t { return __umul24(a, b); };
    const uint32_t q = tid - mul(band, W);
    const uint32_t L = (uint32_t)g.L;
    const uint32_t r0 = mul(band, H);
    uint32_t z = 0, y0 = r0;
    if (D == 3) {
      z = fdiv(r0, divL);
      y0 = r0 - mul(z, L);
    }
    const uint32_t* oth = s + (uint64_t)(1 - c) * Wh;
    // word w of a plane at a 32-bit byte offset from the plane's (uniform)
    // base: the loads and stores take the scalar-base + 32-bit-offset form
    auto ldw = [](const uint32_t* base, uint32_t w) -> uint32_t {
      return *reinterpret_cast<const uint32_t*>(reinterpret_cast<const char*>(base) + (w << 2));
    };
    const uint32_t zrow = mul(L, z);
    const uint32_t qn = q + 1 == W ? 0u : q + 1, qp = q == 0 ? W - 1 : q - 1;
    auto rw = [&](uint32_t zr, uint32_t y) -> uint32_t {  // word index of (row, q); y < 2L
      return mul(zr + (y >= L ? y - L : y), W);
    };
    uint32_t zm_row = 0, zp_row = 0;
    if (D == 3) {
      zm_row = mul(L, z == 0 ? L - 1 : z - 1);
      zp_row = mul(L, z + 1 == L ? 0 : z + 1);
    }
    tq.base = rw(zrow, y0) + q;
    // J planes: J[mu][cc] at (2 mu + cc) * Wh
    const uint32_t pz = (c + z) & 1u;
    // a band stays inside its z-plane (H divides L): the rows' word offsets
    // step by W, and only the y + 1 neighbour of row L - 1 wraps (to row 0)
    const uint32_t row0 = rw(zrow, y0), wrap0 = mul(zrow, W);
    uint32_t up = ldw(oth, rw(zrow, y0 + L - 1) + q);
    uint32_t ct = ldw(oth, row0 + q);
    uint32_t rowb = row0;
    uint32_t zmb = mul(zm_row + y0, W), zpb = mul(zp_row + y0, W);  // z - 1 and z + 1 rows (3D)
    // one row of the band; pc is the row's parity p (1: the x+1 neighbour is
    // the next in-row site), a compile-time constant when the caller knows it
    auto row = [&](uint32_t i, auto pc) {
      const uint32_t y = y0 + i;
      const uint32_t p = pc;
      const uint32_t dn = ldw(oth, (y + 1 == L ? wrap0 : rowb + W) + q);
      const uint32_t o = ldw(own, rowb + q);
      // x+1 neighbours (p = 1: next in-row site) and x-1 (p = 0: previous)
      uint32_t nxp, nxm;
      if constexpr (!std::is_same<decltype(pc), uint32_t>::value) {
        // known parity: only the word on the side where the row leaves this one
        if constexpr (decltype(pc)::value == 1) {
          nxp = __builtin_amdgcn_alignbit(ldw(oth, rowb + qn), ct, 1u);
          nxm = ct;
        } else {
          nxp = ct;
          nxm = __builtin_amdgcn_alignbit(ct, ldw(oth, rowb + qp), 31u);
        }
      } else {
        const uint32_t en = ldw(oth, rowb + qn), ep = ldw(oth, rowb + qp);
        const uint32_t sh_next = __builtin_amdgcn_alignbit(en, ct, 1u);
        const uint32_t sh_prev = __builtin_amdgcn_alignbit(ct, ep, 31u);
        nxp = mask_sel(ct, sh_next, p);
        nxm = mask_sel(sh_prev, ct, p);
      }
      uint32_t u[6];
      u[0] = o ^ nxp;
      u[1] = o ^ nxm;
      u[2] = o ^ dn;
      u[3] = o ^ up;
      uint32_t fz = 0, bz = 0;
      if (D == 3) {
        fz = ldw(oth, zmb + q);
        bz = ldw(oth, zpb + q);
        u[4] = o ^ bz;
        u[5] = o ^ fz;
      }
      if (PM) {
        const uint32_t* Jo = J + (uint64_t)c * Wh;        // J[mu][c] = J + (2 mu + c) Wh
        const uint32_t* Jn = J + (uint64_t)(1 - c) * Wh;  // J[mu][1 - c]
        const uint32_t jc = ldw(Jn, rowb + q);
        const uint32_t jp_prev = ldw(Jn, rowb + qp);
        u[0] ^= ldw(Jo, rowb + q);
        u[1] ^= mask_sel(__builtin_amdgcn_alignbit(jc, jp_prev, 31u), jc, p);
        u[2] ^= ldw(Jo, 2 * Wh + rowb + q);
        u[3] ^= ldw(Jn, 2 * Wh + (y == 0 ? rw(zrow, L - 1) : rowb - W) + q);
        if (D == 3) {
          u[4] ^= ldw(Jo, 4 * Wh + rowb + q);
          u[5] ^= ldw(Jn, 4 * Wh + zmb + q);
        }
      }
      uint32_t k0, k1, k2;
      count_planes<D>(u, k0, k1, k2);
      uint32_t ties;
      const uint32_t flip = FAST ? packed_decide_fast<D>(ft, key, t, c, rowb + q, k0, k1, k2, ties)
                                 : packed_decide<D>(tab, key, t, c, rowb + q, k0, k1, k2, ties);
      const uint32_t on = o ^ flip;
      *reinterpret_cast<uint32_t*>(reinterpret_cast<char*>(own) + ((rowb + q) << 2)) = on;
      packed_queue_word<D, MEASURE, WAVE>(tq, ties, i, rowb + q, k0, k1, k2, tab, key, t, c, own);
      if (MEASURE) {
        // colour 1 after its update: each bond has one colour-1 end; the
        // colour-0 word at the same position covers each colour-0 site once
        const uint32_t fl = o ^ on;  // every bond of a flipped site changes state
        uint32_t v[6];
#pragma unroll
        for (int m = 0; m < 2 * D; ++m) v[m] = u[m] ^ fl;
        uint32_t n0, n1, n2;
        count_planes<D>(v, n0, n1, n2);
        cn0 += popc(n0);
        cn1 += popc(n1);
        cn2 += popc(n2);
        cset += popc(on) + popc(ct);
        ++cwords;
      }
      up = ct;
      ct = dn;
      rowb += W;
      zmb += W;
      zpb += W;
    };
    using P0 = std::integral_constant<uint32_t, 0>;
    using P1 = std::integral_constant<uint32_t, 1>;
    if (WP && (H & 1u) == 0u) {
      // the wave's rows share their parity, which alternates along the band
      // (the bands start at even rows of one z-plane)
      if (__builtin_amdgcn_readfirstlane((pz + y0) & 1u)) {
        for (uint32_t i = 0; i < H; i += 2) {
          row(i, P1());
          row(i + 1, P0());
        }
      } else {
        for (uint32_t i = 0; i < H; i += 2) {
          row(i, P0());
          row(i + 1, P1());
        }
      }
    } else {
      for (uint32_t i = 0; i < H; ++i) row(i, (pz + y0 + i) & 1u);
    }
  }
  if (WAVE)  // the band's queued ties, every thread of the workgroup
    packed_tie_flush_group<D, MEASURE>(tq, tab, key, t, c, own, tie_idx, tie_ent, tie_sum,
                                       WM == kWaveFallback ? 0u : kTieWords * 256u);
  else
    packed_tie_flush<D, MEASURE>(tq, tab, key, t, c, own);
  if (MEASURE) {
    // each measured word: 32 colour-1 sites with 2d bonds (E = -2d per site
    // plus 2 per unsatisfied bond) and the 32 + 32 sites of both colours' words
    // each flipped tied site with k unsatisfied bonds raises E by 4 (d - k)
    // and moves M by -2 s
    const int64_t tk = (int64_t)tq.tk0 + 2 * (int64_t)tq.tk1;
    Esum = -(int64_t)(64 * D) * cwords + 2 * ((int64_t)cn0 + 2 * (int64_t)cn1 + 4 * (int64_t)cn2) +
           tq.dE + 4 * ((int64_t)D * tq.tf - tk);
    Msum = (int64_t)64 * cwords - 2 * (int64_t)cset + tq.dM - 2 * ((int64_t)tq.tf - 2 * (int64_t)tq.tset);
    block_partial_int(Esum, Msum, parts, blockIdx.x);
  }
}

// Rows per band for the packed kernel: the largest power of two up to 64
// dividing L that leaves at least min_waves waves.
uint32_t packed_rows_per_band(const Geom& g, uint32_t min_waves) {
  const uint32_t W = (uint32_t)(g.R / 32);
  uint32_t best = 1;
  for (uint32_t H = 1; H <= 64; H *= 2) {
    if (g.L % H) break;
    const uint64_t waves = (uint64_t)W * (uint64_t)(g.rows / H) / 64;
    if (waves >= min_waves || H == 1) best = H;
  }
  return best;
}

bool packed_supported(const Geom& g, int J_kind) {
  // at most 2^24 rows per plane: the kernel's index products are 24-bit
  return (g.d == 2 || g.d == 3) && J_kind != 2 && g.L % 64 == 0 && g.rows <= ((int64_t)1 << 24);
}

hipError_t launch_packed_half_sweep(const IsingLaunch& a, uint32_t* spins, const uint32_t* J,
                                    uint32_t t, uint32_t c, void* partials, int64_t* nparts,
                                    hipStream_t st) {
  const uint32_t H = a.rows_per_band;
  const uint32_t W = (uint32_t)(a.g.R / 32);
  const uint32_t nbands = (uint32_t)a.g.rows / H;
  const uint64_t lanes = (uint64_t)nbands * W;
  const dim3 grid((unsigned)((lanes + 255) / 256)), block(256);
  const FastDiv dW = make_fastdiv(W), dL = make_fastdiv((uint32_t)a.g.L);
  const bool pm = a.J_kind == 1;
  // the fast decision when every class k >= d always accepts (J0 > 0)
  bool fast = true;
  for (int k = a.g.d; k <= 2 * a.g.d; ++k)
    if ((((k < 4 ? a.tab.al_lo : a.tab.al_hi) >> (8 * (k & 3))) & 0xFFu) != 0xFFu) fast = false;
  Partial* pp = (Partial*)partials;
  const bool wave = a.packed_ties != 1;
  const bool uniform_band = W % 64 == 0;  // every wave inside one band
  // a wave's 64 / W bands start at even rows of one z-plane
  const bool wave_parity = 64 % W == 0 && H % 2 == 0 &&
                           (a.g.d == 2 || (uint32_t)a.g.L % ((64 / W) * H) == 0);
#define SMC_PK(DD, PMM, MM, FF, WW, UU)                                                                     \
  hipLaunchKernelGGL((packed_stream_kernel<DD, PMM, MM, FF, WW, UU>), grid, block, 0, st, a.g, a.key, a.tab, \
                     dW, dL, H, nbands, spins, J, t, c, pp)
#define SMC_PKF(DD, PMM, MM)                                                   \
  do {                                                                         \
    if (!fast) SMC_PK(DD, PMM, MM, false, false, kWaveAny);                    \
    else if (!wave) SMC_PK(DD, PMM, MM, true, false, kWaveAny);                \
    else if (a.packed_ties == 2) SMC_PK(DD, PMM, MM, true, true, kWaveFallback); \
    else if (!uniform_band && wave_parity) SMC_PK(DD, PMM, MM, true, true, kWaveParity); \
    else if (!uniform_band) SMC_PK(DD, PMM, MM, true, true, kWaveAny);         \
    else SMC_PK(DD, PMM, MM, true, true, kWaveBand);                           \
  } while (0)
  if (a.g.d == 2) {
    if (pm) { if (pp) SMC_PKF(2, true, true); else SMC_PKF(2, true, false); }
    else { if (pp) SMC_PKF(2, false, true); else SMC_PKF(2, false, false); }
  } else {
    if (pm) { if (pp) SMC_PKF(3, true, true); else SMC_PKF(3, true, false); }
    else { if (pp) SMC_PKF(3, false, true); else SMC_PKF(3, false, false); }
  }
#undef SMC_PKF
#undef SMC_PK
  if (pp && nparts) *nparts = grid.x;
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Packing, initial states, and a standalone measurement.
// ---------------------------------------------------------------------------

__global__ __launch_bounds__(256) void pack_kernel(const int8_t* __restrict__ src,
                                                   uint32_t* __restrict__ dst, int64_t n_words) {
  const int64_t w = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (w >= n_words) return;
  const uint4* p = reinterpret_cast<const uint4*>(src + 32 * w);
  const uint4 a = p[0], b = p[1];
  const uint32_t v[8] = {a.x, a.y, a.z, a.w, b.x, b.y, b.z, b.w};
  uint32_t out = 0;
#pragma unroll
  for (int k = 0; k < 8; ++k) out |= gather7(v[k]) << (4 * k);  // -1 = 0xFF has bit 7 set
  dst[w] = out;
}

__global__ __launch_bounds__(256) void unpack_kernel(const uint32_t* __restrict__ src,
                                                     int8_t* __restrict__ dst, int64_t n_words) {
  const int64_t w = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (w >= n_words) return;
  const uint32_t v = src[w];
  uint32_t o[8];
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    // 4 bits -> bit 0 of 4 bytes; -1 = 0xFF, +1 = 0x01
    const uint32_t nib = (v >> (4 * k)) & 0xFu;
    const uint32_t ones = ((nib * 0x00204081u) & 0x01010101u);
    o[k] = kOnes | (ones * 0xFEu);
  }
  uint4* p = reinterpret_cast<uint4*>(dst + 32 * w);
  p[0] = make_uint4(o[0], o[1], o[2], o[3]);
  p[1] = make_uint4(o[4], o[5], o[6], o[7]);
}

hipError_t launch_pack(const int8_t* src, uint32_t* dst, int64_t n_words, hipStream_t st) {
  if (n_words <= 0) return hipSuccess;
  hipLaunchKernelGGL(pack_kernel, dim3((unsigned)((n_words + 255) / 256)), dim3(256), 0, st, src,
                     dst, n_words);
  return hipGetLastError();
}

hipError_t launch_unpack(const uint32_t* src, int8_t* dst, int64_t n_words, hipStream_t st) {
  if (n_words <= 0) return hipSuccess;
  hipLaunchKernelGGL(unpack_kernel, dim3((unsigned)((n_words + 255) / 256)), dim3(256), 0, st,
                     src, dst, n_words);
  return hipGetLastError();
}

// Hot/cold start (mode 0 / 1) or +-1 couplings (mode 2) of the packed planes,
// with the draws of the int8 initialisation (keyed by natural site index).
__global__ __launch_bounds__(256) void init_packed_kernel(const Geom g, const RngKey key,
                                                          const int mode,
                                                          uint32_t* __restrict__ out) {
  const int64_t wid = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int64_t Wh = g.Nh / 32;
  const int64_t planes = mode == 2 ? 2 * (int64_t)g.d : 2;
  if (wid >= planes * Wh) return;
  const int64_t pl = wid / Wh;
  const uint32_t c = (uint32_t)(pl & 1);
  const uint32_t mu = (uint32_t)(pl >> 1);
  const int64_t j0 = (wid - pl * Wh) * 32;
  uint32_t word = 0;
  if (mode != 1) {
    const uint32_t purpose = mode == 2 ? kCoupling : kInitSpin;
    const uint32_t w1 = mode == 2 ? mu : 0u;
    for (int b = 0; b < 32; ++b) {
      int32_t x, y, z;
      site_coords(g, c, j0 + b, x, y, z);
      const int64_t i = natural_index(g, x, y, z);
      const Rand4 r = philox((uint32_t)(i >> 7), w1, key.replica, tag(0, purpose), key.k0, key.k1);
      const uint32_t sel = (uint32_t)(i >> 5) & 3u;
      const uint32_t wv = sel == 0 ? r.w[0] : (sel == 1 ? r.w[1] : (sel == 2 ? r.w[2] : r.w[3]));
      word |= ((wv >> (i & 31)) & 1u) << b;
    }
  }
  out[wid] = word;
}

hipError_t launch_init_packed(const Geom& g, RngKey key, int mode, uint32_t* out, hipStream_t st) {
  const int64_t n = (mode == 2 ? 2 * (int64_t)g.d : 2) * (g.Nh / 32);
  hipLaunchKernelGGL(init_packed_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, g,
                     key, mode, out);
  return hipGetLastError();
}

// E and M of a packed state: one lane per colour-1 word (each bond has one
// colour-1 end), plus the colour-0 word at the same position.
template <int D, bool PM>
__global__ __launch_bounds__(256) void measure_packed_kernel(const Geom g,
                                                             const uint32_t* __restrict__ s,
                                                             const uint32_t* __restrict__ J,
                                                             Partial* __restrict__ parts) {
  const int64_t Wh = g.Nh / 32;
  const int64_t wid = (int64_t)blockIdx.x * 256 + threadIdx.x;
  int64_t E = 0, M = 0;
  if (wid < Wh) {
    const uint32_t W = (uint32_t)(g.R / 32);
    const uint32_t L = (uint32_t)g.L;
    const uint32_t r = (uint32_t)(wid / W), q = (uint32_t)(wid - (int64_t)r * W);
    const uint32_t y = r % L, z = r / L;
    const uint32_t p = (1u + y + z) & 1u;
    const uint32_t* s1 = s + Wh;
    const uint32_t* s0 = s;
    auto at = [&](uint32_t yy, uint32_t zz, uint32_t qq) -> int64_t {
      return ((int64_t)zz * L + yy) * W + qq;
    };
    const uint32_t qn = q + 1 == W ? 0u : q + 1, qp = q == 0 ? W - 1 : q - 1;
    const uint32_t ym = y == 0 ? L - 1 : y - 1, yp = y + 1 == L ? 0 : y + 1;
    const uint32_t o = s1[wid];
    const uint32_t ct = s0[wid];
    const uint32_t sn = __builtin_amdgcn_alignbit(s0[at(y, z, qn)], ct, 1u);
    const uint32_t sp = __builtin_amdgcn_alignbit(ct, s0[at(y, z, qp)], 31u);
    uint32_t u[6];
    u[0] = o ^ (p ? sn : ct);
    u[1] = o ^ (p ? ct : sp);
    u[2] = o ^ s0[at(yp, z, q)];
    u[3] = o ^ s0[at(ym, z, q)];
    uint32_t zm = 0, zp = 0;
    if (D == 3) {
      zm = z == 0 ? L - 1 : z - 1;
      zp = z + 1 == L ? 0 : z + 1;
      u[4] = o ^ s0[at(y, zp, q)];
      u[5] = o ^ s0[at(y, zm, q)];
    }
    if (PM) {
      const uint32_t* J1 = J + Wh;  // J[mu][1] = J + (2 mu + 1) Wh
      const uint32_t* J0 = J;       // J[mu][0]
      const uint32_t jc = J0[wid];
      u[0] ^= J1[wid];
      u[1] ^= p ? jc : __builtin_amdgcn_alignbit(jc, J0[at(y, z, qp)], 31u);
      u[2] ^= J1[2 * Wh + wid];
      u[3] ^= J0[2 * Wh + at(ym, z, q)];
      if (D == 3) {
        u[4] ^= J1[4 * Wh + wid];
        u[5] ^= J0[4 * Wh + at(y, zm, q)];
      }
    }
    uint32_t k0, k1, k2;
    count_planes<D>(u, k0, k1, k2);
    E = -(int64_t)(32 * 2 * D) + 2 * (int64_t)(popc(k0) + 2 * popc(k1) + 4 * popc(k2));
    M = (32 - 2 * popc(o)) + (32 - 2 * popc(ct));
  }
  block_partial_int(E, M, parts, blockIdx.x);
}

hipError_t launch_measure_packed(const Geom& g, int J_kind, const uint32_t* s, const uint32_t* J,
                                 void* partials, int64_t* nparts, hipStream_t st) {
  const int64_t Wh = g.Nh / 32;
  const dim3 grid((unsigned)((Wh + 255) / 256)), block(256);
  Partial* pp = (Partial*)partials;
  if (g.d == 2) {
    if (J_kind == 1) hipLaunchKernelGGL((measure_packed_kernel<2, true>), grid, block, 0, st, g, s, J, pp);
    else hipLaunchKernelGGL((measure_packed_kernel<2, false>), grid, block, 0, st, g, s, J, pp);
  } else {
    if (J_kind == 1) hipLaunchKernelGGL((measure_packed_kernel<3, true>), grid, block, 0, st, g, s, J, pp);
    else hipLaunchKernelGGL((measure_packed_kernel<3, false>), grid, block, 0, st, g, s, J, pp);
  }
  *nparts = grid.x;
  return hipGetLastError();
}

}  // namespace smc
