// batch.hip -- many independent Ising lattices of uneven size, temperature and
// disorder realisation in one persistent launch (the paper's trivial
// parallelism over disorder realisations on top of the checkerboard
// decomposition, Sec. 2).
//
// One workgroup owns one lattice: it stages both colour planes (L^d bytes,
// at most 64 KiB) in LDS, runs every sweep of the call there -- colour 0,
// barrier, colour 1, barrier -- and writes the planes back once, so HBM is
// touched only at the start and the end.  Couplings stay in global memory
// (they are re-read from L2 / Infinity Cache).  Lattice r uses replica r in
// the Philox counter, so each lattice reproduces the single-lattice chain
// with that replica bit for bit.  A lane walks groups of 16 consecutive
// same-colour sites (one Philox block of prefix bytes per group); the
// decision per site is the integer threshold test of the single-lattice
// kernels with its exact tie refinement.  Lattices whose plane rows are whole
// 4-site words (L/2 % 4 == 0) take the decision four sites per 32-bit op
// (rows of whole 2-site pairs, L/2 even, two sites per op):
// neighbour words from LDS (the in-row neighbours as the centre word shifted
// by one byte), unsatisfied-bond counts per byte, and the byte-wise threshold
// compare of the single-lattice kernels.  The index arithmetic of a word
// (its row, the periodic wraps of its neighbours) is formed once per call when
// each lane holds one group, and once per group when a group is a whole part
// of one plane row (L/2 % 16 == 0).  With MEASURE the workgroup also
// reduces E and M of its state from LDS after every `every` sweeps (record m
// of the call at obs[m * n_lattices + lattice]; with no sweeps, one record of
// the current state).
#include <type_traits>

#include "chunk.hpp"
#include "packed.hpp"
#include "reduce.hpp"

namespace smc {

constexpr uint32_t kBatchTieSlots = 4;  // deferred ties per lane before a flush

// ---------------------------------------------------------------------------
// Packed path (3D lattices with L % 4 == 0, L <= 40, at most two 32-site
// words of a colour per lane): the lattice sits in LDS at one bit per site --
// word w of colour c holds sites 32 w .. 32 w + 31 of that plane, the two
// colours' words side by side (byte 12 (w + 1) + 4 c, a zero pad pair at each
// end) -- with the signs of each site's 2d bonds as six words aligned with it
// (the -mu bonds gathered from the neighbours' planes when the lattice is
// staged; 52 bytes per word).  A lane owns words w = lane and w = lane + blockDim of both
// colours for the whole call.  The neighbour words of the other colour come
// from funnel shifts of LDS words: in-row x +- 1 (with the wrap at row ends
// and the row parity as per-word masks), y +- 1 (a shift by R = L / 2 sites,
// with the rows at y = L - 1 or 0 taking the wrapped source), and z +- 1 (a
// shift by L^2 / 2 sites: a whole word when L % 8 == 0, otherwise a funnel
// shift with the planes at z = L - 1 or 0 taking the wrapped source).
// Counts, the decision with
// its prefix bit planes and exact ties, and the random bytes per site are
// those of the packed single-lattice kernel, so every lattice keeps the
// chain of its replica bit for bit.
// ---------------------------------------------------------------------------
constexpr uint32_t kPackedBatchWordsPerLane = 2;
// LDS strides of a word's spin pair (colour 0, colour 1, unused) and of its
// twelve bond-sign words (+ one unused): an odd number of dwords, so that 32
// lanes reading consecutive words touch 32 different banks.
constexpr uint32_t kPkSpin = 12, kPkBond = 52;

__host__ __device__ inline bool batch_packed_ok(int d, uint32_t L, uint32_t threads) {
  if (d != 3 || L % 4u != 0u || L > 40u) return false;
  const uint32_t Wp = L * L * L / 64u;  // words per colour
  return Wp <= kPackedBatchWordsPerLane * threads;
}

// LDS bytes of the packed path for edge L: the spin pairs with their pads and
// the aligned bond-sign words (+-1 couplings).  (A lane's tied words -- at
// most one per word it owns -- wait in registers until the end of the
// half-sweep.)
__host__ __device__ inline size_t batch_packed_lds_bytes(uint32_t L, bool pm, uint32_t threads) {
  const size_t Wp = (size_t)L * L * L / 64;
  const size_t sb = (kPkSpin * (Wp + 2) + 15) / 16 * 16;
  const size_t jb = pm ? (kPkBond * Wp + 15) / 16 * 16 : 0;
  (void)threads;
  return sb + jb;
}

struct PackedWord {  // per-call constants of one word of the lane
  uint32_t E, S, Pm0, Ymp, Ymm;  // row end / start, rows of colour-0 parity 1, y = L-1 / y = 0
  uint32_t Zmp, Zmm;             // sites at z = L-1 / z = 0 (used when z-planes split words)
  uint32_t ayp, aym;             // LDS byte addresses (colour 0) of the y wrap sources
  uint32_t azp, azm;             // z +- 1 sources (low words of the funnels)
  uint32_t azpw, azmw;           // z wrap sources (z-planes that split words)
  uint32_t a0;                   // LDS byte address of word w, colour 0
  uint32_t aj;                   // LDS byte address of its bond-sign words
  bool valid;
};

// Funnel shifts of the wrap and z gathers (site offset mod 32).  LR = L^2/2
// sites per z-plane of one colour; when LR % 32 == 0 the z neighbours are
// whole words (zs == 0).
struct PackedZ {
  uint32_t ysw, ysmw;     // y wraps: R - LR, LR - R
  uint32_t zs, zsw;       // +z: LR, LR (1 - L)
  uint32_t zsm, zsmw;     // -z: -LR, LR (L - 1)
};

// Neighbour words (+x, -x, +y, -y, +z, -z) of word `pw` of colour C from the
// other colour's words.
template <uint32_t C>
__device__ __forceinline__ void packed_neighbours(const unsigned char* lds, const PackedWord& pw,
                                                  uint32_t R, const PackedZ& pz, uint32_t nb[6]) {
  constexpr uint32_t O = 4u * (1u - C);  // the other colour's word in a pair
  auto ldw = [&](uint32_t a) -> uint32_t { return *reinterpret_cast<const uint32_t*>(lds + a); };
  const uint32_t wp = ldw(pw.a0 - kPkSpin + O), wc = ldw(pw.a0 + O), wn = ldw(pw.a0 + kPkSpin + O);
  const uint32_t next = __builtin_amdgcn_alignbit(wn, wc, 1u);        // site + 1
  const uint32_t prev = __builtin_amdgcn_alignbit(wc, wp, 31u);       // site - 1
  const uint32_t wst = __builtin_amdgcn_alignbit(wc, wp, 33u - R);    // site - (R - 1): row start
  const uint32_t wen = __builtin_amdgcn_alignbit(wn, wc, R - 1u);     // site + (R - 1): row end
  // row parity of colour C: p = 1 rows take x + 1 = in-row index + 1
  const uint32_t Pm = C == 0 ? pw.Pm0 : ~pw.Pm0;
  nb[0] = __builtin_amdgcn_bitop3_b32(Pm, __builtin_amdgcn_bitop3_b32(pw.E, wst, next, 0xCA), wc, 0xCA);
  nb[1] = __builtin_amdgcn_bitop3_b32(Pm, wc, __builtin_amdgcn_bitop3_b32(pw.S, wen, prev, 0xCA), 0xCA);
  const uint32_t yp = __builtin_amdgcn_alignbit(wn, wc, R);
  const uint32_t ypw = __builtin_amdgcn_alignbit(ldw(pw.ayp + kPkSpin + O), ldw(pw.ayp + O), pz.ysw);
  nb[2] = __builtin_amdgcn_bitop3_b32(pw.Ymp, ypw, yp, 0xCA);
  const uint32_t ym = __builtin_amdgcn_alignbit(wc, wp, 32u - R);
  const uint32_t ymw = __builtin_amdgcn_alignbit(ldw(pw.aym + kPkSpin + O), ldw(pw.aym + O), pz.ysmw);
  nb[3] = __builtin_amdgcn_bitop3_b32(pw.Ymm, ymw, ym, 0xCA);
  if (pz.zs == 0u) {  // z-planes hold whole words
    nb[4] = ldw(pw.azp + O);
    nb[5] = ldw(pw.azm + O);
  } else {
    const uint32_t zp = __builtin_amdgcn_alignbit(ldw(pw.azp + kPkSpin + O), ldw(pw.azp + O), pz.zs);
    const uint32_t zpw = __builtin_amdgcn_alignbit(ldw(pw.azpw + kPkSpin + O), ldw(pw.azpw + O), pz.zsw);
    nb[4] = __builtin_amdgcn_bitop3_b32(pw.Zmp, zpw, zp, 0xCA);
    const uint32_t zm = __builtin_amdgcn_alignbit(ldw(pw.azm + kPkSpin + O), ldw(pw.azm + O), pz.zsm);
    const uint32_t zmw = __builtin_amdgcn_alignbit(ldw(pw.azmw + kPkSpin + O), ldw(pw.azmw + O), pz.zsmw);
    nb[5] = __builtin_amdgcn_bitop3_b32(pw.Zmm, zmw, zm, 0xCA);
  }
}

// Count planes of word `pw` of colour C: unsatisfied bonds (spin bits differ,
// xor the bond's sign bit).
template <uint32_t C, bool PM>
__device__ __forceinline__ uint32_t packed_word_counts(const unsigned char* lds, const PackedWord& pw,
                                                       uint32_t R, const PackedZ& pz, uint32_t& k0,
                                                       uint32_t& k1, uint32_t& k2) {
  const uint32_t o = *reinterpret_cast<const uint32_t*>(lds + pw.a0 + 4u * C);
  uint32_t nb[6];
  packed_neighbours<C>(lds, pw, R, pz, nb);
  uint32_t u[6];
#pragma unroll
  for (int m = 0; m < 6; ++m) {
    const uint32_t js = PM ? *reinterpret_cast<const uint32_t*>(lds + pw.aj + 4u * (2u * m + C)) : 0u;
    u[m] = o ^ nb[m] ^ js;
  }
  count_planes<3>(u, k0, k1, k2);
  return o;
}

template <bool PM, bool MEASURE>
__device__ void batch_packed_lattice(unsigned char* lds, const BatchDesc* dp, uint32_t li,
                                     const RngKey& key0, int8_t* gs, const int8_t* gJ,
                                     uint32_t L, uint32_t R, uint32_t Nh, uint32_t replica,
                                     const TabRegs& tab, uint32_t t0, uint32_t n_sweeps,
                                     uint32_t every, uint32_t n_lattices, ObsOut* obs) {
  constexpr int D = 3;
  const uint32_t T = blockDim.x, q = threadIdx.x;
  const uint32_t Wp = Nh / 32u;
  const uint32_t LR = L * R;  // sites of a z-plane of one colour (a multiple of 32)
  const uint32_t SB = 0, JB = (kPkSpin * (Wp + 2u) + 15u) / 16u * 16u;
  const RngKey key{key0.k0, key0.k1, replica};

  // stage the spins: sign bits of 32 int8 sites per word, zero pad words
  for (uint32_t i = q; i < 2u * Wp; i += T) {
    const uint32_t c = i & 1u, w = i >> 1;
    const uint32_t* src = reinterpret_cast<const uint32_t*>(gs + (size_t)c * Nh + 32u * w);
    uint32_t v = 0;
#pragma unroll
    for (int k = 0; k < 8; ++k) v |= gather7(src[k]) << (4 * k);
    *reinterpret_cast<uint32_t*>(lds + SB + kPkSpin * (w + 1u) + 4u * c) = v;
  }
  if (q < 2u) {
    *reinterpret_cast<uint32_t*>(lds + SB + 4u * q) = 0u;
    *reinterpret_cast<uint32_t*>(lds + SB + kPkSpin * (Wp + 1u) + 4u * q) = 0u;
  }
  // in-plane index of the -mu neighbour of site (c, j)
  const uint32_t sYw = (L - 1) * R, sZ = L * R, sZw = (L - 1) * L * R;
  auto minus_nb = [&](uint32_t c, uint32_t j, int mu) -> uint32_t {
    const uint32_t r = j / R, rowb = r * R, jx = j - rowb;
    const uint32_t z = r / L, y = r - z * L;
    const uint32_t p = (c + y + z) & 1u;
    if (mu == 0) return jx + p == 0 ? rowb + R - 1 : j + p - 1;
    if (mu == 1) return y == 0 ? j + sYw : j - R;
    return z == 0 ? j + sZw : j - sZ;
  };
  if (PM) {
    for (uint32_t i = q; i < 2u * Wp; i += T) {
      const uint32_t c = i & 1u, w = i >> 1;
#pragma unroll
      for (int mu = 0; mu < 3; ++mu) {
        // +mu bond of the site itself: J[mu][c][j]
        const uint32_t* src = reinterpret_cast<const uint32_t*>(gJ + (size_t)(2 * mu + c) * Nh + 32u * w);
        uint32_t vp = 0;
#pragma unroll
        for (int k = 0; k < 8; ++k) vp |= gather7(src[k]) << (4 * k);
        // -mu bond: the +mu bond of the -mu neighbour, J[mu][1 - c][nb]
        const int8_t* Jn = gJ + (size_t)(2 * mu + 1 - c) * Nh;
        uint32_t vm = 0;
#pragma unroll 1  // set-up only: unrolled, it raised the kernel's registers into spills
        for (uint32_t b = 0; b < 32u; ++b)
          vm |= (Jn[minus_nb(c, 32u * w + b, mu)] < 0 ? 1u : 0u) << b;
        *reinterpret_cast<uint32_t*>(lds + JB + kPkBond * w + 4u * (2u * (2u * mu) + c)) = vp;
        *reinterpret_cast<uint32_t*>(lds + JB + kPkBond * w + 4u * (2u * (2u * mu + 1u) + c)) = vm;
      }
    }
  }
  // funnel shifts of the wrap and z gathers
  PackedZ pz;
  pz.ysw = (R - LR) & 31u;
  pz.ysmw = (LR - R) & 31u;
  pz.zs = LR & 31u;
  pz.zsw = (uint32_t)((int32_t)LR * (1 - (int32_t)L)) & 31u;
  pz.zsm = (0u - LR) & 31u;
  pz.zsmw = (LR * (L - 1u)) & 31u;
  // the lane's words: row masks, wrap and z sources
  PackedWord pw[kPackedBatchWordsPerLane];
#pragma unroll
  for (uint32_t p = 0; p < kPackedBatchWordsPerLane; ++p) {
    const uint32_t w = q + p * T;
    PackedWord& x = pw[p];
    x.valid = w < Wp;
    const uint32_t wv = x.valid ? w : 0u;
    x.E = x.S = x.Pm0 = x.Ymp = x.Ymm = x.Zmp = x.Zmm = 0;
#pragma unroll 1  // as above
    for (uint32_t b = 0; b < 32u; ++b) {
      const uint32_t j = 32u * wv + b;
      const uint32_t r = j / R, jx = j - r * R;
      const uint32_t z = r / L, y = r - z * L;
      x.E |= (jx == R - 1 ? 1u : 0u) << b;
      x.S |= (jx == 0 ? 1u : 0u) << b;
      x.Pm0 |= ((y + z) & 1u) << b;
      x.Ymp |= (y == L - 1 ? 1u : 0u) << b;
      x.Ymm |= (y == 0 ? 1u : 0u) << b;
      x.Zmp |= (z == L - 1 ? 1u : 0u) << b;
      x.Zmm |= (z == 0 ? 1u : 0u) << b;
    }
    // Wrap and z sources: bit i of a gather at site offset off is site
    // 32 w + i + off, from the funnel of words w + floor(off / 32) and the
    // next; that low word is clamped to the pads (-1 .. Wp - 1) where the
    // word has no site that uses the gather.  y wraps: rows y = L - 1 take
    // off = R - LR, rows y = 0 off = LR - R; z (when z-planes split words):
    // +-LR, and the wrapped LR (1 - L) / LR (L - 1) for the last / first
    // z-plane.
    auto lo = [&](int32_t off) -> uint32_t {  // LDS byte address of the clamped low word
      const int32_t i = (int32_t)wv + (off >> 5);
      return SB + kPkSpin * (uint32_t)((i < -1 ? -1 : (i > (int32_t)Wp - 1 ? (int32_t)Wp - 1 : i)) + 1);
    };
    const int32_t lr = (int32_t)LR, l = (int32_t)L, rr = (int32_t)R;
    x.ayp = lo(rr - lr);
    x.aym = lo(lr - rr);
    if (pz.zs == 0u) {  // z-planes hold whole words: the z neighbours are words
      const uint32_t zw = LR / 32u;  // words per z-plane
      const uint32_t izp = wv + zw >= Wp ? wv + zw - Wp : wv + zw;
      const uint32_t izm = wv < zw ? wv + Wp - zw : wv - zw;
      x.azp = SB + kPkSpin * (izp + 1u);
      x.azm = SB + kPkSpin * (izm + 1u);
      x.azpw = x.azmw = SB;
    } else {
      x.azp = lo(lr);
      x.azpw = lo(lr * (1 - l));
      x.azm = lo(-lr);
      x.azmw = lo(lr * (l - 1));
    }
    x.a0 = SB + kPkSpin * (wv + 1u);
    x.aj = JB + kPkBond * wv;
  }
  // thresholds of this lattice: the fast decision when only classes k < d can
  // refuse (every class k >= d always accepts)
  bool fast = true;
#pragma unroll
  for (int k = D; k <= 2 * D; ++k) fast = fast && table_byte(tab.al_lo, tab.al_hi, k) == 0xFFu;
  FastTab ft = fast_tab<D>(tab);
  __syncthreads();

  // a word's exact ties wait in registers (tie mask and count planes) until
  // the lane's words of the colour are stored, then take their refinement
  // draws; a lane writes only its own words, so the fix-up is race-free
  auto resolve = [&](uint32_t c, uint32_t t, uint32_t w, uint32_t a, const uint4& en) {
    uint32_t m = en.x, flips = 0;
    while (m) {
      const uint32_t b = __builtin_ctz(m);
      m &= m - 1;
      const uint32_t k = ((en.y >> b) & 1u) | (((en.z >> b) & 1u) << 1) | (((en.w >> b) & 1u) << 2);
      const Rand4 rr = philox(32u * w + b, t, replica, tag(c, kIsingRefine), key.k0, key.k1);
      if ((rr.w[0] & 0xFFFFFFu) < frac_sel(tab.fr, k)) flips |= 1u << b;
    }
    *reinterpret_cast<uint32_t*>(lds + a + 4u * c) ^= flips;
  };
  auto half = [&](auto cc, uint32_t t) {
    constexpr uint32_t C = decltype(cc)::value;
    uint4 tie[kPackedBatchWordsPerLane];
#pragma unroll
    for (uint32_t p = 0; p < kPackedBatchWordsPerLane; ++p) {
      tie[p] = make_uint4(0u, 0u, 0u, 0u);
      if (!pw[p].valid) continue;
      uint32_t k0, k1, k2;
      const uint32_t o = packed_word_counts<C, PM>(lds, pw[p], R, pz, k0, k1, k2);
      const uint32_t w = q + p * T;
      uint32_t ties;
      const uint32_t flip = fast ? packed_decide_fast<D>(ft, key, t, C, w, k0, k1, k2, ties)
                                 : packed_decide<D>(tab, key, t, C, w, k0, k1, k2, ties);
      *reinterpret_cast<uint32_t*>(lds + pw[p].a0 + 4u * C) = o ^ flip;
      tie[p] = make_uint4(ties, k0, k1, k2);
    }
#pragma unroll
    for (uint32_t p = 0; p < kPackedBatchWordsPerLane; ++p)
      if (tie[p].x) resolve(C, t, q + p * T, pw[p].a0, tie[p]);
    __syncthreads();
  };
  auto measure = [&](uint32_t slot, int64_t sweep) {
    int64_t Esum = 0, Msum = 0;
#pragma unroll
    for (uint32_t p = 0; p < kPackedBatchWordsPerLane; ++p) {
      if (!pw[p].valid) continue;
      uint32_t k0, k1, k2;
      const uint32_t o1 = packed_word_counts<1, PM>(lds, pw[p], R, pz, k0, k1, k2);
      const uint32_t o0 = *reinterpret_cast<const uint32_t*>(lds + pw[p].a0);
      const int32_t ks = __builtin_popcount(k0) + 2 * __builtin_popcount(k1) + 4 * __builtin_popcount(k2);
      Esum += 2 * (int64_t)ks - 32 * 2 * D;
      Msum += 64 - 2 * (int64_t)(__builtin_popcount(o1) + __builtin_popcount(o0));
    }
    __shared__ Partial part[1];
    block_partial_int(Esum, Msum, part, 0);
    if (q == 0) {
      ObsOut o;
      o.E_int = part[0].Ei;
      o.M_int = part[0].Mi;
      o.E = (double)part[0].Ei * dp->J0;
      o.M[0] = (double)part[0].Mi;
      o.M[1] = 0.0;
      o.M[2] = 0.0;
      o.absM = fabs((double)part[0].Mi);
      o.sweep = sweep;
      obs[(uint64_t)slot * n_lattices + li] = o;
    }
  };
  for (uint32_t sw = 0; sw < n_sweeps; ++sw) {
    const uint32_t t = t0 + sw;
    half(std::integral_constant<uint32_t, 0>(), t);
    half(std::integral_constant<uint32_t, 1>(), t);
    if (MEASURE && (sw + 1) % every == 0) measure((sw + 1) / every - 1, (int64_t)t + 1);
  }
  if (MEASURE && n_sweeps == 0) measure(0, (int64_t)t0);
  __syncthreads();
  // write both planes back as +-1 bytes
  for (uint32_t i = q; i < 2u * Wp; i += T) {
    const uint32_t c = i & 1u, w = i >> 1;
    const uint32_t v = *reinterpret_cast<const uint32_t*>(lds + SB + kPkSpin * (w + 1u) + 4u * c);
    uint32_t* dst = reinterpret_cast<uint32_t*>(gs + (size_t)c * Nh + 32u * w);
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      const uint32_t spread = (((v >> (4 * k)) & 0xFu) * 0x00204081u) & kOnes;
      dst[k] = kOnes | (spread * 0xFEu);
    }
  }
}


template <int D, bool PM, bool MEASURE>
__global__ __launch_bounds__(1024) void batch_kernel(const BatchDesc* __restrict__ descs,
                                                    const uint32_t* __restrict__ order,
                                                    const RngKey key, int8_t* __restrict__ spins,
                                                    const int8_t* __restrict__ J,
                                                    const uint32_t t0, const uint32_t n_sweeps,
                                                    const uint32_t every, const uint32_t n_lattices,
                                                    ObsOut* __restrict__ obs) {
  extern __shared__ uint32_t lat_words[];  // [2][Nh] spins of this lattice
  int8_t* const lat = reinterpret_cast<int8_t*>(lat_words);
  const uint32_t li = __builtin_amdgcn_readfirstlane(order[blockIdx.x]);
  const BatchDesc* dp = descs + li;
  const uint32_t L = __builtin_amdgcn_readfirstlane(dp->L);
  const uint32_t R = __builtin_amdgcn_readfirstlane(dp->R);
  const uint32_t Nh = __builtin_amdgcn_readfirstlane(dp->Nh);
  FastDiv divR, divL;
  divR.d = R;
  divR.m = (uint32_t)__builtin_amdgcn_readfirstlane(dp->divR_m);
  divR.s = (uint32_t)__builtin_amdgcn_readfirstlane(dp->divR_s);
  divL.d = L;
  divL.m = (uint32_t)__builtin_amdgcn_readfirstlane(dp->divL_m);
  divL.s = (uint32_t)__builtin_amdgcn_readfirstlane(dp->divL_s);
  const uint32_t th_lo = __builtin_amdgcn_readfirstlane(dp->th_lo);
  const uint32_t th_hi = __builtin_amdgcn_readfirstlane(dp->th_hi);
  const uint32_t al_lo = __builtin_amdgcn_readfirstlane(dp->al_lo);
  const uint32_t al_hi = __builtin_amdgcn_readfirstlane(dp->al_hi);
  const uint32_t replica = __builtin_amdgcn_readfirstlane(dp->replica);
  const uint64_t soff = ((uint64_t)__builtin_amdgcn_readfirstlane(dp->spin_off_hi) << 32) |
                        __builtin_amdgcn_readfirstlane(dp->spin_off_lo);
  const uint64_t joff = ((uint64_t)__builtin_amdgcn_readfirstlane(dp->J_off_hi) << 32) |
                        __builtin_amdgcn_readfirstlane(dp->J_off_lo);
  int8_t* gs = spins + soff;
  const int8_t* gJ = J + joff;
  const uint32_t N = 2 * Nh;  // L^d, a multiple of 4 (L even)
  if constexpr (D == 3) {
    if (__builtin_amdgcn_readfirstlane(dp->packed) && batch_packed_ok(D, L, blockDim.x)) {
      TabRegs tab;
      tab.th_lo = th_lo;
      tab.th_hi = th_hi;
      tab.al_lo = al_lo;
      tab.al_hi = al_hi;
      tab.fr.f0 = __builtin_amdgcn_readfirstlane(dp->frac[0]);
      tab.fr.f1 = __builtin_amdgcn_readfirstlane(dp->frac[1]);
      tab.fr.f2 = __builtin_amdgcn_readfirstlane(dp->frac[2]);
      tab.fr.f3 = __builtin_amdgcn_readfirstlane(dp->frac[3]);
      tab.fr.f4 = __builtin_amdgcn_readfirstlane(dp->frac[4]);
      tab.fr.f5 = __builtin_amdgcn_readfirstlane(dp->frac[5]);
      tab.fr.f6 = __builtin_amdgcn_readfirstlane(dp->frac[6]);
      batch_packed_lattice<PM, MEASURE>(reinterpret_cast<unsigned char*>(lat_words), dp, li, key, gs,
                                        gJ, L, R, Nh, replica, tab, t0, n_sweeps, every,
                                        n_lattices, obs);
      return;
    }
  }

  // Stage both planes into LDS as one byte per site: bit 0 = spin -1, bit
  // 1 + m = coupling of bond m negative (m = +x, -x, +y, -y, +z, -z), so the
  // sweep reads couplings from LDS together with the spins.
  // Row and plane strides (wave-uniform): neighbour rows are the own row's
  // offset plus or minus a stride, with the periodic wrap as a select.
  const uint32_t sYw = (L - 1) * R, sZ = L * R, sZw = (L - 1) * L * R;
  auto nbr = [&](uint32_t c, uint32_t j, uint32_t nbi[6]) {  // in-plane neighbour indices
    const uint32_t r = fdiv(j, divR);
    const uint32_t rowb = r * R;
    const uint32_t jx = j - rowb;
    const uint32_t z = D == 3 ? fdiv(r, divL) : 0u;
    const uint32_t y = r - z * L;
    const uint32_t p = (c + r + z) & 1u;  // (c + y + z) & 1 with L even
    nbi[0] = jx + p == R ? rowb : j + p;
    nbi[1] = jx + p == 0 ? rowb + R - 1 : j + p - 1;
    nbi[2] = y + 1 == L ? j - sYw : j + R;
    nbi[3] = y == 0 ? j + sYw : j - R;
    nbi[4] = nbi[5] = 0;
    if (D == 3) {
      nbi[4] = z + 1 == L ? j - sZw : j + sZ;
      nbi[5] = z == 0 ? j + sZw : j - sZ;
    }
  };
  for (uint32_t i = threadIdx.x; i < N; i += blockDim.x) {
    const uint32_t c = i >= Nh ? 1u : 0u;
    const uint32_t j = i - c * Nh;
    uint32_t v = gs[i] < 0 ? 1u : 0u;
    if (PM) {
      uint32_t nbi[6];
      nbr(c, j, nbi);
      const int8_t* Jo = gJ + (uint64_t)c * Nh;        // J[mu][c] = gJ + (2 mu + c) Nh
      const int8_t* Jn = gJ + (uint64_t)(1 - c) * Nh;  // J[mu][1 - c]
#pragma unroll
      for (int mu = 0; mu < D; ++mu) {
        v |= (Jo[2 * (uint64_t)mu * Nh + j] < 0 ? 1u : 0u) << (1 + 2 * mu);
        v |= (Jn[2 * (uint64_t)mu * Nh + nbi[2 * mu + 1]] < 0 ? 1u : 0u) << (2 + 2 * mu);
      }
    }
    lat[i] = (int8_t)v;
  }
  __syncthreads();

  // One site: k = bonds with J s_i s_nb < 0 from the combined bytes.
  auto site_k = [&](const int8_t* own, const int8_t* oth, uint32_t c, uint32_t j,
                    uint32_t& o) -> uint32_t {
    uint32_t nbi[6];
    nbr(c, j, nbi);
    o = (uint8_t)own[j];
    uint32_t nm = 0;
#pragma unroll
    for (int m = 0; m < 2 * D; ++m) nm |= ((uint32_t)(uint8_t)oth[nbi[m]] & 1u) << m;
    const uint32_t om = (0u - (o & 1u)) & ((1u << (2 * D)) - 1u);
    return __builtin_popcount(nm ^ om ^ (PM ? (o >> 1) : 0u));
  };
  // Four sites j .. j + 3 of one plane row (j % 4 == 0, R % 4 == 0): new
  // word of the own plane, decided by prefix word P; ties (prefix byte equal
  // to the threshold byte of a refusable class) take the site's refinement
  // draw on the spot.
  auto ld = [&](const int8_t* base, uint32_t i) -> uint32_t {
    return *reinterpret_cast<const uint32_t*>(base + i);
  };
  // Unsatisfied bonds per byte of the own word W against its 2d neighbour
  // words: the spin bits differ, xor the bond's sign bit.
  auto count_bytes = [&](uint32_t W, const uint32_t nb[6]) -> uint32_t {
    uint32_t k = 0;
#pragma unroll
    for (int m = 0; m < 2 * D; ++m) {
      uint32_t u = W ^ nb[m];
      if (PM) u ^= W >> (1 + m);
      k += u & kOnes;
    }
    return k;
  };
  // Unsatisfied-bond counts (byte b: site j + b) of a WB-site word of plane c
  // (WB = 4: j % 4 == 0 and R % 4 == 0; WB = 2: j even and R even; the word
  // lies in one plane row).  The in-row neighbours are the centre word
  // shifted by one byte with the adjacent word's edge byte.
  auto counts = [&](auto wb, const int8_t* own, const int8_t* oth, uint32_t c, uint32_t j,
                    uint32_t& W) -> uint32_t {
    constexpr uint32_t WB = decltype(wb)::value;
    auto ldw = [&](const int8_t* base, uint32_t i) -> uint32_t {
      if constexpr (WB == 4) return *reinterpret_cast<const uint32_t*>(base + i);
      else return *reinterpret_cast<const uint16_t*>(base + i);
    };
    const uint32_t r = fdiv(j, divR);
    const uint32_t rowb = r * R;
    const uint32_t jx = j - rowb;
    const uint32_t z = D == 3 ? fdiv(r, divL) : 0u;
    const uint32_t y = r - z * L;
    const uint32_t p = (c + r + z) & 1u;  // (c + y + z) & 1 with L even
    W = ldw(own, j);
    const uint32_t C = ldw(oth, j);
    // p = 1: x+1 is the next word's first byte onwards; p = 0: x-1 ends with
    // the previous word's last byte
    const uint32_t Ej = p ? (jx + WB == R ? rowb : j + WB) : (jx == 0 ? rowb + R - WB : j - WB);
    const uint32_t E = ldw(oth, Ej);
    uint32_t S;
    if constexpr (WB == 4)
      S = p ? __builtin_amdgcn_alignbyte(E, C, 1) : __builtin_amdgcn_alignbyte(C, E, 3);
    else
      S = p ? ((C >> 8) | ((E & 0xFFu) << 8)) : (((C << 8) & 0xFF00u) | (E >> 8));
    uint32_t nb[6];
    nb[0] = p ? S : C;  // +x
    nb[1] = p ? C : S;  // -x
    nb[2] = ldw(oth, y + 1 == L ? j - sYw : j + R);
    nb[3] = ldw(oth, y == 0 ? j + sYw : j - R);
    if (D == 3) {
      nb[4] = ldw(oth, z + 1 == L ? j - sZw : j + sZ);
      nb[5] = ldw(oth, z == 0 ? j + sZw : j - sZ);
    }
    return count_bytes(W, nb);
  };
  // New word for prefix bytes P (byte b: site j + b); `tie` gets bit 7 of
  // each byte whose prefix equals the threshold byte of a refusable class
  // (left unflipped), `kout` the counts.  Only the low WB bytes of the
  // result are meaningful.
  auto decide = [&](auto wb, uint32_t W, uint32_t k, uint32_t P, uint32_t& tie) -> uint32_t {
    constexpr uint32_t WB = decltype(wb)::value;
    const uint32_t Th = __builtin_amdgcn_perm(th_hi, th_lo, k);
    const uint32_t Al = __builtin_amdgcn_perm(al_hi, al_lo, k);
    const uint32_t x = P ^ Th;
    const uint32_t dlow = (P | kHigh) - (Th & ~kHigh);
    const uint32_t ge = (x & P) | (~x & dlow);  // bit 7 of each byte: P >= Th
    const uint32_t rej = __builtin_amdgcn_perm(ge, ge << 8, 0x0B090A08u);
    const uint32_t zb = (x & 0x7F7F7F7Fu) + 0x7F7F7F7Fu;
    tie = ~(zb | x | Al) & (WB == 4 ? kHigh : 0x8080u);
    return W ^ ((~rej | Al) & kOnes);
  };
  auto word = [&](auto wb, const int8_t* own, const int8_t* oth, uint32_t c, uint32_t j,
                  uint32_t P, uint32_t& tie, uint32_t& kout) -> uint32_t {
    uint32_t W;
    const uint32_t k = counts(wb, own, oth, c, j, W);
    kout = k;
    return decide(wb, W, k, P, tie);
  };
  using W4 = std::integral_constant<uint32_t, 4>;
  using W2 = std::integral_constant<uint32_t, 2>;
  // Ties wait in a per-lane LDS queue (entry (site << 3) | class, lane-major)
  // and are resolved by their refinement draws before the colour's barrier:
  // a lane alone writes the sites of its groups, so the late flip is
  // race-free, and a wave pays for the longest queue of its lanes once per
  // half-sweep instead of once per word.
  uint32_t* const tq = lat_words + (N + 15) / 16 * 4 + threadIdx.x;
  uint32_t nq = 0;
  auto flush = [&](int8_t* own, uint32_t c, uint32_t t) {
    for (uint32_t i = 0; i < nq; ++i) {
      const uint32_t e = tq[i * blockDim.x];
      const uint32_t js = e >> 3;
      const Rand4 rr = philox(js, t, replica, tag(c, kIsingRefine), key.k0, key.k1);
      if ((rr.w[0] & 0xFFFFFFu) < dp->frac[e & 7u]) own[js] ^= 1;
    }
    nq = 0;
  };
  const bool words = (R & 3u) == 0;
  const bool pairs = !words && (R & 1u) == 0;
  // E = sum over colour-1 sites of (unsatisfied - satisfied) bonds (each bond
  // once), M = sum of the spins of both colours; record `slot` of this call
  auto measure = [&](uint32_t slot, int64_t sweep) {
    int64_t Esum = 0, Msum = 0;
    if (words) {
      for (uint32_t j = 4 * threadIdx.x; j < Nh; j += 4 * blockDim.x) {
        uint32_t W;
        const uint32_t k = counts(W4{}, lat + Nh, lat, 1u, j, W);
        const uint32_t down = __builtin_popcount(W & kOnes) + __builtin_popcount(ld(lat, j) & kOnes);
        Esum += 2 * (int64_t)__builtin_amdgcn_sad_u8(k, 0u, 0u) - 4 * 2 * D;
        Msum += 8 - 2 * (int64_t)down;
      }
    } else if (pairs) {
      for (uint32_t j = 2 * threadIdx.x; j < Nh; j += 2 * blockDim.x) {
        uint32_t W;
        const uint32_t k = counts(W2{}, lat + Nh, lat, 1u, j, W);
        const uint32_t w0 = *reinterpret_cast<const uint16_t*>(lat + j);
        const uint32_t down = __builtin_popcount(W & kOnes) + __builtin_popcount(w0 & kOnes);
        Esum += 2 * (int64_t)__builtin_amdgcn_sad_u8(k, 0u, 0u) - 2 * 2 * D;
        Msum += 4 - 2 * (int64_t)down;
      }
    } else {
      for (uint32_t j = threadIdx.x; j < Nh; j += blockDim.x) {
        uint32_t o;
        const uint32_t k = site_k(lat + Nh, lat, 1u, j, o);
        Esum += 2 * (int64_t)k - 2 * D;
        Msum += (1 - 2 * (int32_t)(o & 1u)) + (1 - 2 * (int32_t)(lat[j] & 1));
      }
    }
    __shared__ Partial part[1];
    block_partial_int(Esum, Msum, part, 0);
    if (threadIdx.x == 0) {
      ObsOut o;
      o.E_int = part[0].Ei;
      o.M_int = part[0].Mi;
      o.E = (double)part[0].Ei * dp->J0;
      o.M[0] = (double)part[0].Mi;
      o.M[1] = 0.0;
      o.M[2] = 0.0;
      o.absM = fabs((double)part[0].Mi);
      o.sweep = sweep;
      obs[(uint64_t)slot * n_lattices + li] = o;
    }
  };
  const uint32_t ngroups = (Nh + 15) / 16;
  // One group per lane (a lattice with no more groups than lanes): the lane
  // sees the same four words in every half-sweep of the call, so their plane
  // indices and those of their neighbour words (periodic wraps included) are
  // formed once here.  Slot s holds word ws = (s + lane / 8) % 4 of the group
  // (the bank-spreading order of the general path); fpar bit s is the
  // word's (row + z) parity, fval bit s marks the words inside the plane.
  const bool fast = words && ngroups <= blockDim.x;
  uint32_t fj[4], fyp[4], fym[4], fzp[4], fzm[4], fe1[4], fe0[4];
  uint32_t fpar = 0, fval = 0;
  if (fast && threadIdx.x < ngroups) {
#pragma unroll
    for (uint32_t sl = 0; sl < 4; ++sl) {
      const uint32_t ws = (sl + (threadIdx.x >> 3)) & 3u;
      const uint32_t j = 16 * threadIdx.x + 4 * ws;
      const uint32_t jc = j < Nh ? j : 0u;  // words past the plane's end: never used
      fval |= (j < Nh ? 1u : 0u) << sl;
      const uint32_t r = fdiv(jc, divR);
      const uint32_t rowb = r * R;
      const uint32_t jx = jc - rowb;
      const uint32_t z = D == 3 ? fdiv(r, divL) : 0u;
      const uint32_t y = r - z * L;
      fpar |= ((r + z) & 1u) << sl;
      fj[sl] = jc;
      fe1[sl] = jx + 4 == R ? rowb : jc + 4;
      fe0[sl] = jx == 0 ? rowb + R - 4 : jc - 4;
      fyp[sl] = y + 1 == L ? jc - sYw : jc + R;
      fym[sl] = y == 0 ? jc + sYw : jc - R;
      fzp[sl] = fzm[sl] = 0;
      if (D == 3) {
        fzp[sl] = z + 1 == L ? jc - sZw : jc + sZ;
        fzm[sl] = z == 0 ? jc + sZw : jc - sZ;
      }
    }
  }
  for (uint32_t sw = 0; sw < n_sweeps; ++sw) {
    const uint32_t t = t0 + sw;
    for (uint32_t c = 0; c < 2; ++c) {
      int8_t* own = lat + c * Nh;
      const int8_t* oth = lat + (1 - c) * Nh;
      if (fast) {
        if (threadIdx.x < ngroups) {
          const uint32_t g = threadIdx.x;
          const Rand4 rp = philox(g, t, replica, tag(c, kIsingPrefix), key.k0, key.k1);
#pragma unroll
          for (uint32_t sl = 0; sl < 4; ++sl) {
            if ((fval >> sl) & 1u) {
              const uint32_t ws = (sl + (g >> 3)) & 3u;
              const uint32_t j = fj[sl];
              const uint32_t p = (c ^ (fpar >> sl)) & 1u;
              const uint32_t W = ld(own, j);
              const uint32_t C = ld(oth, j);
              const uint32_t E = ld(oth, p ? fe1[sl] : fe0[sl]);
              const uint32_t S = p ? __builtin_amdgcn_alignbyte(E, C, 1) : __builtin_amdgcn_alignbyte(C, E, 3);
              uint32_t nb[6];
              nb[0] = p ? S : C;  // +x
              nb[1] = p ? C : S;  // -x
              nb[2] = ld(oth, fyp[sl]);
              nb[3] = ld(oth, fym[sl]);
              nb[4] = nb[5] = 0;
              if (D == 3) {
                nb[4] = ld(oth, fzp[sl]);
                nb[5] = ld(oth, fzm[sl]);
              }
              const uint32_t k = count_bytes(W, nb);
              uint32_t tie;
              const uint32_t nw = decide(W4{}, W, k, word_of(rp.w, ws), tie);
              *reinterpret_cast<uint32_t*>(own + j) = nw;
              while (tie) {
                const uint32_t b = (uint32_t)__builtin_ctz(tie) >> 3;
                tie &= tie - 1;
                if (nq == kBatchTieSlots) flush(own, c, t);
                tq[nq * blockDim.x] = ((j + b) << 3) | ((k >> (8 * b)) & 7u);
                ++nq;
              }
            }
          }
        }
        flush(own, c, t);
        __syncthreads();
        continue;
      }
      if (words && (R & 15u) == 0) {
        // plane rows of whole groups: a group's four words share the row, its
        // parity and the periodic wraps of their y and z neighbours, formed
        // once per group
        for (uint32_t g = threadIdx.x; g < ngroups; g += blockDim.x) {
          const uint32_t j0 = 16 * g;
          const Rand4 rp = philox(g, t, replica, tag(c, kIsingPrefix), key.k0, key.k1);
          const uint32_t r = fdiv(j0, divR);
          const uint32_t rowb = r * R;
          const uint32_t jx0 = j0 - rowb;
          const uint32_t z = D == 3 ? fdiv(r, divL) : 0u;
          const uint32_t y = r - z * L;
          const uint32_t p = (c + r + z) & 1u;
          const uint32_t dyp = y + 1 == L ? 0u - sYw : R, dym = y == 0 ? sYw : 0u - R;
          const uint32_t dzp = z + 1 == L ? 0u - sZw : sZ, dzm = z == 0 ? sZw : 0u - sZ;
#pragma unroll
          for (uint32_t w = 0; w < 4; ++w) {
            const uint32_t ws = (w + (threadIdx.x >> 3)) & 3u;
            const uint32_t j = j0 + 4 * ws;
            const uint32_t jx = jx0 + 4 * ws;
            const uint32_t W = ld(own, j);
            const uint32_t C = ld(oth, j);
            const uint32_t E = ld(oth, p ? (jx + 4 == R ? rowb : j + 4) : (jx == 0 ? rowb + R - 4 : j - 4));
            const uint32_t S = p ? __builtin_amdgcn_alignbyte(E, C, 1) : __builtin_amdgcn_alignbyte(C, E, 3);
            uint32_t nb[6];
            nb[0] = p ? S : C;  // +x
            nb[1] = p ? C : S;  // -x
            nb[2] = ld(oth, j + dyp);
            nb[3] = ld(oth, j + dym);
            nb[4] = nb[5] = 0;
            if (D == 3) {
              nb[4] = ld(oth, j + dzp);
              nb[5] = ld(oth, j + dzm);
            }
            const uint32_t k = count_bytes(W, nb);
            uint32_t tie;
            const uint32_t nw = decide(W4{}, W, k, word_of(rp.w, ws), tie);
            *reinterpret_cast<uint32_t*>(own + j) = nw;
            while (tie) {
              const uint32_t b = (uint32_t)__builtin_ctz(tie) >> 3;
              tie &= tie - 1;
              if (nq == kBatchTieSlots) flush(own, c, t);
              tq[nq * blockDim.x] = ((j + b) << 3) | ((k >> (8 * b)) & 7u);
              ++nq;
            }
          }
        }
        flush(own, c, t);
        __syncthreads();
        continue;
      }
      if (words) {
        // Nh is a multiple of 4: a group holds nj / 4 whole words
        for (uint32_t g = threadIdx.x; g < ngroups; g += blockDim.x) {
          const uint32_t j0 = 16 * g;
          const Rand4 rp = philox(g, t, replica, tag(c, kIsingPrefix), key.k0, key.k1);
          const uint32_t nwords = Nh - j0 < 16 ? (Nh - j0) >> 2 : 4u;
#pragma unroll
          for (uint32_t w = 0; w < 4; ++w) {
            // lanes 8 apart start on different words of their groups: the
            // words of a step then fall in different LDS banks
            const uint32_t ws = (w + (threadIdx.x >> 3)) & 3u;
            if (ws < nwords) {
              const uint32_t j = j0 + 4 * ws;
              uint32_t tie, k;
              const uint32_t nw = word(W4{}, own, oth, c, j, word_of(rp.w, ws), tie, k);
              *reinterpret_cast<uint32_t*>(own + j) = nw;
              while (tie) {
                const uint32_t b = (uint32_t)__builtin_ctz(tie) >> 3;
                tie &= tie - 1;
                if (nq == kBatchTieSlots) flush(own, c, t);
                tq[nq * blockDim.x] = ((j + b) << 3) | ((k >> (8 * b)) & 7u);
                ++nq;
              }
            }
          }
        }
        flush(own, c, t);
        __syncthreads();
        continue;
      }
      if (pairs) {
        // Nh is even: a group holds nj / 2 whole pairs
        for (uint32_t g = threadIdx.x; g < ngroups; g += blockDim.x) {
          const uint32_t j0 = 16 * g;
          const Rand4 rp = philox(g, t, replica, tag(c, kIsingPrefix), key.k0, key.k1);
          const uint32_t npairs = Nh - j0 < 16 ? (Nh - j0) >> 1 : 8u;
          // not unrolled: the few lattices on this path must not raise the
          // register count of the whole kernel
#pragma unroll 1
          for (uint32_t w = 0; w < 8; ++w) {
            // lanes 8 apart start on different dwords of their groups
            const uint32_t ps = (w + 2 * ((threadIdx.x >> 3) & 3u)) & 7u;
            if (ps < npairs) {
              const uint32_t j = j0 + 2 * ps;
              const uint32_t P = word_of(rp.w, ps >> 1) >> (8 * (j & 2u));
              uint32_t tie, k;
              const uint32_t nw = word(W2{}, own, oth, c, j, P, tie, k);
              *reinterpret_cast<uint16_t*>(own + j) = (uint16_t)nw;
              while (tie) {
                const uint32_t b = (uint32_t)__builtin_ctz(tie) >> 3;
                tie &= tie - 1;
                if (nq == kBatchTieSlots) flush(own, c, t);
                tq[nq * blockDim.x] = ((j + b) << 3) | ((k >> (8 * b)) & 7u);
                ++nq;
              }
            }
          }
        }
        flush(own, c, t);
        __syncthreads();
        continue;
      }
      for (uint32_t g = threadIdx.x; g < ngroups; g += blockDim.x) {
        const uint32_t j0 = 16 * g;
        const Rand4 rp = philox(g, t, replica, tag(c, kIsingPrefix), key.k0, key.k1);
        const uint32_t nj = Nh - j0 < 16 ? Nh - j0 : 16u;
        auto one = [&](uint32_t jj, uint32_t word) {
          const uint32_t j = j0 + jj;
          uint32_t o;
          const uint32_t k = site_k(own, oth, c, j, o);
          const uint32_t P = (word >> (8 * (jj & 3))) & 0xFFu;
          const uint32_t Th = table_byte(th_lo, th_hi, k);
          bool accept = P < Th;
          if (P == Th) {
            const Rand4 rr = philox(j, t, replica, tag(c, kIsingRefine), key.k0, key.k1);
            accept = (rr.w[0] & 0xFFFFFFu) < dp->frac[k];  // rare: read from the table
          }
          if (accept) own[j] = (int8_t)(o ^ 1u);
        };
        // not unrolled: the few lattices on this path must not raise the
        // register count of the whole kernel
#pragma unroll 1
        for (uint32_t jj = 0; jj < nj; ++jj) one(jj, word_of(rp.w, jj >> 2));
      }
      __syncthreads();
    }
    // every thread reaches the barrier inside the block reduction after its
    // reads of the planes: none writes them again before all have read
    if (MEASURE && (sw + 1) % every == 0) measure((sw + 1) / every - 1, (int64_t)t + 1);
  }
  if (MEASURE && n_sweeps == 0) measure(0, (int64_t)t0);

  // write both planes back as +-1 bytes
  for (uint32_t i = threadIdx.x; i < N; i += blockDim.x) gs[i] = (lat[i] & 1) ? (int8_t)-1 : (int8_t)1;

}

bool batch_lattice_packed(int d, uint32_t L, uint32_t threads) {
  return batch_packed_ok(d, L, threads);
}

size_t batch_lds_bytes(int d, bool pm, bool packed, const uint32_t* L, uint32_t n,
                       uint32_t threads) {
  size_t bytes = 0;
  for (uint32_t r = 0; r < n; ++r) {
    size_t need;
    if (packed && batch_packed_ok(d, L[r], threads)) {
      need = batch_packed_lds_bytes(L[r], pm, threads);
    } else {
      size_t N = 1;
      for (int k = 0; k < d; ++k) N *= L[r];
      need = (N + 15) / 16 * 16 + (size_t)threads * kBatchTieSlots * 4;
    }
    bytes = need > bytes ? need : bytes;
  }
  return bytes;
}

hipError_t launch_batch(const BatchLaunch& a, int8_t* spins, const int8_t* J, uint32_t t0,
                        uint32_t n_sweeps, uint32_t every, void* dev_obs, hipStream_t st) {
  const dim3 grid(a.n_lattices), block(a.threads);
  const size_t lds = a.lds_bytes;
#define SMC_BK(DD, PMM, MM)                                                                      \
  hipLaunchKernelGGL((batch_kernel<DD, PMM, MM>), grid, block, lds, st, a.descs, a.order, a.key, \
                     spins, J, t0, n_sweeps, every, a.n_lattices, (ObsOut*)dev_obs)
  const bool m = dev_obs != nullptr;
  if (a.d == 2) {
    if (a.pm) { if (m) SMC_BK(2, true, true); else SMC_BK(2, true, false); }
    else { if (m) SMC_BK(2, false, true); else SMC_BK(2, false, false); }
  } else {
    if (a.pm) { if (m) SMC_BK(3, true, true); else SMC_BK(3, true, false); }
    else { if (m) SMC_BK(3, false, true); else SMC_BK(3, false, false); }
  }
#undef SMC_BK
  return hipGetLastError();
}

// Dynamic LDS beyond the default 64 KiB needs the kernels' attribute raised.
hipError_t batch_allow_lds(size_t bytes) {
  hipError_t e = hipSuccess;
#define SMC_BA(DD, PMM, MM)                                                                     \
  if (e == hipSuccess)                                                                          \
    e = allow_dynamic_lds((const void*)batch_kernel<DD, PMM, MM>, bytes)
  SMC_BA(2, true, true); SMC_BA(2, true, false); SMC_BA(2, false, true); SMC_BA(2, false, false);
  SMC_BA(3, true, true); SMC_BA(3, true, false); SMC_BA(3, false, true); SMC_BA(3, false, false);
#undef SMC_BA
  return e;
}

}  // namespace smc

namespace smc {

const void* batch_kernel_fn(int d, bool pm, bool measure) {
  if (d == 2) {
    if (pm) return measure ? (const void*)batch_kernel<2, true, true> : (const void*)batch_kernel<2, true, false>;
    return measure ? (const void*)batch_kernel<2, false, true> : (const void*)batch_kernel<2, false, false>;
  }
  if (pm) return measure ? (const void*)batch_kernel<3, true, true> : (const void*)batch_kernel<3, true, false>;
  return measure ? (const void*)batch_kernel<3, false, true> : (const void*)batch_kernel<3, false, false>;
}

}  // namespace smc
