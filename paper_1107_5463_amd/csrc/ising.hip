// ising.hip -- checkerboard Metropolis half-sweeps for Ising spins (n = 1).
//
// One launch updates every site of one colour (Sec. 2 of the paper: all sites
// of a sublattice are independent given the other sublattice).  Decision per
// site (Eq. (2)): k = number of unsatisfied bonds (J_b s_i s_b < 0), dE =
// 4 J0 (d - k); accept iff class k is "always" (dE <= 0) or the site's 32-bit
// uniform u32 = prefix byte << 24 | refinement word is below the integer
// threshold T[k] = ceil(2^32 exp(-beta dE)).  The prefix byte decides unless
// it equals T[k] >> 24 (probability 2^-8), and only then is the refinement
// block drawn.
//
// Two kernels give bit-identical results:
//  * ising_site_kernel -- one site per thread, any even L, any coupling kind;
//  * ising_chunk_kernel -- one 16-byte chunk (16 consecutive same-colour
//    sites of a plane row) per lane, L % 32 == 0, uniform or +-1 couplings.
//    Neighbour chunks are loaded as whole 16-byte vectors; the in-row
//    neighbour is the centre chunk shifted by one byte (v_alignbyte) with one
//    edge word from the adjacent chunk; unsatisfied-bond counts are formed
//    four sites per 32-bit op (SWAR on bit 1 of the +-1 bytes); the threshold
//    bytes come from a v_perm byte lookup; one Philox block supplies the 16
//    prefix bytes.
#include "chunk.hpp"

namespace smc {

FastDiv make_fastdiv(uint32_t d) {
  FastDiv f{d, 0u, 0u};
  if (d <= 1) return f;
  uint32_t l = 0;
  while ((1ull << l) < d) ++l;
  const unsigned __int128 num = ((unsigned __int128)1 << 32) * (((uint64_t)1 << l) - d);
  f.m = (uint32_t)(num / d + 1);
  f.s = l - 1;
  return f;
}

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

// ---------------------------------------------------------------------------
// One site per thread.
// ---------------------------------------------------------------------------
template <int D, int JK>
__global__ __launch_bounds__(256) void ising_site_kernel(const Geom g, const RngKey key,
                                                         const IsingTable tab,
                                                         const void* __restrict__ J,
                                                         const float beta,
                                                         int8_t* __restrict__ s,
                                                         const uint32_t t, const uint32_t c) {
  const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (j >= g.Nh) return;
  const int64_t Nh = g.Nh;
  int8_t* own = s + (int64_t)c * Nh;
  const int8_t* oth = s + (int64_t)(1 - c) * Nh;
  int32_t x, y, z;
  site_coords(g, c, j, x, y, z);
  const int si = own[j];
  int kunsat = 0;
  float h = 0.0f;
#pragma unroll
  for (int mu = 0; mu < D; ++mu) {
    int32_t xp = x, yp = y, zp = z, xm = x, ym = y, zm = z;
    if (mu == 0) { xp = wrap(x + 1, g.L); xm = wrap(x - 1, g.L); }
    if (mu == 1) { yp = wrap(y + 1, g.L); ym = wrap(y - 1, g.L); }
    if (mu == 2) { zp = wrap(z + 1, g.L); zm = wrap(z - 1, g.L); }
    const int64_t ip = plane_index(g, xp, yp, zp);
    const int64_t im = plane_index(g, xm, ym, zm);
    const int sp = oth[ip], sm = oth[im];
    if (JK == 2) {
      const float* Jf = (const float*)J;
      const float jp = Jf[((int64_t)mu * 2 + c) * Nh + j];
      const float jm = Jf[((int64_t)mu * 2 + (1 - c)) * Nh + im];
      h += jp * (float)sp;
      h += jm * (float)sm;
    } else {
      int sgp = 1, sgm = 1;
      if (JK == 1) {
        const int8_t* Jb = (const int8_t*)J;
        sgp = Jb[((int64_t)mu * 2 + c) * Nh + j];
        sgm = Jb[((int64_t)mu * 2 + (1 - c)) * Nh + im];
      }
      kunsat += (sgp * si * sp < 0) + (sgm * si * sm < 0);
    }
  }
  bool accept;
  if (JK == 2) {
    const float dE = 2.0f * (float)si * h;
    if (dE <= 0.0f) {
      accept = true;
    } else {
      const Rand4 r = philox((uint32_t)(j >> 2), t, key.replica, tag(c, kContinuous), key.k0,
                             key.k1);
      accept = u01f(pick4(r, (uint32_t)j & 3u)) < expf(-beta * dE);
    }
  } else {
    const uint32_t k = (uint32_t)kunsat;
    const Rand4 r = philox((uint32_t)(j >> 4), t, key.replica, tag(c, kIsingPrefix), key.k0,
                           key.k1);
    const uint32_t P = (pick4(r, ((uint32_t)j >> 2) & 3u) >> (8 * ((uint32_t)j & 3u))) & 0xFFu;
    const uint32_t Th = table_byte(tab.th_lo, tab.th_hi, k);
    const bool always = table_byte(tab.al_lo, tab.al_hi, k) != 0;
    accept = always || P < Th;
    if (!accept && P == Th) {
      const Rand4 rr = philox((uint32_t)j, t, key.replica, tag(c, kIsingRefine), key.k0, key.k1);
      accept = (rr.w[0] & 0xFFFFFFu) < frac_of(tab, k);
    }
  }
  if (accept) own[j] = (int8_t)(-si);
}

// ---------------------------------------------------------------------------
// 16 sites per lane.
// ---------------------------------------------------------------------------
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

template <int D, bool PM>
__global__ __launch_bounds__(256) void ising_chunk_kernel(const Geom g, const RngKey key,
                                                          const IsingTable tab,
                                                          const int8_t* __restrict__ J,
                                                          const FastDiv divQ, const FastDiv divL,
                                                          int8_t* __restrict__ s,
                                                          const uint32_t t, const uint32_t c) {
  const uint32_t gid = blockIdx.x * 256u + threadIdx.x;
  if (gid >= (uint32_t)(g.Nh >> 4)) return;
  int64_t base;
  Chunk o, ctr;
  uint32_t kk[4];
  chunk_counts<D, PM>(g, s, J, divQ, divL, c, gid, base, o, ctr, kk);
  int8_t* own = s + (int64_t)c * g.Nh;
  const Rand4 rp = philox((uint32_t)(base >> 4), t, key.replica, tag(c, kIsingPrefix), key.k0,
                          key.k1);
  uint32_t nw[4], tie[4];
  uint32_t tie_any = 0;
#pragma unroll
  for (int w = 0; w < 4; ++w) {
    nw[w] = decide4(tab, o.w[w], kk[w], rp.w[w], tie[w]);
    tie_any |= tie[w];
  }
  if (tie_any) {
    // rare: some prefix byte equals its threshold byte on an uphill move;
    // resolve exactly with the site's 24-bit refinement draw
#pragma unroll
    for (int w = 0; w < 4; ++w) {
      if (!tie[w]) continue;
      for (int b = 0; b < 4; ++b) {
        const uint32_t k = (kk[w] >> (8 * b)) & 0xFFu;
        const uint32_t P = (rp.w[w] >> (8 * b)) & 0xFFu;
        if (P != table_byte(tab.th_lo, tab.th_hi, k) || table_byte(tab.al_lo, tab.al_hi, k))
          continue;
        const uint32_t jsite = (uint32_t)base + 4u * w + b;
        const Rand4 rr = philox(jsite, t, key.replica, tag(c, kIsingRefine), key.k0, key.k1);
        if ((rr.w[0] & 0xFFFFFFu) < frac_of(tab, k)) nw[w] ^= 0xFEu << (8 * b);
      }
    }
  }
  st16(own + base, nw);
}

bool ising_chunk_supported(const Geom& g, int J_kind) {
  return J_kind != 2 && (g.L % 32) == 0;
}

template <int D>
static hipError_t launch_site(const IsingLaunch& a, int8_t* spins, uint32_t t, uint32_t c,
                              hipStream_t st) {
  const dim3 grid((unsigned)((a.g.Nh + 255) / 256));
  switch (a.J_kind) {
    case 0:
      hipLaunchKernelGGL((ising_site_kernel<D, 0>), grid, dim3(256), 0, st, a.g, a.key, a.tab,
                         a.J, a.beta, spins, t, c);
      break;
    case 1:
      hipLaunchKernelGGL((ising_site_kernel<D, 1>), grid, dim3(256), 0, st, a.g, a.key, a.tab,
                         a.J, a.beta, spins, t, c);
      break;
    default:
      hipLaunchKernelGGL((ising_site_kernel<D, 2>), grid, dim3(256), 0, st, a.g, a.key, a.tab,
                         a.J, a.beta, spins, t, c);
      break;
  }
  return hipGetLastError();
}

template <int D>
static hipError_t launch_chunk(const IsingLaunch& a, int8_t* spins, uint32_t t, uint32_t c,
                               hipStream_t st) {
  const uint32_t nchunks = (uint32_t)(a.g.Nh >> 4);
  const dim3 grid((nchunks + 255) / 256);
  if (a.J_kind == 1)
    hipLaunchKernelGGL((ising_chunk_kernel<D, true>), grid, dim3(256), 0, st, a.g, a.key, a.tab,
                       (const int8_t*)a.J, a.divQ, a.divL, spins, t, c);
  else
    hipLaunchKernelGGL((ising_chunk_kernel<D, false>), grid, dim3(256), 0, st, a.g, a.key,
                       a.tab, (const int8_t*)a.J, a.divQ, a.divL, spins, t, c);
  return hipGetLastError();
}

hipError_t launch_ising_half_sweep(const IsingLaunch& a, int8_t* spins, uint32_t t,
                                   uint32_t colour, hipStream_t st) {
  const bool chunk = !a.generic && ising_chunk_supported(a.g, a.J_kind);
  if (a.g.d == 2)
    return chunk ? launch_chunk<2>(a, spins, t, colour, st) : launch_site<2>(a, spins, t, colour, st);
  return chunk ? launch_chunk<3>(a, spins, t, colour, st) : launch_site<3>(a, spins, t, colour, st);
}

}  // namespace smc
