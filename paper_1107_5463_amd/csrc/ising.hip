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
#include "reduce.hpp"

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

// ---------------------------------------------------------------------------
// One site per thread.
// ---------------------------------------------------------------------------
template <int D, int JK>
__global__ __launch_bounds__(256) void ising_site_kernel(const Geom g, const RngKey key,
                                                         const IsingTable tab,
                                                         const void* __restrict__ J,
                                                         const float beta,
                                                         int8_t* __restrict__ s,
                                                         const uint32_t t, const uint32_t c,
                                                         const int heatbath) {
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
      accept = metropolis_fp32(dE, u01f(pick4(r, (uint32_t)j & 3u)), beta_log2e(beta));
    }
  } else {
    const uint32_t k = (uint32_t)kunsat;
    const Rand4 r = philox((uint32_t)(j >> 4), t, key.replica, tag(c, kIsingPrefix), key.k0,
                           key.k1);
    const uint32_t P = (pick4(r, ((uint32_t)j >> 2) & 3u) >> (8 * ((uint32_t)j & 3u))) & 0xFFu;
    if (heatbath) {
      // class: neighbours with sign(J) s_nb = +1; new spin +1 iff u32 < T_hb
      const uint32_t npos = si > 0 ? 2u * D - k : k;
      const uint32_t Th = table_byte(tab.th_lo, tab.th_hi, npos);
      bool upv = P < Th;
      if (P == Th) {
        const Rand4 rr = philox((uint32_t)j, t, key.replica, tag(c, kIsingRefine), key.k0, key.k1);
        upv = (rr.w[0] & 0xFFFFFFu) < frac_of(tab, npos);
      }
      const int8_t nv = upv ? (int8_t)1 : (int8_t)-1;
      if (nv != si) own[j] = nv;
      return;
    }
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
template <int D, bool PM>
__global__ __launch_bounds__(256) void ising_chunk_kernel(const Geom g, const RngKey key,
                                                          const IsingTable tab,
                                                          const int8_t* __restrict__ J,
                                                          const FastDiv divQ, const FastDiv divL,
                                                          int8_t* __restrict__ s,
                                                          const uint32_t t, const uint32_t c) {
  const uint32_t gid = xcd_remap(blockIdx.x, gridDim.x) * 256u + threadIdx.x;
  if (gid >= (uint32_t)(g.Nh >> 4)) return;
  int64_t base;
  Chunk o, ctr;
  uint32_t kk[4];
  chunk_counts<D, PM>(g, s, J, divQ, divL, c, gid, base, o, ctr, kk);
  int8_t* own = s + (int64_t)c * g.Nh;
  // rare prefix ties on uphill moves are resolved exactly by the sites'
  // 24-bit refinement draws
  const Chunk n = update_chunk_now(tab_regs(tab), key, t, c, (uint32_t)base, o, kk);
  const uint32_t nw[4] = {n.w[0], n.w[1], n.w[2], n.w[3]};
  st16(own + base, nw);
}


// ---------------------------------------------------------------------------
// Streaming half-sweep (uniform couplings, L % 32 == 0).  Lane (band, q) owns
// chunk column q of plane rows band*H .. band*H + H - 1 (H divides L, so a
// band stays inside one z-plane) and walks down them, keeping the other
// colour's rows y-1, y, y+1 of its column in registers: per row it loads one
// new other-colour chunk, its own chunk (both one row ahead), one edge word,
// and in 3D the two z-neighbour chunks.  Bands of neighbouring rows fall in
// the same XCD (xcd_remap), so the band halo rows and the z-neighbour rows
// are L2 hits.
// ---------------------------------------------------------------------------
template <int D, bool MEASURE>
__global__ __launch_bounds__(256) void ising_stream_kernel(const Geom g, const RngKey key,
                                                           const IsingTable table,
                                                           const FastDiv divQ, const FastDiv divL,
                                                           const uint32_t H, const uint32_t nbands,
                                                           int8_t* __restrict__ s,
                                                           const uint32_t t, const uint32_t c,
                                                           Partial* __restrict__ parts) {
  __shared__ uint16_t tie_slots[kTieSlots * 256];
  const uint32_t tid = xcd_remap(blockIdx.x, gridDim.x) * 256u + threadIdx.x;
  const uint32_t band = fdiv(tid, divQ);
  int64_t Esum = 0, Msum = 0;
  if (band < nbands) {
    const uint32_t Q = divQ.d;
    const uint32_t q = tid - band * Q;
    const uint32_t L = (uint32_t)g.L;
    const uint32_t R = (uint32_t)g.R;
    const uint32_t r0 = band * H;
    uint32_t z = 0, y0 = r0;
    if (D == 3) {
      z = fdiv(r0, divL);
      y0 = r0 - z * L;
    }
    int8_t* own = s + (int64_t)c * g.Nh;
    const int8_t* oth = s + (int64_t)(1 - c) * g.Nh;
    const uint32_t col = 16 * q;
    const uint32_t zrow = L * z;  // row index of (y = 0, z)
    const uint32_t qn = q + 1 == Q ? 0u : q + 1, qp = q == 0 ? Q - 1 : q - 1;
    // the in-row neighbour chunk's edge word: next chunk's word 0 (parity 1)
    // or previous chunk's word 3 (parity 0); parity alternates with y
    const uint32_t pz = (c + z) & 1u;
    const uint32_t edge_even = pz ? 16 * qn : 16 * qp + 12;  // rows with y even
    const uint32_t edge_odd = pz ? 16 * qp + 12 : 16 * qn;
    auto roff = [&](uint32_t y) -> uint32_t {  // y in [0, 2L)
      return (zrow + (y >= L ? y - L : y)) * R;
    };
    uint32_t zm_row = 0, zp_row = 0;
    if (D == 3) {
      zm_row = L * (z == 0 ? L - 1 : z - 1);
      zp_row = L * (z + 1 == L ? 0 : z + 1);
    }
    auto zoff = [&](uint32_t zr, uint32_t y) -> uint32_t { return (zr + (y >= L ? y - L : y)) * R + col; };
    const TabRegs tab = tab_regs(table);
    TieQueue tq;
    tq.slot = tie_slots + threadIdx.x;
    tq.stride = 256;
    tq.n = 0;
    tq.base = roff(y0) + col;
    tq.R = R;
    tq.dE = 0;
    tq.dM = 0;

    // Software pipeline: slot y & 3 of Ro holds the other colour's row y,
    // slot y & 1 of Ow / Ed / Fz / Bz our own row y, its edge word and its
    // z-neighbours.  A load is issued only into a slot whose row is dead and
    // is consumed at least one full row later, so no wait stalls the stream.
    Chunk Ro[4], Ow[2], Fz[2], Bz[2];
    uint32_t Ed[2];
    const uint32_t ym1 = y0 == 0 ? L - 1 : y0 - 1;
    Ro[3] = ld16(oth + roff(ym1) + col);
    Ro[0] = ld16(oth + roff(y0) + col);
    Ro[1] = ld16(oth + roff(y0 + 1) + col);
    Ro[2] = ld16(oth + roff(y0 + 2) + col);
    Ow[0] = ld16(own + roff(y0) + col);
    Ow[1] = ld16(own + roff(y0 + 1) + col);
    Ed[0] = *reinterpret_cast<const uint32_t*>(oth + roff(y0) + edge_even);
    Ed[1] = *reinterpret_cast<const uint32_t*>(oth + roff(y0 + 1) + edge_odd);
    if (D == 3) {
      Fz[0] = ld16(oth + zoff(zm_row, y0));
      Fz[1] = ld16(oth + zoff(zm_row, y0 + 1));
      Bz[0] = ld16(oth + zoff(zp_row, y0));
      Bz[1] = ld16(oth + zoff(zp_row, y0 + 1));
    }
    for (uint32_t i = 0; i < H; i += 4) {
#pragma unroll
      for (int ph = 0; ph < 4; ++ph) {
        const uint32_t y = y0 + i + ph;  // y0 and i are multiples of 4: y & 3 == ph
        const uint32_t p = (pz + ph) & 1u;
        const Chunk& up = Ro[(ph + 3) & 3];
        const Chunk& ct = Ro[ph];
        const Chunk& dn = Ro[(ph + 1) & 3];
        const Chunk& o = Ow[ph & 1];
        const uint32_t e = Ed[ph & 1];
        const Chunk sh = p ? shift_next(ct, e) : shift_prev(ct, e);
        const uint32_t jbase = roff(y) + col;
        uint32_t kk[4];
#pragma unroll
        for (int w = 0; w < 4; ++w) {
          const uint32_t ow = o.w[w];
          uint32_t k2 = ((ow ^ ct.w[w]) & kBit1) + ((ow ^ sh.w[w]) & kBit1) +
                        ((ow ^ up.w[w]) & kBit1) + ((ow ^ dn.w[w]) & kBit1);
          if (D == 3) k2 += ((ow ^ Fz[ph & 1].w[w]) & kBit1) + ((ow ^ Bz[ph & 1].w[w]) & kBit1);
          kk[w] = k2 >> 1;
        }
        // rare exact ties are queued and resolved at the end of the band
        const Chunk nc = update_chunk_deferred<D>(tab, key, t, c, jbase, i + ph, o, kk, tq, own);
        uint32_t nw[4] = {nc.w[0], nc.w[1], nc.w[2], nc.w[3]};
        st16(own + jbase, nw);
        if (MEASURE) {
          // colour 1 after its update: every bond has one colour-1 end, and the
          // colour-0 chunk at the same position covers each colour-0 site once
          uint32_t kn[4];
#pragma unroll
          for (int w = 0; w < 4; ++w) {
            uint32_t k2 = ((nw[w] ^ ct.w[w]) & kBit1) + ((nw[w] ^ sh.w[w]) & kBit1) +
                          ((nw[w] ^ up.w[w]) & kBit1) + ((nw[w] ^ dn.w[w]) & kBit1);
            if (D == 3)
              k2 += ((nw[w] ^ Fz[ph & 1].w[w]) & kBit1) + ((nw[w] ^ Bz[ph & 1].w[w]) & kBit1);
            kn[w] = k2 >> 1;
          }
          Chunk nc;
          nc.w[0] = nw[0]; nc.w[1] = nw[1]; nc.w[2] = nw[2]; nc.w[3] = nw[3];
          Esum += -(int64_t)(16 * 2 * D) + 2 * (int64_t)chunk_count_sum(kn);
          Msum += chunk_spin_sum(nc) + chunk_spin_sum(ct);
        }
        // refill the dead slots: other row y + 3, own row y + 2 with its edge
        // word and z-neighbours (rows past the band are read, never used)
        Ro[(ph + 3) & 3] = ld16(oth + roff(y + 3) + col);
        Ow[ph & 1] = ld16(own + roff(y + 2) + col);
        Ed[ph & 1] = *reinterpret_cast<const uint32_t*>(oth + roff(y + 2) + ((ph & 1) ? edge_odd : edge_even));
        if (D == 3) {
          Fz[ph & 1] = ld16(oth + zoff(zm_row, y + 2));
          Bz[ph & 1] = ld16(oth + zoff(zp_row, y + 2));
        }
      }
    }
    // deferred ties: the site belongs to this lane's column of its own colour,
    // which no other lane of this launch touches
    tie_flush<D>(tq, tab, key, t, c, own);
    if (MEASURE) {
      Esum += tq.dE;
      Msum += tq.dM;
    }
  }
  if (MEASURE) block_partial_int(Esum, Msum, parts, blockIdx.x);
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
                         a.J, a.beta, spins, t, c, a.heatbath);
      break;
    case 1:
      hipLaunchKernelGGL((ising_site_kernel<D, 1>), grid, dim3(256), 0, st, a.g, a.key, a.tab,
                         a.J, a.beta, spins, t, c, a.heatbath);
      break;
    default:
      hipLaunchKernelGGL((ising_site_kernel<D, 2>), grid, dim3(256), 0, st, a.g, a.key, a.tab,
                         a.J, a.beta, spins, t, c, a.heatbath);
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

// Rows per band of the streaming kernel: the largest divisor of L up to 64
// that still gives at least `min_waves` waves.
uint32_t stream_rows_per_band(const Geom& g, uint32_t min_waves) {
  const uint32_t Q = (uint32_t)(g.R / 16);
  uint32_t best = 4;
  for (uint32_t H = 4; H <= 64; H *= 2) {  // the tie queue holds rows < 64
    if (g.L % H) break;
    const uint64_t waves = (uint64_t)Q * (uint64_t)(g.rows / H) / 64;
    if (waves >= min_waves) best = H;
  }
  return best;
}

template <int D>
static hipError_t launch_stream(const IsingLaunch& a, int8_t* spins, uint32_t t, uint32_t c,
                                hipStream_t st, void* partials = nullptr, int64_t* nparts = nullptr) {
  const uint32_t H = a.rows_per_band;
  const uint32_t nbands = (uint32_t)a.g.rows / H;
  const uint64_t threads = (uint64_t)nbands * a.divQ.d;
  const dim3 grid((unsigned)((threads + 255) / 256));
  if (partials) {
    hipLaunchKernelGGL((ising_stream_kernel<D, true>), grid, dim3(256), 0, st, a.g, a.key, a.tab,
                       a.divQ, a.divL, H, nbands, spins, t, c, (Partial*)partials);
    if (nparts) *nparts = grid.x;
  } else {
    hipLaunchKernelGGL((ising_stream_kernel<D, false>), grid, dim3(256), 0, st, a.g, a.key, a.tab,
                       a.divQ, a.divL, H, nbands, spins, t, c, (Partial*)nullptr);
  }
  return hipGetLastError();
}

// Colour-1 half-sweep of the streaming kernel with the observables of the
// resulting state reduced on the way; false if the handle's kernel is not
// the streaming one (the caller measures separately).
bool ising_half_sweep_measured(const IsingLaunch& a, int8_t* spins, uint32_t t, void* partials,
                               int64_t* nparts, hipStream_t st, hipError_t* err) {
  if (ising_variant_used(a) != kVariantStream) return false;
  *err = a.g.d == 2 ? launch_stream<2>(a, spins, t, 1u, st, partials, nparts)
                    : launch_stream<3>(a, spins, t, 1u, st, partials, nparts);
  return true;
}

int ising_variant_used(const IsingLaunch& a) {
  if (a.heatbath) return kVariantSite;  // the heat-bath rule runs on the site kernel
  int v = a.variant == kVariantFusedWave ? kVariantAuto : a.variant;
  const bool chunk_ok = ising_chunk_supported(a.g, a.J_kind);
  if (v == kVariantAuto) v = !chunk_ok ? kVariantSite : (a.J_kind == 0 ? kVariantStream : kVariantChunk);
  if (v == kVariantStream && !(chunk_ok && a.J_kind == 0 && a.rows_per_band >= 4 &&
                               a.rows_per_band % 4 == 0 && a.g.L % a.rows_per_band == 0))
    v = chunk_ok ? kVariantChunk : kVariantSite;
  if (v == kVariantChunk && !chunk_ok) v = kVariantSite;
  return v;
}

hipError_t launch_ising_half_sweep(const IsingLaunch& a, int8_t* spins, uint32_t t,
                                   uint32_t colour, hipStream_t st) {
  const int v = ising_variant_used(a);
  if (a.g.d == 2) {
    if (v == kVariantStream) return launch_stream<2>(a, spins, t, colour, st);
    if (v == kVariantChunk) return launch_chunk<2>(a, spins, t, colour, st);
    return launch_site<2>(a, spins, t, colour, st);
  }
  if (v == kVariantStream) return launch_stream<3>(a, spins, t, colour, st);
  if (v == kVariantChunk) return launch_chunk<3>(a, spins, t, colour, st);
  return launch_site<3>(a, spins, t, colour, st);
}

}  // namespace smc
