// fused.hip -- one kernel per sweep for the 2D Ising model with uniform
// couplings (the fused alternative to the two colour passes).
//
// The sweep reads the state A (both colours) and writes the next state B, so
// every byte crosses HBM once in each direction (2 B per attempt instead of 3
// for the two in-place passes).  A workgroup spans one whole plane row (Q
// lanes, one 16-byte chunk column each) and walks a band of H rows: step i
// forms the new colour-0 row y = y0 + i from the old colour-1 rows y-1, y,
// y+1, then the new colour-1 row y-1 from the new colour-0 rows y-2, y-1, y.
// The in-row neighbours need one edge word of the adjacent chunk, which the
// neighbouring lane publishes in LDS (double-buffered, one barrier per step;
// the row wraps inside the workgroup).  A band also forms the new colour-0
// rows y0-1 and y0+H, which it does not store: the bands above and below own
// them.  Because the random numbers are keyed by (seed, t, site, colour) the
// result is bit-identical to the two-pass schedule.  With MEASURE the energy
// and magnetisation of the new state are reduced on the way (every bond has
// exactly one colour-1 end).
#include <type_traits>

#include "chunk.hpp"
#include "reduce.hpp"

namespace smc {

// Non-temporal 16-byte load and store: the whole-row kernel streams the old
// state in and the new one out once per launch (its halo rows excepted), and
// the two 256 MiB states of the L = 16384 lattice do not stay in the caches
// between launches; on the MI355X these accesses raised the sweep rate by 8 %.
__device__ __forceinline__ Chunk ld16nt(const int8_t* p) {
  typedef unsigned int v4u __attribute__((ext_vector_type(4)));
  const v4u v = __builtin_nontemporal_load(reinterpret_cast<const v4u*>(p));
  Chunk c;
  c.w[0] = v.x; c.w[1] = v.y; c.w[2] = v.z; c.w[3] = v.w;
  return c;
}
__device__ __forceinline__ void st16nt(int8_t* p, const uint32_t w[4]) {
  typedef unsigned int v4u __attribute__((ext_vector_type(4)));
  v4u v = {w[0], w[1], w[2], w[3]};
  __builtin_nontemporal_store(v, reinterpret_cast<v4u*>(p));
}

template <bool MEASURE>
__global__ __launch_bounds__(512) void ising_fused2d_kernel(const Geom g, const RngKey key,
                                                             const IsingTable table,
                                                             const uint32_t H,
                                                             const int8_t* __restrict__ A,
                                                             int8_t* __restrict__ B,
                                                             const uint32_t t,
                                                             Partial* __restrict__ parts) {
  __shared__ uint32_t edge[2][2][512];  // [step parity][old colour-1 row, new colour-0 row][lane]
  extern __shared__ uint16_t tie_slots[];  // kTieSlots entries per lane
  const int8_t* A0 = A;
  const int8_t* A1g = A + g.Nh;
  int8_t* B0 = B;
  int8_t* B1 = B + g.Nh;
  const uint32_t R = (uint32_t)g.R;
  const uint32_t L = (uint32_t)g.L;
  const uint32_t q = threadIdx.x;
  const uint32_t Q = blockDim.x;
  const uint32_t col = 16 * q;
  const uint32_t qn = q + 1 == Q ? 0u : q + 1;
  const uint32_t qp = q == 0 ? Q - 1 : q - 1;
  const TabRegs tab = tab_regs(table);
  const uint32_t band = xcd_remap(blockIdx.x, gridDim.x);
  const uint32_t y0 = band * H;  // a multiple of 4
  // offset of plane row y (0 <= y < 2L) for this lane's chunk column
  auto frow = [&](uint32_t y) -> uint32_t { return (y >= L ? y - L : y) * R + col; };

  // Rings: A1[y & 3] old colour-1 row y, A0[y & 1] old colour-0 row y,
  // N0[y & 3] new colour-0 row y.
  Chunk A1[4], A0r[2], N0[4];
  int64_t Esum = 0, Msum = 0;
  // colour-1 ties are queued (nothing in this launch reads the new colour 1);
  // colour-0 ties are resolved at once (the new colour 0 feeds colour 1)
  TieQueue tq;
  tq.slot = tie_slots + q;
  tq.stride = Q;
  tq.n = 0;
  tq.base = y0 * R + col;
  tq.R = R;
  tq.dE = 0;
  tq.dM = 0;

  // One step at row y = y0 + i (y & 3 == PH): new colour 0 at row y, then
  // (i >= 1) new colour 1 at row y - 1; then refill the dead ring slots with
  // the old colour-1 row y + 3 and the old colour-0 row y + 2.
  auto step = [&](auto phase, uint32_t y, bool store0, bool do1) {
    constexpr int PH = decltype(phase)::value;
    constexpr uint32_t p = PH & 1;    // parity of colour 0 at y = parity of colour 1 at y - 1
    constexpr uint32_t buf = PH & 1;  // LDS buffer of this step (steps alternate)
    const Chunk& a1m = A1[(PH + 3) & 3];
    const Chunk& a1c = A1[PH];
    const Chunk& a1p = A1[(PH + 1) & 3];
    const Chunk& a0c = A0r[PH & 1];
    const Chunk& n0m1 = N0[(PH + 3) & 3];
    const Chunk& n0m2 = N0[(PH + 2) & 3];
    edge[buf][0][q] = p ? a1c.w[0] : a1c.w[3];
    edge[buf][1][q] = p ? n0m1.w[0] : n0m1.w[3];
    __syncthreads();
    const uint32_t e_a = edge[buf][0][p ? qn : qp];
    const uint32_t e_n = edge[buf][1][p ? qn : qp];
    // new colour 0, row y
    const Chunk sha = p ? shift_next(a1c, e_a) : shift_prev(a1c, e_a);
    uint32_t kk[4];
    counts2d(a0c, a1c, sha, a1m, a1p, kk);
    const uint32_t off0 = frow(y);
    N0[PH] = update_chunk_now(tab, key, t, 0u, off0, a0c, kk);
    const Chunk& n0c = N0[PH];
    if (store0) {
      st16nt(B0 + off0, n0c.w);
      if (MEASURE) Msum += chunk_spin_sum(n0c);
    }
    // new colour 1, row y - 1
    if (do1) {
      const uint32_t off1 = frow(y + L - 1);
      const Chunk shn = p ? shift_next(n0m1, e_n) : shift_prev(n0m1, e_n);
      counts2d(a1m, n0m1, shn, n0m2, n0c, kk);
      const Chunk n1 = update_chunk_deferred<2>(tab, key, t, 1u, off1, y - 1 - y0, a1m, kk, tq, B1);
      st16nt(B1 + off1, n1.w);
      if (MEASURE) {
        uint32_t kn[4];
        counts2d(n1, n0m1, shn, n0m2, n0c, kn);
        Esum += -(int64_t)(16 * 4) + 2 * (int64_t)chunk_count_sum(kn);
        Msum += chunk_spin_sum(n1);
      }
    }
    A1[(PH + 3) & 3] = ld16nt(A1g + frow(y + 3));
    A0r[PH & 1] = ld16nt(A0 + frow(y + 2));
  };

  A1[2] = ld16nt(A1g + frow(y0 + L - 2));  // row y0 - 2 (frow takes rows < 2L)
  A1[3] = ld16nt(A1g + frow(y0 + L - 1));
  A1[0] = ld16nt(A1g + frow(y0));
  A1[1] = ld16nt(A1g + frow(y0 + 1));
  A0r[1] = ld16nt(A0 + frow(y0 + L - 1));
  A0r[0] = ld16nt(A0 + frow(y0));
  N0[0] = N0[1] = N0[2] = A0r[0];
  {
    // prologue: new colour-0 row y0 - 1 (odd row: parity 1), formed, not stored
    edge[1][0][q] = A1[3].w[0];
    __syncthreads();
    const Chunk sh = shift_next(A1[3], edge[1][0][qn]);
    uint32_t kk[4];
    counts2d(A0r[1], A1[3], sh, A1[2], A1[0], kk);
    N0[3] = update_chunk_now(tab, key, t, 0u, frow(y0 + L - 1), A0r[1], kk);
    A1[2] = ld16nt(A1g + frow(y0 + 2));
    A0r[1] = ld16nt(A0 + frow(y0 + 1));
  }
  for (uint32_t i = 0; i < H; i += 4) {
    const uint32_t y = y0 + i;
    step(std::integral_constant<int, 0>(), y, true, i >= 1);
    step(std::integral_constant<int, 1>(), y + 1, true, true);
    step(std::integral_constant<int, 2>(), y + 2, true, true);
    step(std::integral_constant<int, 3>(), y + 3, true, true);
  }
  // last step: new colour 0 at row y0 + H (formed, not stored), colour 1 at y0 + H - 1
  step(std::integral_constant<int, 0>(), y0 + H, false, true);
  tie_flush<2>(tq, tab, key, t, 1u, B1);
  Esum += tq.dE;
  Msum += tq.dM;
  if (MEASURE) block_partial_int(Esum, Msum, parts, blockIdx.x);
}

// Barrier-free variant: every wave works alone on a segment of 62 chunk
// columns of a band (lanes 1..62), with lanes 0 and 63 recomputing the new
// colour-0 chunks just outside the segment (not stored) so that the new
// colour-1 update of the segment's edge chunks has its in-row neighbours.  The
// old colour-1 edge words come from global memory (L2 hits, one row ahead in
// the pipeline), the new colour-0 edge words from the adjacent lane
// (ds_bpermute); no LDS exchange and no workgroup barrier.
template <bool MEASURE>
__global__ __launch_bounds__(256) void ising_fused2d_wave_kernel(
    const Geom g, const RngKey key, const IsingTable table, const uint32_t H, const uint32_t S,
    const uint32_t nbands, const int8_t* __restrict__ A, int8_t* __restrict__ B, const uint32_t t,
    Partial* __restrict__ parts) {
  __shared__ uint16_t tie_slots[kTieSlots * 256];
  const uint32_t lane = threadIdx.x & 63u;
  const uint32_t wave = xcd_remap(blockIdx.x, gridDim.x) * 4u + (threadIdx.x >> 6);
  const uint32_t band = wave / S;  // wave-uniform
  int64_t Esum = 0, Msum = 0;
  if (band < nbands) {
    const uint32_t seg = wave - band * S;
    const int8_t* A0 = A;
    const int8_t* A1g = A + g.Nh;
    int8_t* B0 = B;
    int8_t* B1 = B + g.Nh;
    const uint32_t R = (uint32_t)g.R;
    const uint32_t L = (uint32_t)g.L;
    const uint32_t Q = R / 16;
    const uint32_t xu = 62u * seg + lane;  // unwrapped chunk column + 1
    const uint32_t x = xu == 0 ? Q - 1 : (xu - 1 >= Q ? xu - 1 - Q : xu - 1);
    const bool store = lane >= 1 && lane <= 62 && xu - 1 < Q;
    const uint32_t col = 16 * x;
    const uint32_t xn = x + 1 == Q ? 0u : x + 1, xp = x == 0 ? Q - 1 : x - 1;
    const uint32_t edge_next = 16 * xn, edge_prev = 16 * xp + 12;  // parity 1 / parity 0
    const TabRegs tab = tab_regs(table);
    const uint32_t y0 = band * H;  // a multiple of 4
    auto frow = [&](uint32_t y) -> uint32_t { return (y >= L ? y - L : y) * R; };
    TieQueue tq;
    tq.slot = tie_slots + threadIdx.x;
    tq.stride = 256;
    tq.n = 0;
    tq.base = y0 * R + col;
    tq.R = R;
    tq.dE = 0;
    tq.dM = 0;
    // rings: A1[y & 3] old colour-1 row y with its edge word E1[y & 3] (for
    // the parity of row y), A0r[y & 1] old colour-0 row y, N0[y & 3] new colour 0
    Chunk A1[4], A0r[2], N0[4];
    uint32_t E1[4];
    auto edge1 = [&](uint32_t y, uint32_t par) -> uint32_t {
      return *reinterpret_cast<const uint32_t*>(A1g + frow(y) + (par ? edge_next : edge_prev));
    };
    auto step = [&](auto phase, uint32_t y, bool store0, bool do1) {
      constexpr int PH = decltype(phase)::value;
      constexpr uint32_t p = PH & 1;
      const Chunk& a1m = A1[(PH + 3) & 3];
      const Chunk& a1c = A1[PH];
      const Chunk& a1p = A1[(PH + 1) & 3];
      const Chunk& a0c = A0r[PH & 1];
      const Chunk& n0m1 = N0[(PH + 3) & 3];
      const Chunk& n0m2 = N0[(PH + 2) & 3];
      // new colour 0, row y
      const Chunk sha = p ? shift_next(a1c, E1[PH]) : shift_prev(a1c, E1[PH]);
      uint32_t kk[4];
      counts2d(a0c, a1c, sha, a1m, a1p, kk);
      const uint32_t off0 = frow(y) + col;
      N0[PH] = update_chunk_now(tab, key, t, 0u, off0, a0c, kk);
      const Chunk& n0c = N0[PH];
      if (store0 && store) {
        st16(B0 + off0, n0c.w);
        if (MEASURE) Msum += chunk_spin_sum(n0c);
      }
      // new colour 1, row y - 1: the in-row neighbour's new colour-0 edge word
      // comes from the adjacent lane
      const uint32_t en = p ? (uint32_t)__shfl_down((int)n0m1.w[0], 1, 64)
                            : (uint32_t)__shfl_up((int)n0m1.w[3], 1, 64);
      if (do1 && store) {
        const uint32_t off1 = frow(y + L - 1) + col;
        const Chunk shn = p ? shift_next(n0m1, en) : shift_prev(n0m1, en);
        counts2d(a1m, n0m1, shn, n0m2, n0c, kk);
        const Chunk n1 = update_chunk_deferred<2>(tab, key, t, 1u, off1, y - 1 - y0, a1m, kk, tq, B1);
        st16(B1 + off1, n1.w);
        if (MEASURE) {
          uint32_t kn[4];
          counts2d(n1, n0m1, shn, n0m2, n0c, kn);
          Esum += -(int64_t)(16 * 4) + 2 * (int64_t)chunk_count_sum(kn);
          Msum += chunk_spin_sum(n1);
        }
      }
      A1[(PH + 3) & 3] = ld16(A1g + frow(y + 3) + col);
      E1[(PH + 3) & 3] = edge1(y + 3, (PH + 3) & 1);
      A0r[PH & 1] = ld16(A0 + frow(y + 2) + col);
    };

    A1[2] = ld16(A1g + frow(y0 + L - 2) + col);  // row y0 - 2 (only its chunk is read)
    A1[3] = ld16(A1g + frow(y0 + L - 1) + col);
    E1[3] = edge1(y0 + L - 1, 1u);
    A1[0] = ld16(A1g + frow(y0) + col);
    E1[0] = edge1(y0, 0u);
    A1[1] = ld16(A1g + frow(y0 + 1) + col);
    E1[1] = edge1(y0 + 1, 1u);
    A0r[1] = ld16(A0 + frow(y0 + L - 1) + col);
    A0r[0] = ld16(A0 + frow(y0) + col);
    N0[0] = N0[1] = N0[2] = A0r[0];
    {
      // prologue: new colour-0 row y0 - 1 (odd row), formed, not stored
      const Chunk sh = shift_next(A1[3], E1[3]);
      uint32_t kk[4];
      counts2d(A0r[1], A1[3], sh, A1[2], A1[0], kk);
      N0[3] = update_chunk_now(tab, key, t, 0u, frow(y0 + L - 1) + col, A0r[1], kk);
      A1[2] = ld16(A1g + frow(y0 + 2) + col);
      E1[2] = edge1(y0 + 2, 0u);
      A0r[1] = ld16(A0 + frow(y0 + 1) + col);
    }
    for (uint32_t i = 0; i < H; i += 4) {
      const uint32_t y = y0 + i;
      step(std::integral_constant<int, 0>(), y, true, i >= 1);
      step(std::integral_constant<int, 1>(), y + 1, true, true);
      step(std::integral_constant<int, 2>(), y + 2, true, true);
      step(std::integral_constant<int, 3>(), y + 3, true, true);
    }
    step(std::integral_constant<int, 0>(), y0 + H, false, true);
    tie_flush<2>(tq, tab, key, t, 1u, B1);
    Esum += tq.dE;
    Msum += tq.dM;
  }
  if (MEASURE) block_partial_int(Esum, Msum, parts, blockIdx.x);
}

bool ising_fused_supported(const Geom& g, int J_kind, uint32_t H) {
  const uint32_t Q = (uint32_t)(g.R / 16);
  return g.d == 2 && J_kind == 0 && g.L % 32 == 0 && Q % 64 == 0 && Q <= 512 && H >= 4 &&
         H <= 64 && H % 4 == 0 && g.L % H == 0 && g.L / H >= 2;
}

// Rows per band: the largest divisor of L up to 64 leaving at least
// `min_blocks` workgroups.
uint32_t fused_rows_per_band(const Geom& g, uint32_t min_blocks) {
  uint32_t best = 4;
  for (uint32_t H = 4; H <= 64; H *= 2) {
    if (g.L % H) break;
    if ((uint32_t)g.L / H >= min_blocks) best = H;
  }
  return best;
}

hipError_t launch_ising_sweep_fused(const IsingLaunch& a, const int8_t* src, int8_t* dst,
                                    uint32_t t, void* partials, int64_t* nparts, hipStream_t st) {
  const uint32_t H = a.rows_per_band;
  const uint32_t Q = (uint32_t)(a.g.R / 16);
  if (a.variant == kVariantFusedWave) {
    const uint32_t S = (Q + 61) / 62;  // wave segments per band
    const uint32_t nbands = (uint32_t)a.g.L / H;
    const uint32_t waves = nbands * S;
    const dim3 grid((waves + 3) / 4), block(256);
    if (partials) {
      hipLaunchKernelGGL(ising_fused2d_wave_kernel<true>, grid, block, 0, st, a.g, a.key, a.tab, H,
                         S, nbands, src, dst, t, (Partial*)partials);
      if (nparts) *nparts = grid.x;
    } else {
      hipLaunchKernelGGL(ising_fused2d_wave_kernel<false>, grid, block, 0, st, a.g, a.key, a.tab, H,
                         S, nbands, src, dst, t, (Partial*)nullptr);
    }
    return hipGetLastError();
  }
  const dim3 grid((unsigned)(a.g.L / H)), block(Q);
  const size_t lds = (size_t)Q * kTieSlots * sizeof(uint16_t);
  if (partials) {
    hipLaunchKernelGGL(ising_fused2d_kernel<true>, grid, block, lds, st, a.g, a.key, a.tab, H, src,
                       dst, t, (Partial*)partials);
    if (nparts) *nparts = grid.x;
  } else {
    hipLaunchKernelGGL(ising_fused2d_kernel<false>, grid, block, lds, st, a.g, a.key, a.tab, H, src,
                       dst, t, (Partial*)nullptr);
  }
  return hipGetLastError();
}

}  // namespace smc
