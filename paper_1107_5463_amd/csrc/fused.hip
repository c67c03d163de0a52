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
#include "chunk.hpp"
#include "reduce.hpp"

namespace smc {

template <bool MEASURE>
__global__ __launch_bounds__(1024) void ising_fused2d_kernel(const Geom g, const RngKey key,
                                                             const IsingTable tab,
                                                             const uint32_t H,
                                                             const int8_t* __restrict__ A,
                                                             int8_t* __restrict__ B,
                                                             const uint32_t t,
                                                             Partial* __restrict__ parts) {
  __shared__ uint32_t edge[2][2][1024];  // [buffer][old colour-1 row, new colour-0 row][lane]
  const uint32_t band = xcd_remap(blockIdx.x, gridDim.x);
  const uint32_t q = threadIdx.x;
  const uint32_t Q = blockDim.x;
  const uint32_t L = (uint32_t)g.L;
  const int64_t R = g.R, Nh = g.Nh;
  const int8_t* A0 = A;
  const int8_t* A1 = A + Nh;
  int8_t* B0 = B;
  int8_t* B1 = B + Nh;
  const int64_t col = 16 * (int64_t)q;
  const uint32_t qn = q + 1 == Q ? 0u : q + 1, qp = q == 0 ? Q - 1 : q - 1;
  const uint32_t y0 = band * H;
  auto wr = [&](int64_t y) -> uint32_t { return (uint32_t)(y < 0 ? y + L : (y >= L ? y - L : y)); };
  auto off = [&](uint32_t y) -> int64_t { return (int64_t)y * R + col; };
  auto publish = [&](uint32_t buf, uint32_t kind, uint32_t p, const Chunk& c) {
    edge[buf][kind][q] = p ? c.w[0] : c.w[3];
  };
  auto neighbour_edge = [&](uint32_t buf, uint32_t kind, uint32_t p) -> uint32_t {
    return edge[buf][kind][p ? qn : qp];
  };

  // prologue: new colour-0 row y0 - 1 (formed, not stored)
  const uint32_t ym1 = wr((int64_t)y0 - 1);
  Chunk a1m = ld16(A1 + off(wr((int64_t)y0 - 2)));
  Chunk a1c = ld16(A1 + off(ym1));
  Chunk a1p = ld16(A1 + off(y0));
  Chunk a0c = ld16(A0 + off(ym1));
  Chunk n0m1, n0m2;
  {
    const uint32_t p = ym1 & 1u;
    publish(1, 0, p, a1c);
    __syncthreads();
    const Chunk sh = p ? shift_next(a1c, neighbour_edge(1, 0, p)) : shift_prev(a1c, neighbour_edge(1, 0, p));
    uint32_t kk[4];
    counts2d(a0c, a1c, sh, a1m, a1p, kk);
    n0m1 = update_chunk(tab, key, t, 0u, (uint32_t)off(ym1), a0c, kk);
  }
  // slide the old colour-1 window to rows y0-1, y0, y0+1
  a1m = a1c;
  a1c = a1p;
  a1p = ld16(A1 + off(wr((int64_t)y0 + 1)));
  a0c = ld16(A0 + off(y0));
  n0m2 = n0m1;  // unused before it is overwritten

  int64_t Esum = 0, Msum = 0;
  for (uint32_t i = 0; i <= H; ++i) {
    const uint32_t y = wr((int64_t)y0 + i);
    const uint32_t p = y & 1u;  // parity of colour 0 at row y and of colour 1 at row y-1
    const uint32_t buf = i & 1u;
    // next step's rows, one ahead
    const Chunk a1n = ld16(A1 + off(wr((int64_t)y + 2)));
    const Chunk a0n = ld16(A0 + off(wr((int64_t)y + 1)));
    publish(buf, 0, p, a1c);
    publish(buf, 1, p, n0m1);
    __syncthreads();
    const uint32_t e_a = neighbour_edge(buf, 0, p);
    const uint32_t e_n = neighbour_edge(buf, 1, p);
    // new colour 0, row y
    const Chunk sha = p ? shift_next(a1c, e_a) : shift_prev(a1c, e_a);
    uint32_t kk[4];
    counts2d(a0c, a1c, sha, a1m, a1p, kk);
    const Chunk n0c = update_chunk(tab, key, t, 0u, (uint32_t)off(y), a0c, kk);
    if (i < H) {
      st16(B0 + off(y), n0c.w);
      if (MEASURE) Msum += chunk_spin_sum(n0c);
    }
    // new colour 1, row y - 1
    if (i >= 1) {
      const uint32_t yb = wr((int64_t)y - 1);
      const Chunk shn = p ? shift_next(n0m1, e_n) : shift_prev(n0m1, e_n);
      counts2d(a1m, n0m1, shn, n0m2, n0c, kk);
      const Chunk n1 = update_chunk(tab, key, t, 1u, (uint32_t)off(yb), a1m, kk);
      st16(B1 + off(yb), n1.w);
      if (MEASURE) {
        uint32_t kn[4];
        counts2d(n1, n0m1, shn, n0m2, n0c, kn);
        Esum += -(int64_t)(16 * 4) + 2 * (int64_t)chunk_count_sum(kn);
        Msum += chunk_spin_sum(n1);
      }
    }
    n0m2 = n0m1;
    n0m1 = n0c;
    a1m = a1c;
    a1c = a1p;
    a1p = a1n;
    a0c = a0n;
  }
  if (MEASURE) block_partial_int(Esum, Msum, parts, blockIdx.x);
}

bool ising_fused_supported(const Geom& g, int J_kind, uint32_t H) {
  const uint32_t Q = (uint32_t)(g.R / 16);
  return g.d == 2 && J_kind == 0 && g.L % 32 == 0 && Q % 64 == 0 && Q <= 1024 && H >= 1 &&
         g.L % H == 0 && g.L / H >= 2;
}

// Rows per band: the largest divisor of L up to 64 leaving at least
// `min_blocks` workgroups.
uint32_t fused_rows_per_band(const Geom& g, uint32_t min_blocks) {
  uint32_t best = 1;
  for (uint32_t H = 1; H <= 64; H *= 2) {
    if (g.L % H) break;
    if ((uint32_t)g.L / H >= min_blocks) best = H;
  }
  return best;
}

hipError_t launch_ising_sweep_fused(const IsingLaunch& a, const int8_t* src, int8_t* dst,
                                    uint32_t t, void* partials, int64_t* nparts, hipStream_t st) {
  const uint32_t H = a.rows_per_band;
  const uint32_t Q = (uint32_t)(a.g.R / 16);
  const dim3 grid((unsigned)(a.g.L / H)), block(Q);
  if (partials) {
    hipLaunchKernelGGL(ising_fused2d_kernel<true>, grid, block, 0, st, a.g, a.key, a.tab, H, src,
                       dst, t, (Partial*)partials);
    if (nparts) *nparts = grid.x;
  } else {
    hipLaunchKernelGGL(ising_fused2d_kernel<false>, grid, block, 0, st, a.g, a.key, a.tab, H, src,
                       dst, t, (Partial*)nullptr);
  }
  return hipGetLastError();
}

}  // namespace smc
