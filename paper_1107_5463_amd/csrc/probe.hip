// probe.hip -- measurement probes for the ceilings the sweep kernels are
// compared with (not part of any sweep):
//   * Philox4x32-10 alone: blocks per second when every lane draws blocks
//     back to back, the random-number cost that bounds every Ising kernel;
//   * integer VALU issue: eight independent chains of 32-bit xor / add /
//     shift / byte-permute per lane (the operations of the SWAR and
//     bit-sliced decisions) with nothing else to wait on, so the issued
//     instruction rate is the practical VALU ceiling of such code.
// Each lane folds its results into one word written to `out`, so no work is
// dead.
#include "chunk.hpp"

namespace smc {

__global__ __launch_bounds__(256) void probe_philox_kernel(const uint32_t blocks, const uint32_t k0,
                                                           const uint32_t k1,
                                                           uint32_t* __restrict__ out) {
  const uint32_t lane = blockIdx.x * 256 + threadIdx.x;
  uint32_t acc = 0;
  for (uint32_t b = 0; b < blocks; ++b) {
    const Rand4 r = philox(lane, b, 0u, 0u, k0, k1);
    acc ^= __builtin_amdgcn_bitop3_b32(r.w[0], r.w[1], r.w[2], 0x96) + r.w[3];
  }
  out[lane] = acc;
}

__global__ __launch_bounds__(256) void probe_valu_kernel(const uint32_t iters, const uint32_t seed,
                                                         uint32_t* __restrict__ out) {
  const uint32_t lane = blockIdx.x * 256 + threadIdx.x;
  uint32_t a[8];
#pragma unroll
  for (int k = 0; k < 8; ++k) a[k] = seed ^ (lane * 0x9E3779B9u + 0x85EBCA6Bu * (uint32_t)k);
  for (uint32_t i = 0; i < iters; ++i) {
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      const uint32_t x = __builtin_amdgcn_bitop3_b32(a[k], a[(k + 1) & 7], i, 0x96);
      const uint32_t y = __builtin_amdgcn_perm(x, a[(k + 2) & 7], 0x05040100u | (i & 0x03030303u));
      a[k] = y + (x >> 3);
    }
  }
  uint32_t r = 0;
#pragma unroll
  for (int k = 0; k < 8; ++k) r ^= a[k];
  out[lane] = r;
}

hipError_t launch_probe(int kind, uint32_t n_lanes, uint32_t reps, uint32_t* out, hipStream_t st) {
  const dim3 grid(n_lanes / 256), block(256);
  if (kind == 0)
    hipLaunchKernelGGL(probe_philox_kernel, grid, block, 0, st, reps, 0x1234567u, 0x89ABCDEu, out);
  else
    hipLaunchKernelGGL(probe_valu_kernel, grid, block, 0, st, reps, 0x2545F491u, out);
  return hipGetLastError();
}

}  // namespace smc
