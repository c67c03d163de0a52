// reduce.hpp -- per-block partial sums of the observables (internal).
#pragma once

#include "device.hpp"

namespace smc {

struct Partial {
  int64_t Ei;   // integer energy (uniform / +-1)
  int64_t Mi;   // integer magnetisation
  double E;     // double energy (FP32 couplings, continuous spins)
  double M[3];  // continuous magnetisation
};

struct ObsOut {  // layout of smc_obs
  int64_t E_int;
  int64_t M_int;
  double E;
  double M[3];
  double absM;
  int64_t sweep;
};
static_assert(sizeof(ObsOut) == 64, "ObsOut mirrors the 64-byte smc_obs");

template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  return v;
}

// Block of 256 threads: reduce each field, thread 0 writes the partial.
__device__ __forceinline__ void block_partial(Partial v, Partial* out) {
  __shared__ Partial sh[4];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  v.Ei = wave_sum(v.Ei);
  v.Mi = wave_sum(v.Mi);
  v.E = wave_sum(v.E);
#pragma unroll
  for (int k = 0; k < 3; ++k) v.M[k] = wave_sum(v.M[k]);
  if (lane == 0) sh[wv] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    Partial a = sh[0];
    for (int w = 1; w < 4; ++w) {
      a.Ei += sh[w].Ei;
      a.Mi += sh[w].Mi;
      a.E += sh[w].E;
      for (int k = 0; k < 3; ++k) a.M[k] += sh[w].M[k];
    }
    out[blockIdx.x] = a;
  }
}

// Any block of whole waves (up to 1024 threads): integer energy and
// magnetisation partial of this block into out[slot].
__device__ __forceinline__ void block_partial_int(int64_t E, int64_t M, Partial* out,
                                                  uint32_t slot) {
  __shared__ int64_t shE[16], shM[16];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  E = wave_sum(E);
  M = wave_sum(M);
  if (lane == 0) {
    shE[wv] = E;
    shM[wv] = M;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    const int nw = (int)((blockDim.x + 63) >> 6);
    Partial a{0, 0, 0.0, {0.0, 0.0, 0.0}};
    for (int w = 0; w < nw; ++w) {
      a.Ei += shE[w];
      a.Mi += shM[w];
    }
    out[slot] = a;
  }
}

}  // namespace smc
