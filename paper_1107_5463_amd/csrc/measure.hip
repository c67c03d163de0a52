// measure.hip -- energy and magnetisation (Eq. (1)), bond correlations,
// state validation.
//
// Every bond of the bipartite lattice (L even) has exactly one colour-1 end,
// so E = -sum over colour-1 sites i of sum_b J_b s_i . s_b (all 2d bonds of i),
// and every colour-0 site is the same-index partner (c = 0, j) of exactly one
// colour-1 site (c = 1, j): one pass over colour 1 gives both E and M.
// Partials: one per block, summed in int64 (Ising with integer couplings) or
// double (FP32 products promoted exactly), then reduced by a single block in a
// fixed order, so the result is deterministic.
#include "chunk.hpp"
#include "reduce.hpp"

#include <algorithm>
#include <map>
#include <mutex>

namespace smc {

// grid of the stand-alone measurements (each thread then takes several
// sites or chunks), so the finish kernel reads few partials
constexpr int64_t kMeasureBlocks = 2048;

// Ising, colour-1 sites j = gid, gid + stride, ... per thread, any L /
// coupling kind.
template <int D, int JK>
__global__ __launch_bounds__(256) void measure_ising_site(const Geom g, const int8_t* __restrict__ s,
                                                          const void* __restrict__ J, Partial* out) {
  const int64_t stride = (int64_t)gridDim.x * 256;
  Partial v{0, 0, 0.0, {0.0, 0.0, 0.0}};
  for (int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x; j < g.Nh; j += stride) {
    const int64_t Nh = g.Nh;
    const int8_t* s1 = s + Nh;
    const int8_t* s0 = s;
    int32_t x, y, z;
    site_coords(g, 1u, j, x, y, z);
    const int si = s1[j];
    int64_t e = 0;
    double ef = 0.0;
#pragma unroll
    for (int mu = 0; mu < D; ++mu) {
      int32_t xp = x, yp = y, zp = z, xm = x, ym = y, zm = z;
      if (mu == 0) { xp = wrap(x + 1, g.L); xm = wrap(x - 1, g.L); }
      if (mu == 1) { yp = wrap(y + 1, g.L); ym = wrap(y - 1, g.L); }
      if (mu == 2) { zp = wrap(z + 1, g.L); zm = wrap(z - 1, g.L); }
      const int64_t ip = plane_index(g, xp, yp, zp);
      const int64_t im = plane_index(g, xm, ym, zm);
      const int sp = s0[ip], sm = s0[im];
      if (JK == 2) {
        const float* Jf = (const float*)J;
        ef -= (double)Jf[((int64_t)mu * 2 + 1) * Nh + j] * (double)(si * sp);
        ef -= (double)Jf[((int64_t)mu * 2 + 0) * Nh + im] * (double)(si * sm);
      } else {
        int sgp = 1, sgm = 1;
        if (JK == 1) {
          const int8_t* Jb = (const int8_t*)J;
          sgp = Jb[((int64_t)mu * 2 + 1) * Nh + j];
          sgm = Jb[((int64_t)mu * 2 + 0) * Nh + im];
        }
        e -= sgp * si * sp + sgm * si * sm;
      }
    }
    v.Ei += e;
    v.E += ef;
    v.Mi += si + s0[j];
  }
  block_partial(v, out + 0);
}

// Ising, colour-1 chunks of 16 sites gid, gid + stride, ... per thread
// (L % 32 == 0, integer J).
template <int D, bool PM>
__global__ __launch_bounds__(256) void measure_ising_chunk(const Geom g, const int8_t* __restrict__ s,
                                                           const int8_t* __restrict__ J,
                                                           const FastDiv divQ, const FastDiv divL,
                                                           Partial* out) {
  const uint32_t stride = gridDim.x * 256u;
  Partial v{0, 0, 0.0, {0.0, 0.0, 0.0}};
  for (uint32_t gid = blockIdx.x * 256u + threadIdx.x; gid < (uint32_t)(g.Nh >> 4); gid += stride) {
    int64_t base;
    Chunk o, ctr;
    uint32_t kk[4];
    chunk_counts<D, PM>(g, s, J, divQ, divL, 1u, gid, base, o, ctr, kk);
    uint32_t unsat = 0, down = 0;
#pragma unroll
    for (int w = 0; w < 4; ++w) {
      unsat = __builtin_amdgcn_sad_u8(kk[w], 0u, unsat);
      down = __builtin_amdgcn_sad_u8(o.w[w] & kBit1, 0u, down);
      down = __builtin_amdgcn_sad_u8(ctr.w[w] & kBit1, 0u, down);
    }
    // each site: s_i h_i = 2d - 2k; M: 32 sites, down counted twice (bit value 2)
    v.Ei += -(int64_t)(16 * 2 * D) + 2 * (int64_t)unsat;
    v.Mi += 32 - (int64_t)down;
  }
  block_partial(v, out);
}

// Continuous spins: colour-1 sites j = gid, gid + stride, ... per thread
// (a bounded grid, so the finish kernel reads few partials).
template <int D, int N, int JK>
__global__ __launch_bounds__(256) void measure_cont_site(const Geom g, const float* __restrict__ s,
                                                         const void* __restrict__ J, const double J0,
                                                         Partial* out) {
  const int64_t stride = (int64_t)gridDim.x * 256;
  Partial v{0, 0, 0.0, {0.0, 0.0, 0.0}};
  for (int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x; j < g.Nh; j += stride) {
    const int64_t Nh = g.Nh, Nfull = 2 * Nh;
    const float* s1 = s + Nh;
    const float* s0 = s;
    int32_t x, y, z;
    site_coords(g, 1u, j, x, y, z);
    double si[3] = {0.0, 0.0, 0.0};
#pragma unroll
    for (int k = 0; k < N; ++k) si[k] = (double)s1[k * Nfull + j];
    double e = 0.0;
#pragma unroll
    for (int mu = 0; mu < D; ++mu) {
      int32_t xp = x, yp = y, zp = z, xm = x, ym = y, zm = z;
      if (mu == 0) { xp = wrap(x + 1, g.L); xm = wrap(x - 1, g.L); }
      if (mu == 1) { yp = wrap(y + 1, g.L); ym = wrap(y - 1, g.L); }
      if (mu == 2) { zp = wrap(z + 1, g.L); zm = wrap(z - 1, g.L); }
      const int64_t ip = plane_index(g, xp, yp, zp);
      const int64_t im = plane_index(g, xm, ym, zm);
      double dp = 0.0, dm = 0.0;
#pragma unroll
      for (int k = 0; k < N; ++k) {
        dp += si[k] * (double)s0[k * Nfull + ip];
        dm += si[k] * (double)s0[k * Nfull + im];
      }
      double jp = J0, jm = J0;
      if (JK == 1) {
        const int8_t* Jb = (const int8_t*)J;
        jp = J0 * Jb[((int64_t)mu * 2 + 1) * Nh + j];
        jm = J0 * Jb[((int64_t)mu * 2 + 0) * Nh + im];
      } else if (JK == 2) {
        const float* Jf = (const float*)J;
        jp = Jf[((int64_t)mu * 2 + 1) * Nh + j];
        jm = Jf[((int64_t)mu * 2 + 0) * Nh + im];
      }
      e -= jp * dp + jm * dm;
    }
    v.E += e;
#pragma unroll
    for (int k = 0; k < N; ++k) v.M[k] += si[k] + (double)s0[k * Nfull + j];
  }
  block_partial(v, out);
}

__global__ __launch_bounds__(256) void finish_kernel(const Partial* __restrict__ parts,
                                                     const int64_t nparts, const int ising,
                                                     const int int_couplings, const double J0,
                                                     const int64_t sweep,
                                                     ObsOut* __restrict__ obs) {
  // four independent running sums per thread (partials b, b + 256, b + 512,
  // b + 768 of each stride of 1024), so four loads are in flight instead of
  // one; they are combined in a fixed order, so the result stays deterministic
  auto add = [](Partial& a, const Partial& p) {
    a.Ei += p.Ei;
    a.Mi += p.Mi;
    a.E += p.E;
    for (int k = 0; k < 3; ++k) a.M[k] += p.M[k];
  };
  Partial acc[4];
  for (int u = 0; u < 4; ++u) acc[u] = Partial{0, 0, 0.0, {0.0, 0.0, 0.0}};
  int64_t b = threadIdx.x;
  if (ising && int_couplings) {
    // integer E and M only: 16 of a partial's 48 bytes (one CU reads them all)
    for (; b + 768 < nparts; b += 1024) {
      longlong2 p[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) p[u] = *reinterpret_cast<const longlong2*>(parts + b + 256 * u);
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        acc[u].Ei += p[u].x;
        acc[u].Mi += p[u].y;
      }
    }
    for (; b < nparts; b += 256) {
      const longlong2 p = *reinterpret_cast<const longlong2*>(parts + b);
      acc[0].Ei += p.x;
      acc[0].Mi += p.y;
    }
  } else {
    for (; b + 768 < nparts; b += 1024) {
      Partial p[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) p[u] = parts[b + 256 * u];
#pragma unroll
      for (int u = 0; u < 4; ++u) add(acc[u], p[u]);
    }
    for (; b < nparts; b += 256) add(acc[0], parts[b]);
  }
  Partial v = acc[0];
  for (int u = 1; u < 4; ++u) add(v, acc[u]);
  __shared__ Partial sh[256];
  sh[threadIdx.x] = v;
  __syncthreads();
  // pairwise tree in a fixed order (deterministic)
  for (unsigned s = 128; s > 0; s >>= 1) {
    if (threadIdx.x < s) {
      Partial& a = sh[threadIdx.x];
      const Partial& b = sh[threadIdx.x + s];
      a.Ei += b.Ei;
      a.Mi += b.Mi;
      a.E += b.E;
      for (int k = 0; k < 3; ++k) a.M[k] += b.M[k];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const Partial a = sh[0];
    ObsOut o;
    if (ising) {
      o.E_int = int_couplings ? a.Ei : 0;
      o.M_int = a.Mi;
      o.E = int_couplings ? J0 * (double)a.Ei : a.E;
      o.M[0] = (double)a.Mi;
      o.M[1] = 0.0;
      o.M[2] = 0.0;
      o.absM = fabs((double)a.Mi);
    } else {
      o.E_int = 0;
      o.M_int = 0;
      o.E = a.E;
      for (int k = 0; k < 3; ++k) o.M[k] = a.M[k];
      o.absM = sqrt(a.M[0] * a.M[0] + a.M[1] * a.M[1] + a.M[2] * a.M[2]);
    }
    o.sweep = sweep;
    *obs = o;
  }
}

int64_t measure_partials(const Geom& g) { return (g.Nh + 255) / 256; }

int64_t measure_partials_standalone(const Geom& g, bool packed) {
  if (packed) return (g.Nh / 32 + 255) / 256;
  return std::min<int64_t>((g.Nh + 255) / 256, kMeasureBlocks);
}

// Reduction partials of the allocation-free measurement (no handle, no
// workspace): a file-scope device array of which each GPU holds its own copy
// for the life of the process.  Host code must not pass `scratch` itself to
// a kernel (on the host it only names the symbol): measure_scratch() gives
// the device address.  Concurrent users on one GPU share it.
static __device__ __align__(256) Partial scratch[kMeasureScratchPartials];

hipError_t measure_scratch(void** ptr) {
  static std::mutex mu;
  static std::map<int, void*> addr;  // device -> its copy of `scratch`
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  std::lock_guard<std::mutex> lock(mu);
  auto it = addr.find(dev);
  if (it == addr.end()) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!p) return hipErrorInvalidSymbol;
    it = addr.emplace(dev, p).first;
  }
  *ptr = it->second;
  return hipSuccess;
}

template <int D>
static void launch_measure_d(const MeasureLaunch& a, const void* spins, Partial* parts,
                             int64_t& nparts, hipStream_t st) {
  const Geom& g = a.g;
  if (a.n == 1) {
    if (a.J_kind != 2 && g.L % 32 == 0) {
      const uint32_t nchunks = (uint32_t)(g.Nh >> 4);
      nparts = std::min<int64_t>((nchunks + 255) / 256, kMeasureBlocks);
      const FastDiv dq = make_fastdiv((uint32_t)(g.R / 16)), dl = make_fastdiv((uint32_t)g.L);
      if (a.J_kind == 1)
        hipLaunchKernelGGL((measure_ising_chunk<D, true>), dim3((unsigned)nparts), dim3(256), 0,
                           st, g, (const int8_t*)spins, (const int8_t*)a.J, dq, dl, parts);
      else
        hipLaunchKernelGGL((measure_ising_chunk<D, false>), dim3((unsigned)nparts), dim3(256), 0,
                           st, g, (const int8_t*)spins, (const int8_t*)a.J, dq, dl, parts);
      return;
    }
    nparts = std::min<int64_t>((g.Nh + 255) / 256, kMeasureBlocks);
    const dim3 grid((unsigned)nparts);
    if (a.J_kind == 0)
      hipLaunchKernelGGL((measure_ising_site<D, 0>), grid, dim3(256), 0, st, g,
                         (const int8_t*)spins, a.J, parts);
    else if (a.J_kind == 1)
      hipLaunchKernelGGL((measure_ising_site<D, 1>), grid, dim3(256), 0, st, g,
                         (const int8_t*)spins, a.J, parts);
    else
      hipLaunchKernelGGL((measure_ising_site<D, 2>), grid, dim3(256), 0, st, g,
                         (const int8_t*)spins, a.J, parts);
    return;
  }
  nparts = std::min<int64_t>((g.Nh + 255) / 256, kMeasureBlocks);
  const dim3 grid((unsigned)nparts);
  const float* sf = (const float*)spins;
#define SMC_MC(N, JK) \
  hipLaunchKernelGGL((measure_cont_site<D, N, JK>), grid, dim3(256), 0, st, g, sf, a.J, a.J0, parts)
  if (a.n == 2) {
    if (a.J_kind == 0) SMC_MC(2, 0); else if (a.J_kind == 1) SMC_MC(2, 1); else SMC_MC(2, 2);
  } else {
    if (a.J_kind == 0) SMC_MC(3, 0); else if (a.J_kind == 1) SMC_MC(3, 1); else SMC_MC(3, 2);
  }
#undef SMC_MC
}

hipError_t launch_measure(const MeasureLaunch& a, const void* spins, void* partials,
                          void* dev_obs, hipStream_t st) {
  Partial* parts = (Partial*)partials;
  int64_t nparts = 0;
  if (a.g.d == 2)
    launch_measure_d<2>(a, spins, parts, nparts, st);
  else
    launch_measure_d<3>(a, spins, parts, nparts, st);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  return launch_finish(a, parts, nparts, dev_obs, st);
}

hipError_t launch_finish(const MeasureLaunch& a, const void* partials, int64_t nparts,
                         void* dev_obs, hipStream_t st) {
  hipLaunchKernelGGL(finish_kernel, dim3(1), dim3(256), 0, st, (const Partial*)partials, nparts,
                     a.n == 1 ? 1 : 0, a.J_kind != 2 ? 1 : 0, a.J0, a.sweep, (ObsOut*)dev_obs);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Bond correlations acc[mu][c][j] += s_(c,j) . s_(c,j)+mu
// ---------------------------------------------------------------------------
template <int D, int N>
__global__ __launch_bounds__(256) void bond_acc_kernel(const Geom g, const void* __restrict__ spins,
                                                       void* __restrict__ acc) {
  const int64_t gid = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int64_t Nh = g.Nh, Nfull = 2 * Nh;
  if (gid >= Nfull) return;
  const uint32_t c = gid >= Nh ? 1u : 0u;
  const int64_t j = gid - (int64_t)c * Nh;
  int32_t x, y, z;
  site_coords(g, c, j, x, y, z);
#pragma unroll
  for (int mu = 0; mu < D; ++mu) {
    int32_t xp = x, yp = y, zp = z;
    if (mu == 0) xp = wrap(x + 1, g.L);
    if (mu == 1) yp = wrap(y + 1, g.L);
    if (mu == 2) zp = wrap(z + 1, g.L);
    const int64_t ip = (int64_t)(1 - c) * Nh + plane_index(g, xp, yp, zp);
    const int64_t slot = (int64_t)mu * Nfull + gid;
    if (N == 1) {
      const int8_t* s = (const int8_t*)spins;
      ((int64_t*)acc)[slot] += (int64_t)(s[gid] * s[ip]);
    } else {
      const float* s = (const float*)spins;
      double dp = 0.0;
#pragma unroll
      for (int k = 0; k < N; ++k) dp += (double)s[k * Nfull + gid] * (double)s[k * Nfull + ip];
      ((double*)acc)[slot] += dp;
    }
  }
}

hipError_t launch_bond_accumulate(const MeasureLaunch& a, const void* spins, void* acc,
                                  hipStream_t st) {
  const dim3 grid((unsigned)((2 * a.g.Nh + 255) / 256));
#define SMC_BA(D, N) hipLaunchKernelGGL((bond_acc_kernel<D, N>), grid, dim3(256), 0, st, a.g, spins, acc)
  if (a.g.d == 2) {
    if (a.n == 1) SMC_BA(2, 1); else if (a.n == 2) SMC_BA(2, 2); else SMC_BA(2, 3);
  } else {
    if (a.n == 1) SMC_BA(3, 1); else if (a.n == 2) SMC_BA(3, 2); else SMC_BA(3, 3);
  }
#undef SMC_BA
  return hipGetLastError();
}

// mean = accumulated sum / number of samples (a correctly rounded division)
__global__ __launch_bounds__(256) void bond_mean_kernel(const int64_t total, const int ising,
                                                        const void* __restrict__ acc,
                                                        const double count, double* __restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= total) return;
  const double v = ising ? (double)((const int64_t*)acc)[i] : ((const double*)acc)[i];
  out[i] = count > 0.0 ? v / count : 0.0;
}

hipError_t launch_bond_mean(const MeasureLaunch& a, const void* acc, int64_t samples, double* out,
                            hipStream_t st) {
  const int64_t total = 2 * a.g.Nh * a.g.d;
  hipLaunchKernelGGL(bond_mean_kernel, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, st,
                     total, a.n == 1 ? 1 : 0, acc, (double)samples, out);
  return hipGetLastError();
}

__global__ __launch_bounds__(256) void fill_zero_kernel(uint32_t* __restrict__ p, const int64_t nwords) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i < nwords) p[i] = 0u;
}

hipError_t launch_fill_zero(void* p, size_t bytes, hipStream_t st) {
  const int64_t nwords = (int64_t)(bytes / 4);
  if (nwords == 0) return hipSuccess;
  hipLaunchKernelGGL(fill_zero_kernel, dim3((unsigned)((nwords + 255) / 256)), dim3(256), 0, st,
                     (uint32_t*)p, nwords);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Validation: count out-of-range spins / couplings.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void validate_kernel(const Geom g, const int n, const int J_kind,
                                                       const void* __restrict__ spins,
                                                       const void* __restrict__ J,
                                                       uint32_t* __restrict__ count) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int64_t Nfull = 2 * g.Nh;
  if (i >= Nfull) return;
  uint32_t bad = 0;
  if (n == 1) {
    const int8_t v = ((const int8_t*)spins)[i];
    bad += (v != 1 && v != -1);
  } else {
    const float* s = (const float*)spins;
    float q = 0.0f;
    bool fin = true;
    for (int k = 0; k < n; ++k) {
      const float v = s[k * Nfull + i];
      fin = fin && isfinite(v);
      q += v * v;
    }
    bad += (!fin || fabsf(sqrtf(q) - 1.0f) >= 1e-4f);
  }
  for (int mu = 0; mu < g.d; ++mu) {
    if (J_kind == 1) {
      const int8_t v = ((const int8_t*)J)[mu * Nfull + i];
      bad += (v != 1 && v != -1);
    } else if (J_kind == 2) {
      bad += !isfinite(((const float*)J)[mu * Nfull + i]);
    }
  }
  if (bad) atomicAdd(count, bad);
}

hipError_t launch_validate(const MeasureLaunch& a, const void* spins, uint32_t* dev_count,
                           hipStream_t st) {
  const dim3 grid((unsigned)((2 * a.g.Nh + 255) / 256));
  hipLaunchKernelGGL(validate_kernel, grid, dim3(256), 0, st, a.g, a.n, a.J_kind, spins, a.J,
                     dev_count);
  return hipGetLastError();
}

}  // namespace smc
