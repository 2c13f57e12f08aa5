// Gaussian sketch matrices (the Omega of Section 4.1, transposed: G = Omega^T)
// from a counter-based generator, so that every entry can be drawn by any
// thread in any order.
//
// Philox4x64-10 (Salmon, Moraes, Dror, Shaw, SC'11): counter (c0..c3), key
// (k0, k1); each round multiplies c0 and c2 by the two Philox multipliers
// (full 128-bit products) and mixes the halves with c1, c3 and the key; the
// key is bumped by two Weyl constants between rounds.  Entry (r, g) of the
// block-i sketch uses counter (g, r, i, 0) and key (seed, 1).  Words 0 and 1
// give two uniforms u = ((w >> 12) + 1/2) 2^-52 in (0, 1) (exact in FP64),
// and Box-Muller gives z = sqrt(-2 ln u1) cos(2 pi u2).
#include "common.h"

namespace rq {

namespace {

constexpr uint64_t kM0 = 0xD2E7470EE14C6C93ull;
constexpr uint64_t kM1 = 0xCA5A826395121157ull;
constexpr uint64_t kW0 = 0x9E3779B97F4A7C15ull;
constexpr uint64_t kW1 = 0xBB67AE8584CAA73Bull;

__device__ __forceinline__ void philox4x64_10(uint64_t c[4], uint64_t k0, uint64_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r > 0) { k0 += kW0; k1 += kW1; }
    const uint64_t hi0 = __umul64hi(kM0, c[0]), lo0 = kM0 * c[0];
    const uint64_t hi1 = __umul64hi(kM1, c[2]), lo1 = kM1 * c[2];
    const uint64_t n0 = hi1 ^ c[1] ^ k0, n2 = hi0 ^ c[3] ^ k1;
    c[0] = n0; c[1] = lo1; c[2] = n2; c[3] = lo0;
  }
}

__global__ __launch_bounds__(256) void sketch_kernel(double *__restrict__ G, int64_t ldg, int64_t nsample,
                                                     int64_t nrows, int64_t row0, uint64_t block, uint64_t seed) {
  const int64_t total = nsample * nrows;
  for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
       idx += (int64_t)gridDim.x * blockDim.x) {
    const int64_t r = idx % nsample;
    const int64_t gl = idx / nsample;
    uint64_t c[4] = {(uint64_t)(row0 + gl), (uint64_t)r, block, 0ull};
    philox4x64_10(c, seed, 1ull);
    const double u1 = ((double)(c[0] >> 12) + 0.5) * 0x1p-52;
    const double u2 = ((double)(c[1] >> 12) + 0.5) * 0x1p-52;
    const double two_pi = 2.0 * 3.141592653589793;
    G[r + gl * ldg] = sqrt(-2.0 * log(u1)) * cos(two_pi * u2);
  }
}

}  // namespace

hipError_t launch_sketch(hipStream_t s, uint64_t seed, int64_t block, int64_t nsample, int64_t row0,
                         int64_t nrows, double *G, int64_t ldg, int max_wg) {
  const int64_t total = nsample * nrows;
  if (total <= 0) return hipSuccess;
  int64_t grid = (total + 255) / 256;
  if (grid > 65536) grid = 65536;
  if (max_wg > 0 && grid > max_wg) grid = max_wg;
  hipLaunchKernelGGL(sketch_kernel, dim3((unsigned)grid), dim3(256), 0, s, G, ldg, nsample, nrows, row0,
                     (uint64_t)block, seed);
  return hipGetLastError();
}

namespace {
__global__ void zero_u32_kernel(uint32_t *p, size_t n) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) p[i] = 0u;
}
}  // namespace

hipError_t launch_persistent(const void *func, unsigned nwg, unsigned threads, void **args, size_t lds,
                             hipStream_t s) {
  int dev = 0, ncu = 0, occ = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e == hipSuccess) e = hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
  if (e == hipSuccess) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, func, (int)threads, lds);
  if (e != hipSuccess) return e;
  if ((long)nwg <= (long)occ * (ncu / 2))
    return hipLaunchKernel(func, dim3(nwg), dim3(threads), args, lds, s);
  return hipLaunchCooperativeKernel(func, dim3(nwg), dim3(threads), args, (unsigned)lds, s);
}

hipError_t launch_zero_u32(hipStream_t s, void *p, size_t nwords) {
  if (nwords == 0) return hipSuccess;
  size_t grid = (nwords + 255) / 256;
  if (grid > 4096) grid = 4096;
  hipLaunchKernelGGL(zero_u32_kernel, dim3((unsigned)grid), dim3(256), 0, s, (uint32_t *)p, nwords);
  return hipGetLastError();
}

}  // namespace rq
