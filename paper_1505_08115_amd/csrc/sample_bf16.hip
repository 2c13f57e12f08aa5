// Mixed-precision sketch (an addition to the paper): Y = G X with G rounded
// to BF16 and X read from FP32 storage and rounded to BF16 on the fly, products
// accumulated in FP32 on the matrix cores, and Y handed to the pivoted QR in
// FP64.  Choosing b pivots from Y tolerates this sampling error (Section 4.1
// only needs the linear dependencies among Y's columns to resemble A's).
//
// v_mfma_f32_16x16x32_bf16: lane l supplies 8 consecutive k of row l%16 of the
// first operand and of column l%16 of the second (k = 8 (l/16) .. +7); the
// result D[i][j] lands in lane j + 16 (i/4), register i%4.  The kernel feeds
// the first operand from X^T (so each lane reads 8 consecutive FP32 of one
// column of X, 32 contiguous bytes) and the second from G^T (8 consecutive
// BF16 of one sample row, staged in LDS), giving D = Y^T: every lane holds
// consecutive sample rows of one column of Y.
//
// A workgroup owns all M = b + p sample rows and 128 columns of X, so X is
// read from HBM exactly once; K is split over workgroups to fill the chip,
// FP32 partial products are summed in FP64 in a fixed order.
#include <hip/hip_bf16.h>

#include <algorithm>

#include "common.h"

namespace rq {

namespace {

typedef float f4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));

constexpr int kKS = 32;          // K per MFMA step
constexpr int kBN = 128;         // columns of X per workgroup
constexpr int kMaxMT = 32;       // up to 512 sample rows
constexpr int kLdg = kKS + 8;    // padded LDS row of the G slab (bf16 elements)

template <int MT>
__global__ __launch_bounds__(256) void sample_bf16_kernel(int64_t M, int64_t N, int64_t K, int64_t kchunk,
                                                          const __bf16 *__restrict__ Gb, int64_t ldgb,
                                                          const float *__restrict__ X, int64_t ldx,
                                                          float *__restrict__ part) {
  __shared__ __bf16 Gs[MT * 16][kLdg];
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const int64_t n0 = (int64_t)blockIdx.x * kBN;
  const int64_t kbeg = (int64_t)blockIdx.y * kchunk;
  const int64_t kend = min(K, kbeg + kchunk);
  const int lr = lane & 15, lq = lane >> 4;

  f4 acc[2][MT];
#pragma unroll
  for (int b = 0; b < 2; ++b)
#pragma unroll
    for (int a = 0; a < MT; ++a) acc[b][a] = f4{0.f, 0.f, 0.f, 0.f};

  for (int64_t k0 = kbeg; k0 < kend; k0 += kKS) {
    __syncthreads();
    // stage G(0:M, k0:k0+32) as BF16 rows (8 elements per thread-chunk)
    for (int idx = t; idx < MT * 16 * (kKS / 8); idx += 256) {
      const int m = idx / (kKS / 8), c8 = (idx % (kKS / 8)) * 8;
      bf8 v;
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        const int64_t k = k0 + c8 + q;
        v[q] = (m < M && k < kend) ? Gb[k + (int64_t)m * ldgb] : (__bf16)0.0f;
      }
      *reinterpret_cast<bf8 *>(&Gs[m][c8]) = v;
    }
    __syncthreads();
    // X^T fragments: 8 consecutive k of one column per lane, rounded to BF16
    bf8 xf[2];
#pragma unroll
    for (int b = 0; b < 2; ++b) {
      const int64_t n = n0 + (wave * 2 + b) * 16 + lr;
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        const int64_t k = k0 + lq * 8 + q;
        xf[b][q] = (n < N && k < kend) ? (__bf16)X[k + n * ldx] : (__bf16)0.0f;
      }
    }
#pragma unroll
    for (int a = 0; a < MT; ++a) {
      const bf8 gf = *reinterpret_cast<const bf8 *>(&Gs[a * 16 + lr][lq * 8]);
#pragma unroll
      for (int b = 0; b < 2; ++b) acc[b][a] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(xf[b], gf, acc[b][a], 0, 0, 0);
    }
  }
  // D = Y^T: lane holds Y(m = a*16 + lr, n = tile + 4 lq + r)
  float *out = part + (int64_t)blockIdx.y * M * N;
#pragma unroll
  for (int b = 0; b < 2; ++b) {
#pragma unroll
    for (int a = 0; a < MT; ++a) {
      const int64_t m = a * 16 + lr;
      if (m >= M) continue;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t n = n0 + (wave * 2 + b) * 16 + lq * 4 + r;
        if (n < N) out[m + n * M] = acc[b][a][r];
      }
    }
  }
}

__global__ __launch_bounds__(256) void reduce_to_f64_kernel(int64_t M, int64_t N, int splits,
                                                            const float *__restrict__ part, double *__restrict__ Y,
                                                            int64_t ldy) {
  const int64_t MN = M * N;
  for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < MN;
       idx += (int64_t)gridDim.x * blockDim.x) {
    double s = 0.0;
    for (int z = 0; z < splits; ++z) s += (double)part[(int64_t)z * MN + idx];
    Y[idx % M + (idx / M) * ldy] = s;
  }
}

// G (FP64, nsample x nrows, ld ldg, sample index fastest) -> BF16 with the
// row index of X fastest (ld ldgb): Gb[g + r*ldgb] = bf16(G[r + g*ldg]).
__global__ __launch_bounds__(256) void g_to_bf16_kernel(const double *__restrict__ G, int64_t ldg, int64_t nsample,
                                                        int64_t nrows, __bf16 *__restrict__ Gb, int64_t ldgb) {
  const int64_t total = nsample * nrows;
  for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
       idx += (int64_t)gridDim.x * blockDim.x) {
    const int64_t g = idx % nrows, r = idx / nrows;
    Gb[g + r * ldgb] = (__bf16)(float)G[r + g * ldg];
  }
}

// K is split so that the grid fills `slots` workgroups (the 256 CUs, or the
// cap of a product that runs beside a persistent kernel)
void plan(int64_t M, int64_t N, int64_t K, int *splits, int64_t *kchunk, int slots = 256) {
  const int64_t tiles = (N + kBN - 1) / kBN;
  int64_t sp = (slots + tiles - 1) / tiles;
  if (slots < 256) sp = std::max<int64_t>(1, slots / tiles);   // stay within the cap
  const int64_t maxsp = std::max<int64_t>(1, K / (kKS * 8));
  if (sp > maxsp) sp = maxsp;
  if (sp > 64) sp = 64;
  int64_t kc = (K + sp - 1) / sp;
  kc = ((kc + kKS - 1) / kKS) * kKS;
  if (kc < kKS) kc = kKS;
  *splits = (int)((K + kc - 1) / kc);
  if (*splits < 1) *splits = 1;
  *kchunk = kc;
  (void)M;
}

template <int MT>
void launch_mt(hipStream_t s, dim3 grid, int64_t M, int64_t N, int64_t K, int64_t kc, const __bf16 *Gb, int64_t ldgb,
               const float *X, int64_t ldx, float *part) {
  hipLaunchKernelGGL((sample_bf16_kernel<MT>), grid, dim3(256), 0, s, M, N, K, kc, Gb, ldgb, X, ldx, part);
}

}  // namespace

size_t sample_bf16_part_floats(int64_t M, int64_t N, int64_t K) {
  int sp; int64_t kc;
  plan(M, N, K, &sp, &kc);
  return (size_t)sp * M * N;
}

hipError_t launch_g_to_bf16(hipStream_t s, const double *G, int64_t ldg, int64_t nsample, int64_t nrows, void *Gb,
                            int64_t ldgb, int max_wg) {
  const int64_t total = nsample * nrows;
  if (total <= 0) return hipSuccess;
  int64_t grid = (total + 255) / 256;
  if (grid > 16384) grid = 16384;
  if (max_wg > 0 && grid > max_wg) grid = max_wg;
  hipLaunchKernelGGL(g_to_bf16_kernel, dim3((unsigned)grid), dim3(256), 0, s, G, ldg, nsample, nrows,
                     static_cast<__bf16 *>(Gb), ldgb);
  return hipGetLastError();
}

hipError_t launch_sample_bf16(hipStream_t s, int64_t M, int64_t N, int64_t K, const void *Gb, int64_t ldgb,
                              const float *X, int64_t ldx, float *part, double *Y, int64_t ldy, int max_wg) {
  if (M <= 0 || N <= 0) return hipSuccess;
  if (M > kMaxMT * 16) return hipErrorInvalidValue;
  int sp; int64_t kc;
  plan(M, N, K, &sp, &kc, max_wg > 0 && max_wg < 256 ? max_wg : 256);
  dim3 grid((unsigned)((N + kBN - 1) / kBN), (unsigned)sp);
  const __bf16 *G = static_cast<const __bf16 *>(Gb);
  const int mt = (int)((M + 15) / 16);
  if (mt <= 4) launch_mt<4>(s, grid, M, N, K, kc, G, ldgb, X, ldx, part);
  else if (mt <= 8) launch_mt<8>(s, grid, M, N, K, kc, G, ldgb, X, ldx, part);
  else if (mt <= 12) launch_mt<12>(s, grid, M, N, K, kc, G, ldgb, X, ldx, part);
  else if (mt <= 17) launch_mt<17>(s, grid, M, N, K, kc, G, ldgb, X, ldx, part);
  else if (mt <= 24) launch_mt<24>(s, grid, M, N, K, kc, G, ldgb, X, ldx, part);
  else launch_mt<32>(s, grid, M, N, K, kc, G, ldgb, X, ldx, part);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int64_t MN = M * N;
  int64_t g2 = (MN + 255) / 256;
  if (g2 > 8192) g2 = 8192;
  if (max_wg > 0 && g2 > max_wg) g2 = max_wg;
  hipLaunchKernelGGL(reduce_to_f64_kernel, dim3((unsigned)g2), dim3(256), 0, s, M, N, sp, part, Y, ldy);
  return hipGetLastError();
}

}  // namespace rq
