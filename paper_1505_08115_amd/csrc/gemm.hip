// GEMM on CDNA4 matrix cores (FP64 and FP32): C = alpha op(A) op(B) + beta C,
// all column-major.  Used for the sketch Y = G X (Section 4.1, eq. defY), the
// WY products of the trailing update C <- C - V T^T V^T C (Section 5.1) and
// the products of the orthonormal pivoting variant and of the truncation.
//
// Design (gfx950, wave64):
//  * v_mfma_{f64,f32}_16x16x4: lane l supplies X[l%16][l/16] and Y[l/16][l%16]
//    of D = X Y (the output layouts are in Mfma<T> below).  The kernel feeds
//    X = op(B)^T and Y = op(A)^T, so that D = C^T and each lane holds 16
//    consecutive rows of a column of C: stores are contiguous segments.
//  * 256 threads = 4 waves in a 2 x 2 grid, each wave owns a (BM/2) x (BN/2)
//    block of 16 x 16 MFMA tiles; K advances by BK = 16 through two LDS
//    stages, the next K slab is prefetched into registers during the MFMAs.
//    The grid-capped FP64 trailing update uses 256 x 128 tiles by 512
//    threads (8 waves in 4 x 2, the same 64 x 64 block per wave), so that
//    one workgroup per CU still has two waves per SIMD.  (A lone wave issues
//    FP64 MFMAs at about half the SIMD's rate, 45 % measured with sixteen
//    independent accumulators; two waves reach 99 %.)
//  * C -= ... epilogues (beta != 0) load C in batches before storing, since
//    interleaved loads and stores of C serialise on the memory latency.
//  * Global loads are flattened so that consecutive lanes read consecutive
//    addresses along the contiguous dimension of each operand.
//  * Split-K: when the M x N tile grid is too small to fill 256 CUs, K is cut
//    into slabs whose partial products are summed in a fixed order by a
//    second kernel, so results do not depend on scheduling.
#include <algorithm>

#include "common.h"

namespace rq {

namespace {

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));

#ifndef RQ_GEMM_BK
#define RQ_GEMM_BK 16
#endif
#ifndef RQ_GEMM_PAD
#define RQ_GEMM_PAD 4
#endif
constexpr int kBK = RQ_GEMM_BK;
constexpr int kPad = RQ_GEMM_PAD;

// Matrix-core instruction per element type.  Both are 16 x 16 x 4 with lane l
// supplying X[l%16][l/16] and Y[l/16][l%16]; they differ in where D lands:
// FP64: D[i][j] in lane j + 16 (i%4), register i/4;
// FP32: D[i][j] in lane j + 16 (i/4), register i%4.
template <typename T> struct Mfma;
template <> struct Mfma<double> {
  typedef d4 acc_t;
  static __device__ __forceinline__ acc_t mma(double x, double y, acc_t c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(x, y, c, 0, 0, 0);
  }
  // row index i of D (a column of C in the transposed feed) held in register r
  static __device__ __forceinline__ int drow(int lane, int r) { return 4 * r + (lane >> 4); }
  static constexpr int dstep = 4;   // drow(lane, r) - drow(lane, 0) = dstep r
};
template <> struct Mfma<float> {
  typedef f4 acc_t;
  static __device__ __forceinline__ acc_t mma(float x, float y, acc_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(x, y, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int drow(int lane, int r) { return 4 * (lane >> 4) + r; }
  static constexpr int dstep = 1;
};

// One BM x BN tile of C by NT threads: waves in a WGM x (NT/64/WGM) grid, each
// owning a (BM/WGM) x (BN/WGN) block.  Each thread prefetches AE elements of
// the A slab and BE of the B slab; the elements of one thread sit at a fixed
// base plus a uniform stride (the flattened index t + NT q maps to (t mod L)
// and (t / L) + q NT/L along the contiguous dimension L), so no per-element
// addresses stay live.  Interior
// tiles on full K slabs load without bounds checks.  Two LDS stages: the
// next slab is written to the other stage while this one feeds the MFMAs,
// one barrier per K slab.
template <typename T, int BM, int BN, bool TA, bool TB, bool SPLIT, int NT = 256, int WGM = 2, bool AL = false>
__device__ __forceinline__ void gemm_tile(int64_t M, int64_t N, int64_t K, int64_t kchunk, const T *__restrict__ A,
                                          int64_t lda, const T *__restrict__ B, int64_t ldb, T *__restrict__ C,
                                          int64_t ldc, T alpha, T beta, T *__restrict__ partial, int64_t m0,
                                          int64_t n0, int64_t nb0) {
  typedef typename Mfma<T>::acc_t acc_t;
  constexpr int WGN = NT / 64 / WGM;
  constexpr int WBM = BM / WGM, WBN = BN / WGN;   // one wave's block
  constexpr int TM = WBM / 16, TN = WBN / 16;
  constexpr int AE = BM * kBK / NT, BE = BN * kBK / NT;
  // per-thread element coordinates: (first index, step per q) along rows/cols and k
  constexpr int A_QI = TA ? NT / kBK : 0, A_QK = TA ? 0 : NT / BM;
  constexpr int B_QJ = TB ? 0 : NT / kBK, B_QK = TB ? NT / BN : 0;
  __shared__ T As[2][kBK][BM + kPad];
  __shared__ T Bs[2][kBK][BN + kPad];

  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const int wm = wave % WGM, wn = wave / WGM;
  const int64_t kbeg = (int64_t)blockIdx.z * kchunk;
  const int64_t kend = min(K, kbeg + kchunk);
  // AL: M, N and K are multiples of the tile and of BK (the launcher checks),
  // so every tile is interior and every K slab full: no edge code is built
  const bool interior = AL || (m0 + BM <= M && n0 + BN <= N);

  const int a_i = TA ? t / kBK : t % BM, a_k = TA ? t % kBK : t / BM;
  const int b_j = TB ? t % BN : t / kBK, b_k = TB ? t / BN : t % kBK;
  const int64_t a_step = TA ? (int64_t)A_QI * lda : (int64_t)A_QK * lda;   // pointer step per q
  const int64_t b_step = TB ? (int64_t)B_QK * ldb : (int64_t)B_QJ * ldb;

  T ra[AE], rb[BE];
  auto load = [&](int64_t k0) {
    const T *pa = TA ? A + (k0 + a_k) + (m0 + a_i) * lda : A + (m0 + a_i) + (k0 + a_k) * lda;
    const T *pb = TB ? B + (nb0 + b_j) + (k0 + b_k) * ldb : B + (k0 + b_k) + (nb0 + b_j) * ldb;
    if (interior && (AL || k0 + kBK <= kend)) {
#pragma unroll
      for (int q = 0; q < AE; ++q) ra[q] = pa[q * a_step];
#pragma unroll
      for (int q = 0; q < BE; ++q) rb[q] = pb[q * b_step];
    } else {
#pragma unroll
      for (int q = 0; q < AE; ++q) {
        const int64_t gi = m0 + a_i + q * A_QI, gk = k0 + a_k + q * A_QK;
        ra[q] = (gi < M && gk < kend) ? pa[q * a_step] : T(0);
      }
#pragma unroll
      for (int q = 0; q < BE; ++q) {
        const int64_t gj = n0 + b_j + q * B_QJ, gk = k0 + b_k + q * B_QK;
        rb[q] = (gj < N && gk < kend) ? pb[q * b_step] : T(0);
      }
    }
  };
  auto stash = [&](int st) {
#pragma unroll
    for (int q = 0; q < AE; ++q) As[st][a_k + q * A_QK][a_i + q * A_QI] = ra[q];
#pragma unroll
    for (int q = 0; q < BE; ++q) Bs[st][b_k + q * B_QK][b_j + q * B_QJ] = rb[q];
  };

  acc_t acc[TM][TN];
#pragma unroll
  for (int a = 0; a < TM; ++a)
#pragma unroll
    for (int b = 0; b < TN; ++b) acc[a][b] = acc_t{T(0), T(0), T(0), T(0)};

  const int lr = lane & 15, lk = lane >> 4;
  int st = 0;
  if (kbeg < kend) {
    load(kbeg);
    stash(0);
  }
  __syncthreads();
  for (int64_t k0 = kbeg; k0 < kend; k0 += kBK) {
    const bool more = k0 + kBK < kend;
    if (more) load(k0 + kBK);
#pragma unroll
    for (int kk = 0; kk < kBK; kk += 4) {
      T xa[TN], yb[TM];
#pragma unroll
      for (int b = 0; b < TN; ++b) xa[b] = Bs[st][kk + lk][wn * WBN + b * 16 + lr];
#pragma unroll
      for (int a = 0; a < TM; ++a) yb[a] = As[st][kk + lk][wm * WBM + a * 16 + lr];
#pragma unroll
      for (int a = 0; a < TM; ++a)
#pragma unroll
        for (int b = 0; b < TN; ++b)
          acc[a][b] = Mfma<T>::mma(xa[b], yb[a], acc[a][b]);
    }
    if (more) stash(st ^ 1);
    __syncthreads();
    st ^= 1;
  }

  // Interior tiles with beta != 0 load a batch of C entries (two 16-column
  // blocks of a row block) before storing any of them, with no bounds
  // branches.  The compiler must assume that a store to C may alias a later
  // load of C, so loads interleaved with the stores (or sunk into per-entry
  // bounds branches) each wait for the store before them: one memory latency
  // per entry, 64 in a row per tile, a quarter of the trailing update's time.
  if (!SPLIT && beta != T(0) && interior) {
    constexpr int NB = TN >= 2 ? 2 : 1;
    // the lane's own row and column enter the base; the offsets below are
    // the same for every lane of the wave
    T *cbase = C + (m0 + wm * WBM + lr) + (n0 + wn * WBN + Mfma<T>::drow(lane, 0)) * ldc;
#pragma unroll
    for (int a = 0; a < TM; ++a)
#pragma unroll
      for (int b0 = 0; b0 < TN; b0 += NB) {
        T cv[NB][4];
#pragma unroll
        for (int b = 0; b < NB; ++b)
#pragma unroll
          for (int r = 0; r < 4; ++r)
            cv[b][r] = cbase[a * 16 + ((b0 + b) * 16 + Mfma<T>::dstep * r) * ldc];
#pragma unroll
        for (int b = 0; b < NB; ++b)
#pragma unroll
          for (int r = 0; r < 4; ++r)
            cbase[a * 16 + ((b0 + b) * 16 + Mfma<T>::dstep * r) * ldc] =
                alpha * acc[a][b0 + b][r] + beta * cv[b][r];
      }
    return;
  }
#pragma unroll
  for (int a = 0; a < TM; ++a) {
    const int64_t row = m0 + wm * WBM + a * 16 + lr;
    if (row >= M) continue;
#pragma unroll
    for (int b = 0; b < TN; ++b) {
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t col = n0 + wn * WBN + b * 16 + Mfma<T>::drow(lane, r);
        if (col >= N) continue;
        const T v = acc[a][b][r];
        if (SPLIT) {
          partial[(int64_t)blockIdx.z * M * N + row + col * M] = v;
        } else {
          T *cp = C + row + col * ldc;
          *cp = (beta == T(0)) ? alpha * v : alpha * v + beta * (*cp);
        }
      }
    }
  }
}

// One tile per workgroup (blockIdx.x, blockIdx.y).  TAG only gives two of
// the factorization's products kernel names of their own in profiles:
// kTagTrail for the trailing update C -= (V T^T) W, kTagW for W = V^T C.
template <typename T, int BM, int BN, bool TA, bool TB, bool SPLIT, int TAG = 0>
__global__ __launch_bounds__(256, 2) void gemm_kernel(int64_t M, int64_t N, int64_t K, int64_t kchunk,
                                                      const T *__restrict__ A, int64_t lda,
                                                      const T *__restrict__ B, int64_t ldb,
                                                      T *__restrict__ C, int64_t ldc, T alpha,
                                                      T beta, T *__restrict__ partial) {
  gemm_tile<T, BM, BN, TA, TB, SPLIT>(M, N, K, kchunk, A, lda, B, ldb, C, ldc, alpha, beta, partial,
                                      (int64_t)blockIdx.x * BM, (int64_t)blockIdx.y * BN, (int64_t)blockIdx.y * BN);
}

// A capped grid: each workgroup takes tiles blockIdx.x, blockIdx.x + gridDim.x,
// ... of the tile grid in column-major order (each tile's K loop ends with a
// barrier, so the LDS stages are free for the next tile).  A capped grid has
// about one workgroup per CU, so the register budget is that of one.
template <typename T, int BM, int BN, bool TA, bool TB, bool SPLIT, int TAG = 0, int NT = 256, int WGM = 2,
          bool AL = false>
__global__ __launch_bounds__(NT, 1) void gemm_kernel_capped(int64_t M, int64_t N, int64_t K, int64_t kchunk,
                                                            const T *__restrict__ A, int64_t lda,
                                                            const T *__restrict__ B, int64_t ldb,
                                                            T *__restrict__ C, int64_t ldc, T alpha,
                                                            T beta, T *__restrict__ partial,
                                                            const T *__restrict__ B2 = nullptr, int64_t ldb2 = 0,
                                                            int64_t n2 = 0) {
  const int64_t ntm = (M + BM - 1) / BM, ntiles = ntm * ((N + BN - 1) / BN);
  for (int64_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
    // columns below n2 (a multiple of BN) come from B2, the others from B
    const int64_t n0 = (tile / ntm) * BN;
    const bool first = n0 < n2;
    gemm_tile<T, BM, BN, TA, TB, SPLIT, NT, WGM, AL>(M, N, K, kchunk, A, lda, first ? B2 : B, first ? ldb2 : ldb, C,
                                                     ldc, alpha, beta, partial, (tile % ntm) * BM, n0,
                                                     first ? n0 : n0 - n2);
  }
}

// Short, wide products C (M x N) = alpha op(A) B + beta C with M <= 448 (the
// sketch Y = G X and W = V^T C): one workgroup holds all M rows of a
// 128-column slab of C, so the large operand B is read from HBM exactly once
// (a tiled kernel with 128-row tiles re-reads it once per row tile).  512
// threads = 8 waves, wave w owns columns 16w .. 16w+15 of the slab and all
// MT row blocks of 16; K is split over workgroups to fill the chip.  With TB
// the large operand is stored N x K (the power iteration's Y X^T): it is read
// with the column index fastest, so each row of a K slab is one coalesced
// 1 KiB segment.
constexpr int kRowsBN = 128;
constexpr int kTagTrail = 1, kTagW = 2;   // kernel-name tags (profiles only)
constexpr int kRowsThreads = 512;

template <typename T, int MT, bool TA, bool TB, bool SPLIT>
__device__ __forceinline__ void gemm_rows_slab(int64_t M, int64_t N, int64_t K, int64_t kchunk,
                                               const T *__restrict__ A, int64_t lda, const T *__restrict__ B,
                                               int64_t ldb, T *__restrict__ C, int64_t ldc, T alpha, T beta,
                                               T *__restrict__ partial, int64_t n0) {
  typedef typename Mfma<T>::acc_t acc_t;
  constexpr int MP = 16 * MT;                                   // padded rows
  constexpr int AE = (MP * kBK + kRowsThreads - 1) / kRowsThreads;
  constexpr int BE = kRowsBN * kBK / kRowsThreads;              // 4
  __shared__ T As[2][kBK][MP + kPad];
  __shared__ T Bs[2][kBK][kRowsBN + kPad];

  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const int64_t kbeg = (int64_t)blockIdx.y * kchunk;
  const int64_t kend = min(K, kbeg + kchunk);
  const bool interior = n0 + kRowsBN <= N;

  // B slab: k = t % 16, column j = t / 16 + 32 q (k fastest); with TB
  // column j = t % 128, k = t / 128 + 4 q (column fastest)
  constexpr int KQ = kRowsThreads / kRowsBN;   // 4 rows of the K slab per pass with TB
  const int b_k = TB ? t / kRowsBN : t % kBK, b_j = TB ? t % kRowsBN : t / kBK;
  T ra[AE], rb[BE];
  auto load = [&](int64_t k0) {
    const bool fullk = k0 + kBK <= kend;
    const T *pb = TB ? B + (n0 + b_j) + (k0 + b_k) * ldb : B + (k0 + b_k) + (n0 + b_j) * ldb;
#pragma unroll
    for (int q = 0; q < BE; ++q) {
      if constexpr (TB) {
        const bool okq = (interior && fullk) || (n0 + b_j < N && k0 + b_k + KQ * q < kend);
        rb[q] = okq ? pb[(int64_t)KQ * q * ldb] : T(0);
      } else {
        const bool okq = (interior && fullk) || (n0 + b_j + 32 * q < N && k0 + b_k < kend);
        rb[q] = okq ? pb[(int64_t)32 * q * ldb] : T(0);
      }
    }
#pragma unroll
    for (int q = 0; q < AE; ++q) {
      const int f = t + kRowsThreads * q;
      // TA: k fastest (A stored K x M); otherwise rows fastest (A stored M x K)
      const int r = TA ? f / kBK : f % MP, kk = TA ? f % kBK : f / MP;
      const int64_t gk = k0 + kk;
      const bool okq = f < MP * kBK && r < M && gk < kend;
      ra[q] = okq ? (TA ? A[gk + (int64_t)r * lda] : A[r + gk * lda]) : T(0);
    }
  };
  auto stash = [&](int st) {
#pragma unroll
    for (int q = 0; q < BE; ++q) {
      if constexpr (TB) Bs[st][b_k + KQ * q][b_j] = rb[q];
      else Bs[st][b_k][b_j + 32 * q] = rb[q];
    }
#pragma unroll
    for (int q = 0; q < AE; ++q) {
      const int f = t + kRowsThreads * q;
      const int r = TA ? f / kBK : f % MP, kk = TA ? f % kBK : f / MP;
      if (f < MP * kBK) As[st][kk][r] = ra[q];
    }
  };

  acc_t acc[MT];
#pragma unroll
  for (int a = 0; a < MT; ++a) acc[a] = acc_t{T(0), T(0), T(0), T(0)};
  const int lr = lane & 15, lk = lane >> 4;
  int st = 0;
  if (kbeg < kend) {
    load(kbeg);
    stash(0);
  }
  __syncthreads();
  for (int64_t k0 = kbeg; k0 < kend; k0 += kBK) {
    const bool more = k0 + kBK < kend;
    if (more) load(k0 + kBK);
#pragma unroll
    for (int kk = 0; kk < kBK; kk += 4) {
      const T xb = Bs[st][kk + lk][16 * wave + lr];
#pragma unroll
      for (int a = 0; a < MT; ++a) acc[a] = Mfma<T>::mma(xb, As[st][kk + lk][16 * a + lr], acc[a]);
    }
    if (more) stash(st ^ 1);
    __syncthreads();
    st ^= 1;
  }
  // D = C^T: lane holds row 16 a + lr of columns 16 wave + drow(lane, r)
#pragma unroll
  for (int a = 0; a < MT; ++a) {
    const int64_t row = 16 * a + lr;
    if (row >= M) continue;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int64_t col = n0 + 16 * wave + Mfma<T>::drow(lane, r);
      if (col >= N) continue;
      const T v = acc[a][r];
      if (SPLIT) {
        partial[(int64_t)blockIdx.y * M * N + row + col * M] = v;
      } else {
        T *cp = C + row + col * ldc;
        *cp = (beta == T(0)) ? alpha * v : alpha * v + beta * (*cp);
      }
    }
  }
}

template <typename T, int MT, bool TA, bool TB, bool SPLIT, int TAG = 0>
__global__ __launch_bounds__(kRowsThreads) void gemm_rows_kernel(int64_t M, int64_t N, int64_t K, int64_t kchunk,
                                                                 const T *__restrict__ A, int64_t lda,
                                                                 const T *__restrict__ B, int64_t ldb,
                                                                 T *__restrict__ C, int64_t ldc, T alpha, T beta,
                                                                 T *__restrict__ partial) {
  gemm_rows_slab<T, MT, TA, TB, SPLIT>(M, N, K, kchunk, A, lda, B, ldb, C, ldc, alpha, beta, partial,
                                       (int64_t)blockIdx.x * kRowsBN);
}

// A capped grid: slabs blockIdx.x, blockIdx.x + gridDim.x, ... of 128 columns.
template <typename T, int MT, bool TA, bool TB, bool SPLIT>
__global__ __launch_bounds__(kRowsThreads) void gemm_rows_kernel_capped(int64_t M, int64_t N, int64_t K,
                                                                        int64_t kchunk, const T *__restrict__ A,
                                                                        int64_t lda, const T *__restrict__ B,
                                                                        int64_t ldb, T *__restrict__ C, int64_t ldc,
                                                                        T alpha, T beta, T *__restrict__ partial) {
  const int64_t nslab = (N + kRowsBN - 1) / kRowsBN;
  for (int64_t sl = blockIdx.x; sl < nslab; sl += gridDim.x)
    gemm_rows_slab<T, MT, TA, TB, SPLIT>(M, N, K, kchunk, A, lda, B, ldb, C, ldc, alpha, beta, partial,
                                         sl * kRowsBN);
}

template <typename T, int TAG = 0>
__global__ __launch_bounds__(256) void reduce_partials_kernel(int64_t M, int64_t N, int splits,
                                                              const T *__restrict__ partial,
                                                              T *__restrict__ C, int64_t ldc,
                                                              T alpha, T beta) {
  const int64_t MN = M * N;
  for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < MN;
       idx += (int64_t)gridDim.x * blockDim.x) {
    // the partials are added in split order; eight loads are issued before
    // their adds so that they are in flight together (a loop of one load and
    // one add waits a memory latency per split)
    T s = T(0);
    int z = 0;
    for (; z + 8 <= splits; z += 8) {
      T v[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) v[u] = partial[(int64_t)(z + u) * MN + idx];
#pragma unroll
      for (int u = 0; u < 8; ++u) s += v[u];
    }
    if (z + 4 <= splits) {
      T v[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) v[u] = partial[(int64_t)(z + u) * MN + idx];
#pragma unroll
      for (int u = 0; u < 4; ++u) s += v[u];
      z += 4;
    }
    for (; z < splits; ++z) s += partial[(int64_t)z * MN + idx];
    const int64_t i = idx % M, j = idx / M;
    T *cp = C + i + j * ldc;
    *cp = (beta == T(0)) ? alpha * s : alpha * s + beta * (*cp);
  }
}

template <typename T, int BM, int BN, bool TA, bool TB, int TAG>
hipError_t launch_tiles_tag(hipStream_t s, const Gemm<T> &g, int splits, int64_t kchunk, T *partial) {
  const int64_t tiles = ((g.M + BM - 1) / BM) * ((g.N + BN - 1) / BN);
  if (g.max_wg > 0 && tiles * splits > g.max_wg) {
    dim3 cg((unsigned)std::max<int64_t>(1, g.max_wg / splits), 1, (unsigned)splits);
    if (splits > 1)
      hipLaunchKernelGGL((gemm_kernel_capped<T, BM, BN, TA, TB, true, TAG>), cg, dim3(256), 0, s, g.M, g.N, g.K,
                         kchunk, g.A, g.lda, g.B, g.ldb, g.C, g.ldc, g.alpha, g.beta, partial);
    else
      hipLaunchKernelGGL((gemm_kernel_capped<T, BM, BN, TA, TB, false, TAG>), cg, dim3(256), 0, s, g.M, g.N, g.K,
                         kchunk, g.A, g.lda, g.B, g.ldb, g.C, g.ldc, g.alpha, g.beta, partial);
    return hipGetLastError();
  }
  dim3 grid((unsigned)((g.M + BM - 1) / BM), (unsigned)((g.N + BN - 1) / BN), (unsigned)splits);
  if (splits > 1)
    hipLaunchKernelGGL((gemm_kernel<T, BM, BN, TA, TB, true, TAG>), grid, dim3(256), 0, s, g.M, g.N, g.K, kchunk,
                       g.A, g.lda, g.B, g.ldb, g.C, g.ldc, g.alpha, g.beta, partial);
  else
    hipLaunchKernelGGL((gemm_kernel<T, BM, BN, TA, TB, false, TAG>), grid, dim3(256), 0, s, g.M, g.N, g.K, kchunk,
                       g.A, g.lda, g.B, g.ldb, g.C, g.ldc, g.alpha, g.beta, partial);
  return hipGetLastError();
}

template <typename T, int BM, int BN, bool TA, bool TB>
hipError_t launch_tiles(hipStream_t s, const Gemm<T> &g, int splits, int64_t kchunk, T *partial) {
  if constexpr (!TA && !TB) {
    // a capped FP64 trailing update: 256 x 128 tiles by 8 waves (two per
    // SIMD, the same per-wave block as the uncapped kernel), so that one
    // workgroup per CU still hides latency
    if constexpr (BM == 128 && BN == 128 && sizeof(T) == 8)
      if (g.trailing && g.max_wg > 0 && splits == 1 && g.M >= 256) {
        const int64_t tiles = ((g.M + 255) / 256) * ((g.N + 127) / 128);
        dim3 cg((unsigned)std::min<int64_t>(tiles, g.max_wg));
        // shapes that are multiples of the tile (every block of a square
        // factorization with n a multiple of b = 256) get an instance without
        // edge code: the same tile loop built beside the edge code measured
        // 1.68 ms on an 8192 x 7936 x 256 update at 128 workgroups, 1.28 ms
        // without it
        if (g.M % 256 == 0 && g.N % 128 == 0 && g.K % kBK == 0 && kchunk == g.K)
          hipLaunchKernelGGL((gemm_kernel_capped<T, 256, 128, false, false, false, kTagTrail, 512, 4, true>), cg,
                             dim3(512), 0, s, g.M, g.N, g.K, kchunk, g.A, g.lda, g.B, g.ldb, g.C, g.ldc, g.alpha,
                             g.beta, partial);
        else
          hipLaunchKernelGGL((gemm_kernel_capped<T, 256, 128, false, false, false, kTagTrail, 512, 4>), cg, dim3(512),
                             0, s, g.M, g.N, g.K, kchunk, g.A, g.lda, g.B, g.ldb, g.C, g.ldc, g.alpha, g.beta,
                             partial);
        return hipGetLastError();
      }
    if (g.trailing) return launch_tiles_tag<T, BM, BN, false, false, kTagTrail>(s, g, splits, kchunk, partial);
    if (g.wprod) return launch_tiles_tag<T, BM, BN, false, false, kTagW>(s, g, splits, kchunk, partial);
  }
  return launch_tiles_tag<T, BM, BN, TA, TB, 0>(s, g, splits, kchunk, partial);
}

template <typename T, bool TA, bool TB>
hipError_t launch_shape(hipStream_t s, const Gemm<T> &g, int splits, int64_t kchunk, T *partial) {
  const bool sm = g.M <= 64, sn = g.N <= 64;
  if (sm && sn) return launch_tiles<T, 64, 64, TA, TB>(s, g, splits, kchunk, partial);
  if (sm) return launch_tiles<T, 64, 128, TA, TB>(s, g, splits, kchunk, partial);
  if (sn) return launch_tiles<T, 128, 64, TA, TB>(s, g, splits, kchunk, partial);
  return launch_tiles<T, 128, 128, TA, TB>(s, g, splits, kchunk, partial);
}

template <typename T>
void split_plan(const Gemm<T> &g, int *splits, int64_t *kchunk) {
  const int64_t bm = g.M <= 64 ? 64 : 128, bn = g.N <= 64 ? 64 : 128;
  const int64_t tiles = ((g.M + bm - 1) / bm) * ((g.N + bn - 1) / bn);
  int64_t sp = 1;
  if (tiles < 512 && g.K > 4 * kBK * 8) {
    sp = (512 + tiles - 1) / tiles;
    const int64_t maxsp = g.K / (kBK * 8);   // keep at least 128 of K per split
    if (sp > maxsp) sp = maxsp;
    if (sp > 64) sp = 64;
    if (sp < 1) sp = 1;
  }
  int64_t kc = (g.K + sp - 1) / sp;
  kc = ((kc + kBK - 1) / kBK) * kBK;
  if (kc < kBK) kc = kBK;
  sp = (g.K + kc - 1) / kc;
  if (sp < 1) sp = 1;
  *splits = (int)sp;
  *kchunk = kc;
}

// The all-rows kernel takes products with 64 < M <= 448 (288 in FP64), A
// untransposed, B either way, and a long K (the sketch G X, V^T C with V^T
// stored explicitly, the power iteration's Y X^T); everything else goes to
// the tiled kernel.  (A transposed A would be read as many short strided
// segments, which measured slower than the tiled kernel.)
template <typename T>
constexpr int rows_max_mt() { return sizeof(T) == 8 ? 18 : 28; }   // FP64 accumulators: 8 VGPRs per block

template <typename T>
bool use_rows(const Gemm<T> &g) {
  return !g.ta && g.M > 64 && g.M <= 16 * rows_max_mt<T>() && g.K >= 256 && g.N >= 256;
}

// One workgroup per CU (its LDS stages take most of the CU's 160 KiB), so the
// grid should fit one round on the 256 CUs of an MI355X: a second, partial
// round would cost nearly as much as the first.
constexpr int64_t kRowsSlots = 256;

template <typename T>
void rows_split_plan(const Gemm<T> &g, int *splits, int64_t *kchunk) {
  const int64_t tiles = (g.N + kRowsBN - 1) / kRowsBN;
  const int64_t slots = g.max_wg > 0 ? std::min<int64_t>(g.max_wg, kRowsSlots) : kRowsSlots;
  int64_t sp = slots / tiles;                                // tiles * splits <= one round
  // at least 64 of K per split: short products (the late blocks' W = V^T C,
  // a few 128-column slabs) then still spread over most of the CUs
  const int64_t maxsp = g.K / (kBK * 4);
  if (sp > maxsp) sp = maxsp;
  if (sp > 64) sp = 64;
  if (sp < 1) sp = 1;
  int64_t kc = (g.K + sp - 1) / sp;
  kc = ((kc + kBK - 1) / kBK) * kBK;
  if (kc < kBK) kc = kBK;
  sp = (g.K + kc - 1) / kc;
  *splits = (int)(sp < 1 ? 1 : sp);
  *kchunk = kc;
}

template <typename T, int MT, bool TA, bool TB, int TAG>
hipError_t launch_rows_tag(hipStream_t s, const Gemm<T> &g, int splits, int64_t kchunk, T *partial) {
  const int64_t slabs = (g.N + kRowsBN - 1) / kRowsBN;
  if (g.max_wg > 0 && slabs * splits > g.max_wg) {
    dim3 cg((unsigned)std::max<int64_t>(1, g.max_wg / splits), (unsigned)splits);
    if (splits > 1)
      hipLaunchKernelGGL((gemm_rows_kernel_capped<T, MT, TA, TB, true>), cg, dim3(kRowsThreads), 0, s, g.M, g.N, g.K,
                         kchunk, g.A, g.lda, g.B, g.ldb, g.C, g.ldc, g.alpha, g.beta, partial);
    else
      hipLaunchKernelGGL((gemm_rows_kernel_capped<T, MT, TA, TB, false>), cg, dim3(kRowsThreads), 0, s, g.M, g.N, g.K,
                         kchunk, g.A, g.lda, g.B, g.ldb, g.C, g.ldc, g.alpha, g.beta, partial);
    return hipGetLastError();
  }
  dim3 grid((unsigned)slabs, (unsigned)splits);
  if (splits > 1)
    hipLaunchKernelGGL((gemm_rows_kernel<T, MT, TA, TB, true, TAG>), grid, dim3(kRowsThreads), 0, s, g.M, g.N, g.K,
                       kchunk, g.A, g.lda, g.B, g.ldb, g.C, g.ldc, g.alpha, g.beta, partial);
  else
    hipLaunchKernelGGL((gemm_rows_kernel<T, MT, TA, TB, false, TAG>), grid, dim3(kRowsThreads), 0, s, g.M, g.N, g.K,
                       kchunk, g.A, g.lda, g.B, g.ldb, g.C, g.ldc, g.alpha, g.beta, partial);
  return hipGetLastError();
}

template <typename T, int MT, bool TA>
hipError_t launch_rows_mt(hipStream_t s, const Gemm<T> &g, int splits, int64_t kchunk, T *partial) {
  if (g.tb) return launch_rows_tag<T, MT, TA, true, 0>(s, g, splits, kchunk, partial);
  if (g.wprod) return launch_rows_tag<T, MT, TA, false, kTagW>(s, g, splits, kchunk, partial);
  return launch_rows_tag<T, MT, TA, false, 0>(s, g, splits, kchunk, partial);
}

template <typename T, bool TA>
hipError_t launch_rows(hipStream_t s, const Gemm<T> &g, int splits, int64_t kchunk, T *partial) {
  const int mt = (int)((g.M + 15) / 16);
  if (mt <= 8) return launch_rows_mt<T, 8, TA>(s, g, splits, kchunk, partial);
  if (mt <= 12) return launch_rows_mt<T, 12, TA>(s, g, splits, kchunk, partial);
  // M = 256 (W = V^T C at b = 256) gets its own instance: under MT = 18 two of
  // the 18 row blocks would be padding, an eighth of the MFMAs
  if (mt <= 16) return launch_rows_mt<T, 16, TA>(s, g, splits, kchunk, partial);
  if (mt <= 18 || rows_max_mt<T>() <= 18) return launch_rows_mt<T, 18, TA>(s, g, splits, kchunk, partial);
  if constexpr (rows_max_mt<T>() > 18) {
    if (mt <= 24) return launch_rows_mt<T, 24, TA>(s, g, splits, kchunk, partial);
    return launch_rows_mt<T, 28, TA>(s, g, splits, kchunk, partial);
  }
  return hipErrorInvalidValue;
}

// W = V^T C in FP64 with exactly 256 rows (b = 256), on the main stream: the
// tiled 256 x 128 form, whose 8 waves each own a 64 x 64 block (8 LDS reads
// per 16 MFMAs, against 17 when a wave owns 16 columns of all rows as in the
// all-rows kernel), with the all-rows kernel's K split and fixed-order sum;
// 0.64 -> 0.56 ms on 256 x 7936 x 8192.
template <typename T>
hipError_t launch_w256(hipStream_t s, const Gemm<T> &g, int splits, int64_t kchunk, T *partial) {
  if constexpr (sizeof(T) != 8) {
    return hipErrorInvalidValue;   // FP64 only
  } else {
    const dim3 grid((unsigned)((g.N + 127) / 128), 1, (unsigned)splits);
    const bool al = g.N % 128 == 0 && g.K % kBK == 0 && kchunk % kBK == 0;
#define RQ_W256(SP, AL)                                                                                              \
    hipLaunchKernelGGL((gemm_kernel_capped<T, 256, 128, false, false, SP, kTagW, 512, 4, AL>), grid, dim3(512), 0, \
                       s, g.M, g.N, g.K, kchunk, g.A, g.lda, g.B, g.ldb, g.C, g.ldc, g.alpha, g.beta, partial,   \
                       g.B2, g.ldb2, g.n2)
    if (splits > 1) {
      if (al) RQ_W256(true, true);
      else RQ_W256(true, false);
    } else {
      if (al) RQ_W256(false, true);
      else RQ_W256(false, false);
    }
#undef RQ_W256
    return hipGetLastError();
  }
}

}  // namespace

template <typename T>
int gemm_splits(const Gemm<T> &g) {
  int sp; int64_t kc;
  if (use_rows(g)) rows_split_plan(g, &sp, &kc);
  else split_plan(g, &sp, &kc);
  return sp;
}

template <typename T>
hipError_t launch_gemm(hipStream_t s, const Gemm<T> &g, T *partial) {
  if (g.M <= 0 || g.N <= 0) return hipSuccess;
  int splits; int64_t kchunk;
  const bool rows = use_rows(g);
  if (rows) rows_split_plan(g, &splits, &kchunk);
  else split_plan(g, &splits, &kchunk);
  if (g.K <= 0) splits = 1;
  hipError_t e;
  const bool w256 = sizeof(T) == 8 && rows && g.wprod && g.M == 256 && g.max_wg == 0;
  if (g.n2 != 0 && (!w256 || g.n2 < 0 || g.n2 % 128 != 0 || g.n2 > g.N || g.B2 == nullptr)) return hipErrorInvalidValue;
  if (w256) e = launch_w256(s, g, splits, kchunk, partial);
  else if (rows) e = launch_rows<T, false>(s, g, splits, kchunk, partial);
  else if (!g.ta && !g.tb) e = launch_shape<T, false, false>(s, g, splits, kchunk, partial);
  else if (g.ta && !g.tb) e = launch_shape<T, true, false>(s, g, splits, kchunk, partial);
  else if (!g.ta && g.tb) e = launch_shape<T, false, true>(s, g, splits, kchunk, partial);
  else e = launch_shape<T, true, true>(s, g, splits, kchunk, partial);
  if (e != hipSuccess || splits == 1) return e;
  const int64_t MN = g.M * g.N;
  int64_t grid = (MN + 255) / 256;
  if (grid > 8192) grid = 8192;
  if (g.max_wg > 0 && grid > g.max_wg) grid = g.max_wg;
  if (g.wprod)
    hipLaunchKernelGGL((reduce_partials_kernel<T, kTagW>), dim3((unsigned)grid), dim3(256), 0, s, g.M, g.N, splits,
                       partial, g.C, g.ldc, g.alpha, g.beta);
  else
    hipLaunchKernelGGL((reduce_partials_kernel<T, 0>), dim3((unsigned)grid), dim3(256), 0, s, g.M, g.N, splits,
                       partial, g.C, g.ldc, g.alpha, g.beta);
  return hipGetLastError();
}

template int gemm_splits<double>(const Gemm<double> &);
template int gemm_splits<float>(const Gemm<float> &);
template hipError_t launch_gemm<double>(hipStream_t, const Gemm<double> &, double *);
template hipError_t launch_gemm<float>(hipStream_t, const Gemm<float> &, float *);

}  // namespace rq
