// Launchers of the data-movement kernels in misc.hip.
#pragma once
#include "common.h"

namespace rq {
hipError_t launch_copy2d(hipStream_t s, const double *src, int64_t lds, double *dst, int64_t ldd, int64_t rows,
                         int64_t cols);
hipError_t launch_transpose(hipStream_t s, const double *src, int64_t lds, double *dst, int64_t ldd, int64_t rows,
                            int64_t cols);
hipError_t launch_extract_v(hipStream_t s, const double *F, int64_t ldf, int64_t mi, int64_t bi, double *V,
                            int64_t ldv);
hipError_t launch_extract_r(hipStream_t s, const double *F, int64_t ldf, int64_t k, int64_t n, double *R,
                            int64_t ldr);
hipError_t launch_gather_cols(hipStream_t s, const double *src, int64_t lds, int64_t rows, int64_t scols,
                              const int32_t *idx, int64_t ncols, double *dst, int64_t ldd);
hipError_t launch_scatter_cols(hipStream_t s, const double *src, int64_t lds, int64_t rows, const int32_t *idx,
                               int64_t ncols, double *dst, int64_t ldd, int64_t dcols, bool add);
hipError_t launch_scatter_rows_t(hipStream_t s, const double *src, int64_t lds, int64_t k, const int32_t *idx,
                                 int64_t ncols, double *dst, int64_t ldd);
hipError_t launch_set_identity(hipStream_t s, double *E, int64_t lde, int64_t rows, int64_t cols);
hipError_t launch_iota(hipStream_t s, int32_t *p, int64_t n);
hipError_t launch_tri_inv_upper(hipStream_t s, const double *R, int64_t ldr, int64_t k, double *Ri, int64_t ldi);
// y <- 2^-e y (rows x cols, ld ldy) with e the exponent of max |y|, so that
// repeated products stay within FP32's range; word: one 32-bit device word of
// scratch.  The scaling is exact and changes no pivot decision.
hipError_t launch_normalise_pow2(hipStream_t s, float *y, int64_t ldy, int64_t rows, int64_t cols, unsigned *word);
hipError_t launch_copy_f32_f64(hipStream_t s, const float *src, int64_t lds, double *dst, int64_t ldd, int64_t rows,
                               int64_t cols);
hipError_t launch_copy_f64_f32(hipStream_t s, const double *src, int64_t lds, float *dst, int64_t ldd, int64_t rows,
                               int64_t cols);
hipError_t launch_copy2d_f32(hipStream_t s, const float *src, int64_t lds, float *dst, int64_t ldd, int64_t rows,
                             int64_t cols);
hipError_t launch_gather_cols_f32(hipStream_t s, const float *src, int64_t lds, int64_t rows, int64_t scols,
                                  const int32_t *idx, int64_t ncols, float *dst, int64_t ldd);
hipError_t launch_scatter_cols_f32(hipStream_t s, const float *src, int64_t lds, int64_t rows, const int32_t *idx,
                                   int64_t ncols, float *dst, int64_t ldd, int64_t dcols, bool add);

// overloads by element type, for code templated on the storage type
inline hipError_t launch_copy2d_t(hipStream_t s, const double *a, int64_t la, double *b, int64_t lb, int64_t r,
                                  int64_t c) { return launch_copy2d(s, a, la, b, lb, r, c); }
inline hipError_t launch_copy2d_t(hipStream_t s, const float *a, int64_t la, float *b, int64_t lb, int64_t r,
                                  int64_t c) { return launch_copy2d_f32(s, a, la, b, lb, r, c); }
inline hipError_t launch_to_f64(hipStream_t s, const double *a, int64_t la, double *b, int64_t lb, int64_t r,
                                int64_t c) { return launch_copy2d(s, a, la, b, lb, r, c); }
inline hipError_t launch_to_f64(hipStream_t s, const float *a, int64_t la, double *b, int64_t lb, int64_t r,
                                int64_t c) { return launch_copy_f32_f64(s, a, la, b, lb, r, c); }
inline hipError_t launch_from_f64(hipStream_t s, const double *a, int64_t la, double *b, int64_t lb, int64_t r,
                                  int64_t c) { return launch_copy2d(s, a, la, b, lb, r, c); }
inline hipError_t launch_from_f64(hipStream_t s, const double *a, int64_t la, float *b, int64_t lb, int64_t r,
                                  int64_t c) { return launch_copy_f64_f32(s, a, la, b, lb, r, c); }
inline hipError_t launch_gather_cols_t(hipStream_t s, const double *a, int64_t la, int64_t rows, int64_t sc,
                                       const int32_t *idx, int64_t nc, double *b, int64_t lb) {
  return launch_gather_cols(s, a, la, rows, sc, idx, nc, b, lb);
}
inline hipError_t launch_gather_cols_t(hipStream_t s, const float *a, int64_t la, int64_t rows, int64_t sc,
                                       const int32_t *idx, int64_t nc, float *b, int64_t lb) {
  return launch_gather_cols_f32(s, a, la, rows, sc, idx, nc, b, lb);
}
inline hipError_t launch_scatter_cols_t(hipStream_t s, const double *a, int64_t la, int64_t rows, const int32_t *idx,
                                        int64_t nc, double *b, int64_t lb, int64_t dc, bool add) {
  return launch_scatter_cols(s, a, la, rows, idx, nc, b, lb, dc, add);
}
inline hipError_t launch_scatter_cols_t(hipStream_t s, const float *a, int64_t la, int64_t rows, const int32_t *idx,
                                        int64_t nc, float *b, int64_t lb, int64_t dc, bool add) {
  return launch_scatter_cols_f32(s, a, la, rows, idx, nc, b, lb, dc, add);
}

// mixed-precision sketch (sample_bf16.hip)
size_t sample_bf16_part_floats(int64_t M, int64_t N, int64_t K);
// max_wg > 0: at most that many workgroups (beside a persistent kernel)
hipError_t launch_g_to_bf16(hipStream_t s, const double *G, int64_t ldg, int64_t nsample, int64_t nrows, void *Gb,
                            int64_t ldgb, int max_wg = 0);
hipError_t launch_sample_bf16(hipStream_t s, int64_t M, int64_t N, int64_t K, const void *Gb, int64_t ldgb,
                              const float *X, int64_t ldx, float *part, double *Y, int64_t ldy, int max_wg = 0);
}  // namespace rq
