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
}  // namespace rq
