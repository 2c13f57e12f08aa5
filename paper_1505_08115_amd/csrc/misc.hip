// Small data-movement kernels around the factorization: copies, transposes,
// extraction of the explicit Householder vectors V and of R from the factored
// matrix, column gathers/scatters for the permutation P, and the inverse of
// an upper-triangular block.  All are bandwidth-bound element maps with
// coalesced accesses along the column-major leading dimension.
#include "common.h"
#include "misc.h"

namespace rq {

namespace {

inline unsigned grid_for(int64_t n) {
  int64_t g = (n + 255) / 256;
  if (g > 16384) g = 16384;
  if (g < 1) g = 1;
  return (unsigned)g;
}

#define GRID_STRIDE(i, n) for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < (n); i += (int64_t)gridDim.x * blockDim.x)

__global__ void copy2d_kernel(const double *__restrict__ s, int64_t lds, double *__restrict__ d, int64_t ldd,
                              int64_t rows, int64_t cols) {
  GRID_STRIDE(i, rows * cols) {
    const int64_t r = i % rows, c = i / rows;
    d[r + c * ldd] = s[r + c * lds];
  }
}

__global__ void transpose_kernel(const double *__restrict__ s, int64_t lds, double *__restrict__ d, int64_t ldd,
                                 int64_t rows, int64_t cols) {
  // d (cols x rows) = s^T; reads coalesced along rows of s
  GRID_STRIDE(i, rows * cols) {
    const int64_t r = i % rows, c = i / rows;
    d[c + r * ldd] = s[r + c * lds];
  }
}

__global__ void extract_v_kernel(const double *__restrict__ F, int64_t ldf, int64_t mi, int64_t bi,
                                 double *__restrict__ V, int64_t ldv) {
  GRID_STRIDE(i, mi * bi) {
    const int64_t r = i % mi, c = i / mi;
    V[r + c * ldv] = r > c ? F[r + c * ldf] : (r == c ? 1.0 : 0.0);
  }
}

__global__ void extract_r_kernel(const double *__restrict__ F, int64_t ldf, int64_t k, int64_t n,
                                 double *__restrict__ R, int64_t ldr) {
  GRID_STRIDE(i, k * n) {
    const int64_t r = i % k, c = i / k;
    R[r + c * ldr] = r <= c ? F[r + c * ldf] : 0.0;
  }
}

__global__ void gather_cols_kernel(const double *__restrict__ s, int64_t lds, int64_t rows, int64_t scols,
                                   const int32_t *__restrict__ idx, int64_t ncols, double *__restrict__ d,
                                   int64_t ldd) {
  GRID_STRIDE(i, rows * ncols) {
    const int64_t r = i % rows, c = i / rows;
    const int64_t src = idx[c];
    // an index outside the source (not a permutation) yields NaN, never a stray read
    d[r + c * ldd] = (src >= 0 && src < scols) ? s[r + src * lds] : __builtin_nan("");
  }
}

__global__ void scatter_cols_kernel(const double *__restrict__ s, int64_t lds, int64_t rows, const int32_t *__restrict__ idx,
                                    int64_t ncols, double *__restrict__ d, int64_t ldd, int64_t dcols, int add) {
  GRID_STRIDE(i, rows * ncols) {
    const int64_t r = i % rows, c = i / rows;
    const int64_t dc = idx[c];
    if (dc < 0 || dc >= dcols) continue;
    double *p = d + r + dc * ldd;
    *p = add ? *p + s[r + c * lds] : s[r + c * lds];
  }
}

__global__ void scatter_rows_t_kernel(const double *__restrict__ s, int64_t lds, int64_t k, const int32_t *__restrict__ idx,
                                      int64_t ncols, double *__restrict__ d, int64_t ldd) {
  // d(idx[j], c) = s(c, j) for c < k, j < ncols
  GRID_STRIDE(i, k * ncols) {
    const int64_t c = i % k, j = i / k;
    const int64_t dr = idx[j];
    if (dr < 0 || dr >= ncols) continue;
    d[dr + c * ldd] = s[c + j * lds];
  }
}

__global__ void set_identity_kernel(double *__restrict__ E, int64_t lde, int64_t rows, int64_t cols) {
  GRID_STRIDE(i, rows * cols) {
    const int64_t r = i % rows, c = i / rows;
    E[r + c * lde] = r == c ? 1.0 : 0.0;
  }
}

__global__ void iota_kernel(int32_t *__restrict__ p, int64_t n) {
  GRID_STRIDE(i, n) p[i] = (int32_t)i;
}

// Rinv = R^{-1} for an upper-triangular k x k R: column j solves R x = e_j by
// back substitution in column order, one workgroup per column, x in LDS:
// for i = j, j-1, ..., 0: x_i /= R_ii, then x_{0:i} -= x_i R_{0:i,i} with the
// threads spread over the rows (each step reads one column of R, coalesced;
// the next step's column is loaded while this one is applied).
constexpr int kTriThreads = 256;
__global__ __launch_bounds__(kTriThreads) void tri_inv_upper_kernel(const double *__restrict__ R, int64_t ldr,
                                                                    int64_t k, double *__restrict__ Ri, int64_t ldi) {
  extern __shared__ double x[];
  const int64_t j = blockIdx.x;
  const int t = threadIdx.x;
  for (int64_t r = t; r < k; r += kTriThreads) x[r] = r == j ? 1.0 : 0.0;
  __syncthreads();
  for (int64_t i = j; i >= 0; --i) {
    const double xi = x[i] / R[i + i * ldr];
    __syncthreads();   // every thread has read x[i] before it changes
    if (t == 0) x[i] = xi;
    const double *col = R + i * ldr;
    for (int64_t r = t; r < i; r += kTriThreads) x[r] -= xi * col[r];
    __syncthreads();
  }
  for (int64_t r = t; r < k; r += kTriThreads) Ri[r + j * ldi] = x[r];
}

template <typename S, typename D>
__global__ void copy_cast_kernel(const S *__restrict__ s, int64_t lds, D *__restrict__ d, int64_t ldd, int64_t rows,
                                 int64_t cols) {
  GRID_STRIDE(i, rows * cols) {
    const int64_t r = i % rows, c = i / rows;
    d[r + c * ldd] = (D)s[r + c * lds];
  }
}

template <typename T>
__global__ void gather_cols_t_kernel(const T *__restrict__ s, int64_t lds, int64_t rows, int64_t scols,
                                     const int32_t *__restrict__ idx, int64_t ncols, T *__restrict__ d, int64_t ldd) {
  GRID_STRIDE(i, rows * ncols) {
    const int64_t r = i % rows, c = i / rows;
    const int64_t src = idx[c];
    d[r + c * ldd] = (src >= 0 && src < scols) ? s[r + src * lds] : (T)__builtin_nan("");
  }
}

template <typename T>
__global__ void scatter_cols_t_kernel(const T *__restrict__ s, int64_t lds, int64_t rows, const int32_t *__restrict__ idx,
                                      int64_t ncols, T *__restrict__ d, int64_t ldd, int64_t dcols, int add) {
  GRID_STRIDE(i, rows * ncols) {
    const int64_t r = i % rows, c = i / rows;
    const int64_t dc = idx[c];
    if (dc < 0 || dc >= dcols) continue;
    T *p = d + r + dc * ldd;
    *p = add ? *p + s[r + c * lds] : s[r + c * lds];
  }
}

// Largest |y| of a column-major block, as the bits of a non-negative float
// (which order like the values), combined over workgroups with atomicMax on
// *out (zeroed beforehand).  NaNs are passed over (fmaxf keeps the number).
__global__ void absmax_bits_kernel(const float *__restrict__ y, int64_t ldy, int64_t rows, int64_t cols,
                                   unsigned *__restrict__ out) {
  float mx = 0.f;
  GRID_STRIDE(i, rows * cols) mx = fmaxf(mx, fabsf(y[i % rows + (i / rows) * ldy]));
  for (int o = 32; o > 0; o >>= 1) mx = fmaxf(mx, __shfl_xor(mx, o));
  if ((threadIdx.x & 63) == 0) atomicMax(out, __float_as_uint(mx));
}

// y <- 2^-e y with e the exponent of the largest |y| (an exact scaling, so
// that the block's largest entry lies in [1, 2)); nothing for a zero or
// non-finite maximum.
__global__ void scale_pow2_kernel(float *__restrict__ y, int64_t ldy, int64_t rows, int64_t cols,
                                  const unsigned *__restrict__ maxbits) {
  const float mx = __uint_as_float(*maxbits);
  if (!(mx > 0.f) || !isfinite(mx)) return;
  int e = ilogbf(mx);
  e = e > 120 ? 120 : (e < -120 ? -120 : e);
  const float sc = ldexpf(1.f, -e);
  GRID_STRIDE(i, rows * cols) y[i % rows + (i / rows) * ldy] *= sc;
}

}  // namespace

#define LAUNCH1D(kern, n, ...)                                                         \
  do {                                                                                 \
    if ((n) <= 0) return hipSuccess;                                                   \
    hipLaunchKernelGGL(kern, dim3(grid_for(n)), dim3(256), 0, s, __VA_ARGS__);         \
    return hipGetLastError();                                                          \
  } while (0)

hipError_t launch_copy2d(hipStream_t s, const double *src, int64_t lds, double *dst, int64_t ldd, int64_t rows,
                         int64_t cols) {
  LAUNCH1D(copy2d_kernel, rows * cols, src, lds, dst, ldd, rows, cols);
}
hipError_t launch_transpose(hipStream_t s, const double *src, int64_t lds, double *dst, int64_t ldd, int64_t rows,
                            int64_t cols) {
  LAUNCH1D(transpose_kernel, rows * cols, src, lds, dst, ldd, rows, cols);
}
hipError_t launch_extract_v(hipStream_t s, const double *F, int64_t ldf, int64_t mi, int64_t bi, double *V,
                            int64_t ldv) {
  LAUNCH1D(extract_v_kernel, mi * bi, F, ldf, mi, bi, V, ldv);
}
hipError_t launch_extract_r(hipStream_t s, const double *F, int64_t ldf, int64_t k, int64_t n, double *R,
                            int64_t ldr) {
  LAUNCH1D(extract_r_kernel, k * n, F, ldf, k, n, R, ldr);
}
hipError_t launch_gather_cols(hipStream_t s, const double *src, int64_t lds, int64_t rows, int64_t scols,
                              const int32_t *idx, int64_t ncols, double *dst, int64_t ldd) {
  LAUNCH1D(gather_cols_kernel, rows * ncols, src, lds, rows, scols, idx, ncols, dst, ldd);
}
hipError_t launch_scatter_cols(hipStream_t s, const double *src, int64_t lds, int64_t rows, const int32_t *idx,
                               int64_t ncols, double *dst, int64_t ldd, int64_t dcols, bool add) {
  LAUNCH1D(scatter_cols_kernel, rows * ncols, src, lds, rows, idx, ncols, dst, ldd, dcols, add ? 1 : 0);
}
hipError_t launch_scatter_rows_t(hipStream_t s, const double *src, int64_t lds, int64_t k, const int32_t *idx,
                                 int64_t ncols, double *dst, int64_t ldd) {
  LAUNCH1D(scatter_rows_t_kernel, k * ncols, src, lds, k, idx, ncols, dst, ldd);
}
hipError_t launch_set_identity(hipStream_t s, double *E, int64_t lde, int64_t rows, int64_t cols) {
  LAUNCH1D(set_identity_kernel, rows * cols, E, lde, rows, cols);
}
hipError_t launch_iota(hipStream_t s, int32_t *p, int64_t n) { LAUNCH1D(iota_kernel, n, p, n); }
hipError_t launch_copy_f32_f64(hipStream_t s, const float *src, int64_t lds, double *dst, int64_t ldd, int64_t rows,
                               int64_t cols) {
  LAUNCH1D((copy_cast_kernel<float, double>), rows * cols, src, lds, dst, ldd, rows, cols);
}
hipError_t launch_copy_f64_f32(hipStream_t s, const double *src, int64_t lds, float *dst, int64_t ldd, int64_t rows,
                               int64_t cols) {
  LAUNCH1D((copy_cast_kernel<double, float>), rows * cols, src, lds, dst, ldd, rows, cols);
}
hipError_t launch_copy2d_f32(hipStream_t s, const float *src, int64_t lds, float *dst, int64_t ldd, int64_t rows,
                             int64_t cols) {
  LAUNCH1D((copy_cast_kernel<float, float>), rows * cols, src, lds, dst, ldd, rows, cols);
}
hipError_t launch_gather_cols_f32(hipStream_t s, const float *src, int64_t lds, int64_t rows, int64_t scols,
                                  const int32_t *idx, int64_t ncols, float *dst, int64_t ldd) {
  LAUNCH1D(gather_cols_t_kernel<float>, rows * ncols, src, lds, rows, scols, idx, ncols, dst, ldd);
}
hipError_t launch_scatter_cols_f32(hipStream_t s, const float *src, int64_t lds, int64_t rows, const int32_t *idx,
                                   int64_t ncols, float *dst, int64_t ldd, int64_t dcols, bool add) {
  LAUNCH1D(scatter_cols_t_kernel<float>, rows * ncols, src, lds, rows, idx, ncols, dst, ldd, dcols, add ? 1 : 0);
}
hipError_t launch_tri_inv_upper(hipStream_t s, const double *R, int64_t ldr, int64_t k, double *Ri, int64_t ldi) {
  if (k <= 0) return hipSuccess;
  const size_t lds = (size_t)k * sizeof(double);
  if (lds > 64 * 1024) return hipErrorInvalidValue;   // at most 8192 columns
  hipLaunchKernelGGL(tri_inv_upper_kernel, dim3((unsigned)k), dim3(kTriThreads), (unsigned)lds, s, R, ldr, k, Ri, ldi);
  return hipGetLastError();
}

hipError_t launch_normalise_pow2(hipStream_t s, float *y, int64_t ldy, int64_t rows, int64_t cols, unsigned *word) {
  if (rows <= 0 || cols <= 0) return hipSuccess;
  hipError_t e = launch_zero_u32(s, word, 1);
  if (e != hipSuccess) return e;
  const int64_t n = rows * cols;
  hipLaunchKernelGGL(absmax_bits_kernel, dim3(grid_for(n) < 1024 ? grid_for(n) : 1024), dim3(256), 0, s, y, ldy,
                     rows, cols, word);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(scale_pow2_kernel, dim3(grid_for(n)), dim3(256), 0, s, y, ldy, rows, cols, word);
  return hipGetLastError();
}

}  // namespace rq
