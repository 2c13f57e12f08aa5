// Standalone driver of librqrcp through its C ABI only (no Python, no torch):
// factors a seeded m x n matrix with uniform entries in [-1, 1) `steps`
// times, timing each factorization with HIP events, then runs one plain copy
// kernel over 2^26 doubles (2^29 bytes read, 2^29 bytes written).  It serves
// hardware-counter runs under rocprofv3, where the copy kernel calibrates the
// HBM byte counters, and shows the minimal use of the C ABI.
//
//   rqrcp_bench [m n b p steps f64|f32 plain|mixed]      (default 8192 8192 256 10 1 f64 plain)
//
// The trailing-update GEMMs launched for a given (m, n, b) do the same work
// and move the same bytes whatever the matrix entries are, so this input
// stands in for the Haar-based test matrices when only counters are wanted.
#include <hip/hip_runtime.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "rqrcp.h"

#define HCHECK(x)                                                                                \
  do {                                                                                           \
    hipError_t e_ = (x);                                                                         \
    if (e_ != hipSuccess) {                                                                      \
      fprintf(stderr, "HIP error %s at %s:%d\n", hipGetErrorString(e_), __FILE__, __LINE__);     \
      exit(1);                                                                                   \
    }                                                                                            \
  } while (0)

#define RCHECK(h, x)                                                                             \
  do {                                                                                           \
    rqrcp_status_t s_ = (x);                                                                     \
    if (s_ != RQRCP_OK) {                                                                        \
      fprintf(stderr, "rqrcp error %s: %s\n", rqrcp_status_string(s_), rqrcp_last_error(h));    \
      exit(1);                                                                                   \
    }                                                                                            \
  } while (0)

__device__ __forceinline__ double uniform_pm1(uint64_t i, uint64_t seed) {
  uint64_t z = i + seed * 0x9E3779B97F4A7C15ull;   // splitmix64 finaliser
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  z ^= z >> 31;
  return (double)(z >> 11) * 0x1.0p-52 - 1.0;
}

template <typename T>
__global__ void fill_kernel(T *a, size_t n, uint64_t seed) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    a[i] = (T)uniform_pm1(i, seed);
}

__global__ void calib_copy_kernel(const double *__restrict__ x, double *__restrict__ y, size_t n) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    y[i] = x[i];
}

int main(int argc, char **argv) {
  int64_t m = 8192, n = 8192, b = 256, p = 10;
  int steps = 1;
  rqrcp_dtype_t dt = RQRCP_F64;
  int prec = RQRCP_PREC_PLAIN;
  if (argc > 1) m = atoll(argv[1]);
  if (argc > 2) n = atoll(argv[2]);
  if (argc > 3) b = atoll(argv[3]);
  if (argc > 4) p = atoll(argv[4]);
  if (argc > 5) steps = atoi(argv[5]);
  if (argc > 6) dt = strcmp(argv[6], "f32") == 0 ? RQRCP_F32 : RQRCP_F64;
  if (argc > 7) prec = strcmp(argv[7], "mixed") == 0 ? RQRCP_PREC_MIXED : RQRCP_PREC_PLAIN;
  if (m < 1 || n < 1 || m < n || steps < 0) {
    fprintf(stderr, "usage: rqrcp_bench [m n b p steps f64|f32 plain|mixed] with m >= n >= 1\n");
    return 2;
  }
  const size_t esz = dt == RQRCP_F64 ? sizeof(double) : sizeof(float);

  HCHECK(hipSetDevice(0));
  rqrcp_handle_t h = NULL;
  RCHECK(NULL, rqrcp_create(&h, NULL));
  rqrcp_opts_t o;
  rqrcp_default_opts(&o);
  o.block = b;
  o.oversample = p;
  o.precision = prec;
  o.seed = 6;
  size_t tau_n = 0, T_n = 0, S_n = 0, work_b = 0;
  RCHECK(h, rqrcp_factor_sizes(dt, m, n, &o, &tau_n, &T_n, &S_n, &work_b));

  void *A0, *A, *work;
  int32_t *jpvt, *info;
  double *tau, *T, *S = NULL;
  HCHECK(hipMalloc(&A0, (size_t)m * n * esz));
  HCHECK(hipMalloc(&A, (size_t)m * n * esz));
  HCHECK(hipMalloc(&jpvt, (size_t)n * sizeof(int32_t)));
  HCHECK(hipMalloc(&info, 4 * sizeof(int32_t)));
  HCHECK(hipMalloc(&tau, (tau_n ? tau_n : 1) * sizeof(double)));
  HCHECK(hipMalloc(&T, (T_n ? T_n : 1) * sizeof(double)));
  if (S_n) HCHECK(hipMalloc(&S, S_n * sizeof(double)));
  HCHECK(hipMalloc(&work, work_b ? work_b : 256));
  o.info = info;
  if (dt == RQRCP_F64)
    hipLaunchKernelGGL(fill_kernel<double>, dim3(4096), dim3(256), 0, 0, (double *)A0, (size_t)m * n, 1ull);
  else
    hipLaunchKernelGGL(fill_kernel<float>, dim3(4096), dim3(256), 0, 0, (float *)A0, (size_t)m * n, 1ull);
  HCHECK(hipGetLastError());
  HCHECK(hipDeviceSynchronize());

  hipEvent_t e0, e1;
  HCHECK(hipEventCreate(&e0));
  HCHECK(hipEventCreate(&e1));
  for (int s = 0; s < steps; ++s) {
    HCHECK(hipMemcpyAsync(A, A0, (size_t)m * n * esz, hipMemcpyDeviceToDevice, 0));
    HCHECK(hipEventRecord(e0, 0));
    RCHECK(h, rqrcp_factor(h, dt, m, n, A, m, jpvt, tau, T, S, &o, work, work_b));
    HCHECK(hipEventRecord(e1, 0));
    HCHECK(hipEventSynchronize(e1));
    float ms = 0.f;
    HCHECK(hipEventElapsedTime(&ms, e0, e1));
    int32_t hinfo[4];
    HCHECK(hipMemcpy(hinfo, info, sizeof(hinfo), hipMemcpyDeviceToHost));
    const double nf = (double)n, mf = (double)m;
    printf("factor %lld x %lld b=%lld p=%lld %s %s: %.3f ms, %.1f normalised GFLOP/s, info %d %d %d\n",
           (long long)m, (long long)n, (long long)b, (long long)p, dt == RQRCP_F64 ? "f64" : "f32",
           prec == RQRCP_PREC_MIXED ? "mixed" : "plain", ms, (2.0 * mf * nf * nf - 2.0 * nf * nf * nf / 3.0) / ms / 1e6,
           hinfo[0], hinfo[1], hinfo[2]);
    fflush(stdout);
    if (hinfo[2]) return 3;
  }

  const size_t nc = (size_t)1 << 26;
  double *x, *y;
  HCHECK(hipMalloc(&x, nc * sizeof(double)));
  HCHECK(hipMalloc(&y, nc * sizeof(double)));
  hipLaunchKernelGGL(fill_kernel<double>, dim3(4096), dim3(256), 0, 0, x, nc, 2ull);
  HCHECK(hipDeviceSynchronize());
  HCHECK(hipEventRecord(e0, 0));
  hipLaunchKernelGGL(calib_copy_kernel, dim3(8192), dim3(256), 0, 0, x, y, nc);
  HCHECK(hipGetLastError());
  HCHECK(hipEventRecord(e1, 0));
  HCHECK(hipEventSynchronize(e1));
  float cms = 0.f;
  HCHECK(hipEventElapsedTime(&cms, e0, e1));
  printf("calibration copy: %zu bytes read + %zu written in %.3f ms (%.0f GB/s)\n", nc * 8, nc * 8, cms,
         2.0 * nc * 8 / cms / 1e6);
  fflush(stdout);

  HCHECK(hipFree(x));
  HCHECK(hipFree(y));
  HCHECK(hipFree(A0));
  HCHECK(hipFree(A));
  HCHECK(hipFree(jpvt));
  HCHECK(hipFree(info));
  HCHECK(hipFree(tau));
  HCHECK(hipFree(T));
  if (S) HCHECK(hipFree(S));
  HCHECK(hipFree(work));
  RCHECK(h, rqrcp_destroy(h));
  printf("done\n");
  fflush(stdout);
  return 0;
}
