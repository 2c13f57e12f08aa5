// SVD of a small upper-triangular block for the diagonalised blocks of
// Section 6.2: R22 = U' D V'^T with R22 the b x b triangle of a factored
// panel (b <= 64).  One workgroup holds the working matrix and V' in LDS and
// runs one-sided Jacobi (Hestenes): every sweep visits each column pair once,
// in the round-robin order that splits a sweep into b - 1 rounds of b/2
// disjoint pairs, and rotates the pair until it is orthogonal.  The squared
// column norms are computed at the start of a sweep and carried through each
// rotation (a' = a - t g, b' = b + t g), so a pair needs one reduction.  At
// convergence the columns are U' D; D is sorted in decreasing order (the
// usual convention of the SVD), U' = columns / D, and columns whose singular
// value is at rounding level are replaced by an orthonormal completion of the
// others.
#include "common.h"

namespace rq {

namespace {

constexpr int kSvdMaxB = 64;
constexpr int kSvdThreads = 256;
constexpr int kSvdGroup = 8;            // lanes per column pair
constexpr int kSvdMaxSweeps = 40;

__global__ __launch_bounds__(kSvdThreads) void svd_jacobi_kernel(double *__restrict__ F, int64_t ldf, int nb,
                                                                double *__restrict__ U, int64_t ldu,
                                                                double *__restrict__ V, int64_t ldv) {
  __shared__ double a[kSvdMaxB][kSvdMaxB + 1];   // a[column][row]
  __shared__ double v[kSvdMaxB][kSvdMaxB + 1];
  __shared__ double sig[kSvdMaxB];
  __shared__ double nrm[kSvdMaxB];   // squared column norms within a sweep
  __shared__ int order[kSvdMaxB];
  __shared__ int rotated;
  __shared__ int accepted[kSvdMaxB];
  __shared__ double resid[kSvdMaxB], coef[kSvdMaxB];
  __shared__ int pick;
  const int t = threadIdx.x;
  const int n = nb;
  const int ne = (n + 1) & ~1;   // an odd count gets a zero column that never rotates
  for (int i = t; i < kSvdMaxB * kSvdMaxB; i += kSvdThreads) {
    const int c = i / kSvdMaxB, r = i % kSvdMaxB;
    a[c][r] = (c < n && r < n && r <= c) ? F[r + (int64_t)c * ldf] : 0.0;
    v[c][r] = c == r ? 1.0 : 0.0;
  }
  __syncthreads();   // the sweep's norms read columns loaded by other threads
  const int g = t / kSvdGroup, l = t % kSvdGroup;
  const double tol = (double)n * 2.220446049250313e-16;
  for (int sweep = 0; sweep < kSvdMaxSweeps; ++sweep) {
    if (t == 0) rotated = 0;
    if (t < kSvdMaxB) {
      double s2 = 0.0;
      for (int r = 0; r < n; ++r) s2 += a[t][r] * a[t][r];
      nrm[t] = s2;
    }
    __syncthreads();
    for (int k = 0; k + 1 < ne; ++k) {
      // round k of the circle method: (k, ne-1) and ((k+j), (k-j)) mod (ne-1)
      if (g < ne / 2) {
        const int m1 = ne - 1;
        int p = g == 0 ? k : (k + g) % m1;
        int q = g == 0 ? m1 : (k - g + m1) % m1;
        if (p > q) { const int x = p; p = q; q = x; }
        const double al = nrm[p], be = nrm[q];
        // the pair's rows of this lane, read once (rows past n read as zero:
        // the padding rows of a and v hold zeros and are never written)
        constexpr int kRows = kSvdMaxB / kSvdGroup;
        double xp[kRows], xq[kRows], yp[kRows], yq[kRows];
        double ga = 0.0;
#pragma unroll
        for (int j = 0; j < kRows; ++j) {
          const int r = l + j * kSvdGroup;
          xp[j] = a[p][r]; xq[j] = a[q][r];
          yp[j] = v[p][r]; yq[j] = v[q][r];
        }
#pragma unroll
        for (int j = 0; j < kRows; ++j) ga += xp[j] * xq[j];
#pragma unroll
        for (int o = 1; o < kSvdGroup; o <<= 1) ga += __shfl_xor(ga, o, kSvdGroup);
        if (ga * ga > tol * tol * al * be) {
          const double zeta = (be - al) / (2.0 * ga);
          const double az = fabs(zeta);
          const double root = az > 1.0 ? az * sqrt(1.0 + 1.0 / (zeta * zeta)) : sqrt(1.0 + zeta * zeta);
          const double tn = (zeta >= 0.0 ? 1.0 : -1.0) / (az + root);
          const double cs = 1.0 / sqrt(1.0 + tn * tn), sn = cs * tn;
#pragma unroll
          for (int j = 0; j < kRows; ++j) {
            const int r = l + j * kSvdGroup;
            if (r < n) {
              a[p][r] = cs * xp[j] - sn * xq[j];
              a[q][r] = sn * xp[j] + cs * xq[j];
              v[p][r] = cs * yp[j] - sn * yq[j];
              v[q][r] = sn * yp[j] + cs * yq[j];
            }
          }
          if (l == 0) {
            nrm[p] = al - tn * ga;
            nrm[q] = be + tn * ga;
            rotated = 1;
          }
        }
      }
      __syncthreads();
    }
    const int any = rotated;
    __syncthreads();
    if (!any) break;
  }
  if (t < n) {
    double s2 = 0.0;
    for (int r = 0; r < n; ++r) s2 += a[t][r] * a[t][r];
    sig[t] = sqrt(s2);
  }
  __syncthreads();
  if (t == 0) {
    // decreasing singular values; equal values keep their column order
    for (int j = 0; j < n; ++j) order[j] = j;
    for (int j = 0; j < n; ++j) {
      int best = j;
      for (int c = j + 1; c < n; ++c)
        if (sig[order[c]] > sig[order[best]]) best = c;
      const int x = order[j]; order[j] = order[best]; order[best] = x;
    }
  }
  __syncthreads();
  const double smax = sig[order[0]];
  const double thr = tol * smax;
  // U' columns (unsorted slots): a_j / sigma_j where sigma_j is above rounding level
  for (int i = t; i < n * n; i += kSvdThreads) {
    const int c = i / n, r = i % n;
    const double sc = sig[c];
    if (sc > thr && sc > 0.0) a[c][r] = a[c][r] / sc;
  }
  __syncthreads();
  // Orthonormal completion of the columns at rounding level, in sorted
  // order.  With the accepted columns orthonormal, unit vector e keeps the
  // squared residual 1 - sum_o u_o(e)^2 after projection; these residuals sum
  // to the number d of missing directions, so the largest is at least d/n
  // and the choice below never fails, whatever subspace the accepted columns
  // span.  The chosen unit vector is orthogonalised by two passes of
  // classical Gram-Schmidt and normalised.
  if (t < n) accepted[t] = (sig[t] > thr && sig[t] > 0.0) ? 1 : 0;
  __syncthreads();
  for (int j = 0; j < n; ++j) {
    const int c = order[j];
    if (accepted[c]) continue;   // uniform: every thread reads the same LDS word
    if (t < n) {
      double s2 = 0.0;
      for (int o = 0; o < n; ++o)
        if (accepted[o]) s2 += a[o][t] * a[o][t];
      resid[t] = 1.0 - s2;
    }
    __syncthreads();
    if (t == 0) {
      int best = 0;
      for (int e = 1; e < n; ++e)
        if (resid[e] > resid[best]) best = e;
      pick = best;
    }
    __syncthreads();
    const int e = pick;
    if (t < n) a[c][t] = t == e ? 1.0 : 0.0;
    __syncthreads();
    for (int pass = 0; pass < 2; ++pass) {
      if (t < n) {
        double d = 0.0;
        if (accepted[t])
          for (int r = 0; r < n; ++r) d += a[t][r] * a[c][r];
        coef[t] = d;
      }
      __syncthreads();
      double x = 0.0;
      if (t < n) {
        x = a[c][t];
        for (int o = 0; o < n; ++o)
          if (accepted[o]) x -= coef[o] * a[o][t];
      }
      __syncthreads();
      if (t < n) a[c][t] = x;
      __syncthreads();
    }
    if (t == 0) {
      double nn = 0.0;
      for (int r = 0; r < n; ++r) nn += a[c][r] * a[c][r];
      resid[0] = sqrt(nn);
      accepted[c] = 1;
    }
    __syncthreads();
    if (t < n) a[c][t] /= resid[0];
    __syncthreads();
  }
  for (int i = t; i < n * n; i += kSvdThreads) {
    const int j = i / n, r = i % n;
    const int c = order[j];
    U[r + (int64_t)j * ldu] = a[c][r];
    V[r + (int64_t)j * ldv] = v[c][r];
    // the triangle of F becomes D (the reflectors below it stay)
    if (r <= j) F[r + (int64_t)j * ldf] = r == j ? sig[c] : 0.0;
  }
}

}  // namespace

int svd_small_max_block() { return kSvdMaxB; }

hipError_t launch_svd_small(hipStream_t s, double *F, int64_t ldf, int nb, double *U, int64_t ldu, double *V,
                            int64_t ldv) {
  if (nb < 1 || nb > kSvdMaxB || ldf < nb || ldu < nb || ldv < nb) return hipErrorInvalidValue;
  hipLaunchKernelGGL(svd_jacobi_kernel, dim3(1), dim3(kSvdThreads), 0, s, F, ldf, nb, U, ldu, V, ldv);
  return hipGetLastError();
}

}  // namespace rq
