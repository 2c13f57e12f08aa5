// SVD of a small upper-triangular block for the diagonalised blocks of
// Section 6.2: R22 = U' D V'^T with R22 the b x b triangle of a factored
// panel.  One-sided Jacobi (Hestenes): every sweep visits each column pair
// once and rotates the pair until it is orthogonal; the rotations
// accumulated on the identity give V'.  At convergence the columns are
// U' D; D is sorted in decreasing order (the usual convention of the SVD),
// U' = columns / D, and columns whose singular value is at rounding level are
// replaced by an orthonormal completion of the others.
//
// Two kernels.  b <= 64: one workgroup holds the working matrix and V' in
// LDS, a sweep is b - 1 rounds of b/2 disjoint pairs (the round-robin
// order), and the squared column norms computed at the start of a sweep are
// carried through each rotation (a' = a - t g, b' = b + t g), so a pair needs
// one reduction.  64 < b <= 256 (the working pair of b x b matrices, 1 MB at
// b = 256, exceeds one CU's LDS): block Jacobi over blocks of 16 columns.  A
// cooperative launch of one workgroup per pair of blocks; in each round every
// workgroup loads its two blocks (32 columns of the working matrix and of V')
// into LDS, rotates column pairs (one wave per pair) and writes them back;
// the block pairs follow the round-robin order over blocks, the first round
// of a sweep takes all pairs of the 32 columns and the others the pairs
// across the two blocks, so a sweep meets every column pair once.  The
// iteration stops after the first sweep in which no workgroup rotated any
// pair: then every pair passed the orthogonality test in that sweep.  A
// single-workgroup kernel then forms D, the sorted U' and V' and the
// completion from the working columns.
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
  // a pair counts as orthogonal once |a_p^T a_q| <= sqrt(n) u |a_p| |a_q| (the
  // one-sided Jacobi test of LAPACK's dgesvj): the columns of U' then meet
  // |U'^T U' - I| at about 1e-13 for b = 256, where n eps per pair left 3e-12
  const double tol = sqrt((double)n) * 1.1102230246251565e-16;
  const double thr_rel = (double)n * 2.220446049250313e-16;   // rounding level of a singular value
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
  const double thr = thr_rel * smax;
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


// ---------------------------------------------------------------------------
// Blocks of 65 to 256 columns

constexpr int kCoopMaxN = 256;
constexpr int kCoopW = 16;                  // columns per block
constexpr int kCoopCols = 2 * kCoopW;       // columns a workgroup holds
constexpr int kCoopThreads = 1024;          // one wave per pair of a local round
constexpr int kCoopRows = kCoopMaxN / 64;   // rows per lane
constexpr size_t kCoopLds = (size_t)2 * kCoopCols * kCoopMaxN * sizeof(double);
static_assert(kCoopCols / 2 == kCoopThreads / 64, "one wave per pair");
static_assert(kCoopCols * kCoopMaxN % kCoopThreads == 0, "whole loads per thread");
static_assert(kBarrierWords + kSvdMaxSweeps <= 448, "rotation words inside the barrier slot");

struct SvdCoopArgs {
  const double *F; int64_t ldf; int n;
  double *a; double *v;   // working columns and V' (n x n each, ld n)
  unsigned *rot;          // kSvdMaxSweeps words, zero on entry: a rotation happened in sweep s
  int32_t *info;
};

__global__ __launch_bounds__(kCoopThreads) void svd_jacobi_coop_kernel(SvdCoopArgs s, GridBarrier gb) {
  extern __shared__ double lds[];
  double(*la)[kCoopMaxN] = reinterpret_cast<double(*)[kCoopMaxN]>(lds);
  double(*lv)[kCoopMaxN] = reinterpret_cast<double(*)[kCoopMaxN]>(lds + kCoopCols * kCoopMaxN);
  __shared__ double nrm[kCoopCols];
  __shared__ int lrot, done;
  const int n = s.n;
  const int nblk0 = (n + kCoopW - 1) / kCoopW;
  const int nblk = nblk0 + (nblk0 & 1);   // an odd count gets a block of zero columns
  const int t = threadIdx.x, wave = t >> 6, lane = t & 63;
  const double tol = sqrt((double)n) * 1.1102230246251565e-16;   // the test of the one-workgroup kernel
  unsigned gen = 0;
  for (int sweep = 0; sweep < kSvdMaxSweeps; ++sweep) {
    for (int k = 0; k + 1 < nblk; ++k) {
      // this workgroup's block pair in round k of the round-robin order
      const int m1 = nblk - 1, g = blockIdx.x;
      const int bp = g == 0 ? k : (k + g) % m1;
      const int bq = g == 0 ? m1 : (k - g + m1) % m1;
      const bool first = sweep == 0 && k == 0;   // every block is met once per round
      // all of a thread's loads in flight before the first LDS store
      constexpr int kPer = kCoopCols * kCoopMaxN / kCoopThreads;
      double xs[kPer], ys[kPer];
#pragma unroll
      for (int e = 0; e < kPer; ++e) {
        const int i = t + e * kCoopThreads, c = i / kCoopMaxN, r = i % kCoopMaxN;
        const int gc = (c < kCoopW ? bp : bq) * kCoopW + c % kCoopW;
        xs[e] = 0.0;
        ys[e] = 0.0;
        if (gc < n && r < n) {
          if (first) {
            xs[e] = r <= gc ? s.F[r + (int64_t)gc * s.ldf] : 0.0;
            ys[e] = r == gc ? 1.0 : 0.0;
          } else {
            xs[e] = ld_agent(s.a + r + (int64_t)gc * n);
            ys[e] = ld_agent(s.v + r + (int64_t)gc * n);
          }
        }
      }
#pragma unroll
      for (int e = 0; e < kPer; ++e) {
        const int i = t + e * kCoopThreads;
        la[i / kCoopMaxN][i % kCoopMaxN] = xs[e];
        lv[i / kCoopMaxN][i % kCoopMaxN] = ys[e];
      }
      if (t == 0) lrot = 0;
      __syncthreads();
      for (int c = wave; c < kCoopCols; c += kCoopThreads / 64) {
        double s2 = 0.0;
#pragma unroll
        for (int j = 0; j < kCoopRows; ++j) {
          const double x = la[c][lane + 64 * j];
          s2 += x * x;
        }
        s2 = wave_sum(s2);
        if (lane == 0) nrm[c] = s2;
      }
      __syncthreads();
      // The column pairs of this visit; rows past n hold zeros, which every
      // rotation keeps.  The first round of a sweep meets every block once:
      // there all pairs of the 32 columns (31 rounds of 16 pairs); the other
      // rounds take the 16 x 16 pairs across the two blocks only (16 rounds:
      // wave i pairs column i with 16 + (i + r) mod 16), so that a sweep
      // visits every pair once, as the one-workgroup kernel does (the same
      // number of sweeps as all pairs at every visit in an FP64 model of the
      // iteration, with 45 % fewer rounds and fewer rotations on V')
      const int nlr = k == 0 ? kCoopCols - 1 : kCoopW;
      for (int lr = 0; lr < nlr; ++lr) {
        int p, q;
        if (k == 0) {
          const int mm = kCoopCols - 1;
          p = wave == 0 ? lr : (lr + wave) % mm;
          q = wave == 0 ? mm : (lr - wave + mm) % mm;
          if (p > q) { const int x = p; p = q; q = x; }
        } else {
          p = wave;
          q = kCoopW + (wave + lr) % kCoopW;
        }
        const double al = nrm[p], be = nrm[q];
        double xp[kCoopRows], xq[kCoopRows], yp[kCoopRows], yq[kCoopRows];
        double ga = 0.0;
#pragma unroll
        for (int j = 0; j < kCoopRows; ++j) {
          const int r = lane + 64 * j;
          xp[j] = la[p][r]; xq[j] = la[q][r];
        }
#pragma unroll
        for (int j = 0; j < kCoopRows; ++j) ga += xp[j] * xq[j];
        ga = wave_sum(ga);   // the same bits in every lane: the test below is uniform
        if (ga * ga > tol * tol * al * be) {
#pragma unroll
          for (int j = 0; j < kCoopRows; ++j) {   // V' rows only for a rotation
            const int r = lane + 64 * j;
            yp[j] = lv[p][r]; yq[j] = lv[q][r];
          }
          const double zeta = (be - al) / (2.0 * ga);
          const double az = fabs(zeta);
          const double root = az > 1.0 ? az * sqrt(1.0 + 1.0 / (zeta * zeta)) : sqrt(1.0 + zeta * zeta);
          const double tn = (zeta >= 0.0 ? 1.0 : -1.0) / (az + root);
          const double cs = 1.0 / sqrt(1.0 + tn * tn), sn = cs * tn;
#pragma unroll
          for (int j = 0; j < kCoopRows; ++j) {
            const int r = lane + 64 * j;
            la[p][r] = cs * xp[j] - sn * xq[j];
            la[q][r] = sn * xp[j] + cs * xq[j];
            lv[p][r] = cs * yp[j] - sn * yq[j];
            lv[q][r] = sn * yp[j] + cs * yq[j];
          }
          if (lane == 0) {
            nrm[p] = al - tn * ga;
            nrm[q] = be + tn * ga;
            lrot = 1;
          }
        }
        __syncthreads();
      }
      for (int i = t; i < kCoopCols * kCoopMaxN; i += kCoopThreads) {
        const int c = i / kCoopMaxN, r = i % kCoopMaxN;
        const int gc = (c < kCoopW ? bp : bq) * kCoopW + c % kCoopW;
        if (gc < n && r < n) {
          st_agent(s.a + r + (int64_t)gc * n, la[c][r]);
          st_agent(s.v + r + (int64_t)gc * n, lv[c][r]);
        }
      }
      if (t == 0 && lrot) __hip_atomic_store(s.rot + sweep, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      if (!grid_sync(gb, gen, true, true)) {
        if (t == 0 && s.info) atomicExch(&s.info[2], 1);
        return;
      }
    }
    // every workgroup reads the same word after the same barrier: the same decision
    if (t == 0) done = __hip_atomic_load(s.rot + sweep, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 0u;
    __syncthreads();
    if (done) break;
  }
}

// D, the sorted U' and V', and the completion, from the working columns that
// the cooperative kernel left in a and v (n x n, ld n).
__global__ __launch_bounds__(kCoopThreads) void svd_finish_kernel(double *__restrict__ F, int64_t ldf, int n,
                                                                 double *__restrict__ a,
                                                                 const double *__restrict__ v,
                                                                 double *__restrict__ U, int64_t ldu,
                                                                 double *__restrict__ V, int64_t ldv) {
  __shared__ double sig[kCoopMaxN], resid[kCoopMaxN], coef[kCoopMaxN];
  __shared__ int order[kCoopMaxN], accepted[kCoopMaxN];
  __shared__ int pick;
  __shared__ double cnorm;
  const int t = threadIdx.x, wave = t >> 6, lane = t & 63;
  const double thr_rel = (double)n * 2.220446049250313e-16;
  auto col = [&](int c) { return a + (int64_t)c * n; };
  for (int c = wave; c < n; c += kCoopThreads / 64) {
    double s2 = 0.0;
    for (int r = lane; r < n; r += 64) s2 += col(c)[r] * col(c)[r];
    s2 = wave_sum(s2);
    if (lane == 0) sig[c] = sqrt(s2);
  }
  __syncthreads();
  // decreasing singular values; equal values keep their column order, and a
  // non-finite value (from a non-finite input) sorts last, so that the ranks
  // always form a permutation
  if (t < n) {
    auto key = [&](int c) { return sig[c] == sig[c] ? sig[c] : -1.0; };
    const double kt = key(t);
    int rank = 0;
    for (int o = 0; o < n; ++o) {
      const double ko = key(o);
      rank += (ko > kt) || (ko == kt && o < t);
    }
    order[rank] = t;
  }
  __syncthreads();
  const double thr = thr_rel * sig[order[0]];
  for (int i = t; i < n * n; i += kCoopThreads) {
    const int c = i / n, r = i % n;
    const double sc = sig[c];
    if (sc > thr && sc > 0.0) col(c)[r] = col(c)[r] / sc;
  }
  if (t < n) accepted[t] = (sig[t] > thr && sig[t] > 0.0) ? 1 : 0;
  __syncthreads();
  // orthonormal completion, as in the one-workgroup kernel: the unit vector
  // with the largest residual against the accepted columns (at least d/n for
  // d missing directions), two passes of classical Gram-Schmidt, normalised
  for (int j = 0; j < n; ++j) {
    const int c = order[j];
    if (accepted[c]) continue;   // uniform
    if (t < n) {
      double s2 = 0.0;
      for (int o = 0; o < n; ++o)
        if (accepted[o]) s2 += col(o)[t] * col(o)[t];
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
    if (t < n) col(c)[t] = t == pick ? 1.0 : 0.0;
    __syncthreads();
    for (int pass = 0; pass < 2; ++pass) {
      if (t < n) {
        double d = 0.0;
        if (accepted[t])
          for (int r = 0; r < n; ++r) d += col(t)[r] * col(c)[r];
        coef[t] = d;
      }
      __syncthreads();
      double x = 0.0;
      if (t < n) {
        x = col(c)[t];
        for (int o = 0; o < n; ++o)
          if (accepted[o]) x -= coef[o] * col(o)[t];
      }
      __syncthreads();
      if (t < n) col(c)[t] = x;
      __syncthreads();
    }
    if (wave == 0) {
      double s2 = 0.0;
      for (int r = lane; r < n; r += 64) s2 += col(c)[r] * col(c)[r];
      s2 = wave_sum(s2);
      if (lane == 0) {
        cnorm = sqrt(s2);
        accepted[c] = 1;
      }
    }
    __syncthreads();
    if (t < n) col(c)[t] /= cnorm;
    __syncthreads();
  }
  for (int i = t; i < n * n; i += kCoopThreads) {
    const int j = i / n, r = i % n;
    const int c = order[j];
    U[r + (int64_t)j * ldu] = col(c)[r];
    V[r + (int64_t)j * ldv] = v[r + (int64_t)c * n];
    if (r <= j) F[r + (int64_t)j * ldf] = r == j ? sig[c] : 0.0;
  }
}

}  // namespace

int svd_small_max_block() { return kCoopMaxN; }

size_t svd_small_work_doubles(int nb) { return nb > kSvdMaxB ? (size_t)2 * nb * nb : 0; }

hipError_t launch_svd_small(hipStream_t s, const SvdSmall &p) {
  const int nb = p.nb;
  if (nb < 1 || nb > kCoopMaxN || p.ldf < nb || p.ldu < nb || p.ldv < nb) return hipErrorInvalidValue;
  if (nb <= kSvdMaxB) {
    hipLaunchKernelGGL(svd_jacobi_kernel, dim3(1), dim3(kSvdThreads), 0, s, p.F, p.ldf, nb, p.U, p.ldu, p.V,
                       p.ldv);
    return hipGetLastError();
  }
  if (!p.work || !p.bar || !p.abort_flag) return hipErrorInvalidValue;
  static bool attr_done = false;
  if (!attr_done) {
    hipError_t e = hipFuncSetAttribute((const void *)svd_jacobi_coop_kernel,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)kCoopLds);
    if (e != hipSuccess) return e;
    attr_done = true;
  }
  const int nblk0 = (nb + kCoopW - 1) / kCoopW;
  const int nwg = (nblk0 + (nblk0 & 1)) / 2;
  SvdCoopArgs a{p.F, p.ldf, nb, p.work, p.work + (size_t)nb * nb, p.bar + kBarrierWords, p.info};
  GridBarrier gb{p.bar, p.abort_flag, p.limit_ticks};
  void *args[] = {&a, &gb};
  hipError_t e = hipLaunchCooperativeKernel((const void *)svd_jacobi_coop_kernel, dim3(nwg), dim3(kCoopThreads),
                                            args, (unsigned)kCoopLds, s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(svd_finish_kernel, dim3(1), dim3(kCoopThreads), 0, s, p.F, p.ldf, nb, a.a, a.v, p.U, p.ldu,
                     p.V, p.ldv);
  return hipGetLastError();
}

}  // namespace rq
