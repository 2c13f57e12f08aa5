// Pivot selection on the small sketch Y (k x n', k = b + p): the classical
// column-pivoted Householder QR of Section 3.3 (Fig. 2) run for only the
// first nsteps steps (Section 4.1 eq. Yrows, Section 4.3).  Only the pivot
// decisions leave the kernel; Y is scratch.  The same kernel also runs the
// classical QRCP of the last block of Fig. 3 with Y := X.
//
// Rule: at step j take the column with the largest 2-norm over rows j..k-1
// (norms recomputed exactly after every reflector, not downdated); ties go to
// the lowest current position; the winner swaps places with position j.
//
// One persistent cooperative launch.  Columns are dealt in contiguous slabs
// of cpw columns to workgroups and stay resident in LDS for all steps.  A
// step is: local argmax -> publish (norm, position, column id) and the
// candidate's current values -> one grid barrier -> every workgroup reduces
// the published records in the same way, reads the winning column, forms the
// reflector redundantly and applies it to its own columns.  Positions are
// tracked per column, so the swaps themselves never move data; at the end
// each column's final position (dest) and the list of columns that moved are
// written for the data-movement kernels.
#include <climits>

#include "common.h"

namespace rq {

namespace {

constexpr int kQThreads = 512;
constexpr int kQWaves = kQThreads / 64;
constexpr size_t kLdsDoubles = 20480 - 256;   // 160 KiB minus room for static shared data

__device__ __forceinline__ bool better(double v1, int p1, double v2, int p2) {
  return v1 > v2 || (v1 == v2 && p1 < p2);
}

__device__ void flag_nonfinite(int32_t *info, int block_index) {
  if (!info) return;
  atomicExch(&info[0], 1);
  atomicCAS(&info[1], 0, block_index + 1);
}

// Block-wide argmax over (val, pos, idx) held at red_*[0..kQThreads).
__device__ void block_argmax(double *rv, int *rp, int *ri) {
  const int t = threadIdx.x;
  for (int s = kQThreads / 2; s > 0; s >>= 1) {
    __syncthreads();
    if (t < s && better(rv[t + s], rp[t + s], rv[t], rp[t])) {
      rv[t] = rv[t + s];
      rp[t] = rp[t + s];
      ri[t] = ri[t + s];
    }
  }
  __syncthreads();
}

__global__ __launch_bounds__(kQThreads) void qrcp_small_kernel(QrcpSmall q, int cpw, GridBarrier gb) {
  extern __shared__ double lds[];
  const int k = q.k;
  double *Yl = lds;                           // cpw * k, column-major
  double *nrm = Yl + (size_t)cpw * k;         // cpw   squared norms of the remaining rows
  double *v = nrm + cpw;                      // k     reflector / winning column
  double *rv = v + k;                         // kQThreads
  int *rp = (int *)(rv + kQThreads);          // kQThreads
  int *ri = rp + kQThreads;                   // kQThreads
  int *pos = ri + kQThreads;                  // cpw   current position of each column
  int *act = pos + cpw;                       // cpw   1 while not yet chosen
  __shared__ double s_tau;
  __shared__ int s_win_wg, s_win_pos, s_win_col;

  const int nwg = gridDim.x, wg = blockIdx.x, t = threadIdx.x;
  const int lane = t & 63, wave = t >> 6;
  const int c0 = wg * cpw;
  const int nloc = max(0, min(cpw, q.ncols - c0));

  for (int64_t idx = t; idx < (int64_t)nloc * k; idx += kQThreads) {
    const int c = (int)(idx / k), r = (int)(idx % k);
    Yl[(size_t)c * k + r] = q.Y[r + (int64_t)(c0 + c) * q.ldy];
  }
  for (int c = t; c < cpw; c += kQThreads) {
    pos[c] = c0 + c;
    act[c] = c < nloc ? 1 : 0;
  }
  __syncthreads();
  for (int c = wave; c < nloc; c += kQWaves) {
    const double *y = Yl + (size_t)c * k;
    double s = 0.0;
    for (int r = lane; r < k; r += 64) s += y[r] * y[r];
    s = wave_sum(s);
    if (lane == 0) nrm[c] = s;
  }

  unsigned gen = 0;
  bool ok = true;
  for (int j = 0; j < q.nsteps && ok; ++j) {
    __syncthreads();
    // local argmax over active columns
    double bv = -1.0;
    int bp = INT_MAX, bi = -1;
    for (int c = t; c < nloc; c += kQThreads) {
      if (!act[c]) continue;
      double x = nrm[c];
      if (!(x == x) || x > 1.79e308) { flag_nonfinite(q.info, q.block_index); x = -0.5; }
      if (better(x, pos[c], bv, bp)) { bv = x; bp = pos[c]; bi = c; }
    }
    rv[t] = bv; rp[t] = bp; ri[t] = bi;
    block_argmax(rv, rp, ri);
    const int buf = j & 1;
    double *myrec = q.rec + ((size_t)buf * nwg + wg) * 4;
    double *mycand = q.cand + ((size_t)buf * nwg + wg) * k;
    const int lbest = ri[0];
    if (t == 0) {
      myrec[0] = rv[0];
      myrec[1] = (double)rp[0];
      myrec[2] = (double)(lbest >= 0 ? c0 + lbest : -1);
    }
    if (lbest >= 0)
      for (int r = j + t; r < k; r += kQThreads) mycand[r] = Yl[(size_t)lbest * k + r];
    ok = grid_sync(gb, gen);
    if (!ok) break;
    // global argmax over the published records (same order in every workgroup)
    {
      double gv = -1.0;
      int gp = INT_MAX, gi = -1;
      for (int w2 = t; w2 < nwg; w2 += kQThreads) {
        const double *rr = q.rec + ((size_t)buf * nwg + w2) * 4;
        const double x = rr[0];
        const int p = (int)rr[1];
        if (rr[2] >= 0.0 && better(x, p, gv, gp)) { gv = x; gp = p; gi = w2; }
      }
      rv[t] = gv; rp[t] = gp; ri[t] = gi;
      block_argmax(rv, rp, ri);
      if (t == 0) {
        s_win_wg = ri[0];
        s_win_pos = rp[0];
        s_win_col = ri[0] >= 0 ? (int)q.rec[((size_t)buf * nwg + ri[0]) * 4 + 2] : -1;
      }
      __syncthreads();
    }
    if (s_win_wg < 0) { ok = false; break; }   // no candidate left: cannot happen for nsteps <= ncols
    const int wwg = s_win_wg, wpos = s_win_pos, wcol = s_win_col;
    const double *wc = q.cand + ((size_t)buf * nwg + wwg) * k;
    for (int r = j + t; r < k; r += kQThreads) v[r] = wc[r];
    __syncthreads();
    // reflector of the winning column (Section 3.1)
    if (wave == 0) {
      double s = 0.0;
      for (int r = j + lane; r < k; r += 64) s += v[r] * v[r];
      s = wave_sum(s);
      if (lane == 0) {
        const double alpha = v[j];
        double tau = 0.0, scale = 1.0;
        if (j < k - 1 && s != 0.0) {
          const double beta = (alpha >= 0.0 ? -1.0 : 1.0) * sqrt(s);
          tau = (beta - alpha) / beta;
          scale = alpha - beta;
        }
        s_tau = tau;
        rv[0] = scale;
      }
    }
    __syncthreads();
    const double tau = s_tau;
    const double scale = rv[0];
    __syncthreads();
    if (tau != 0.0)
      for (int r = j + 1 + t; r < k; r += kQThreads) v[r] = v[r] / scale;
    if (t == 0) v[j] = 1.0;
    // bookkeeping of positions: the winner goes to j, the column at j to wpos
    for (int c = t; c < nloc; c += kQThreads) {
      if (c0 + c == wcol) { act[c] = 0; pos[c] = j; }
      else if (pos[c] == j) pos[c] = wpos;
    }
    if (wg == 0 && t == 0) q.piv[j] = wpos;
    __syncthreads();
    // apply H_j to the remaining local columns, recompute their norms
    for (int c = wave; c < nloc; c += kQWaves) {
      if (!act[c]) continue;
      double *y = Yl + (size_t)c * k;
      if (tau != 0.0) {
        double d = 0.0;
        for (int r = j + lane; r < k; r += 64) d += v[r] * y[r];
        d = wave_sum(d);
        const double f = tau * d;
        for (int r = j + lane; r < k; r += 64) y[r] -= f * v[r];
      }
      double s = 0.0;
      for (int r = j + 1 + lane; r < k; r += 64) s += y[r] * y[r];
      s = wave_sum(s);
      if (lane == 0) nrm[c] = s;
    }
  }
  if (!ok && q.info && t == 0) atomicExch(&q.info[2], 1);
  __syncthreads();
  for (int c = t; c < nloc; c += kQThreads) {
    q.dest[c0 + c] = pos[c];
    if (pos[c] != c0 + c) {
      const int slot = atomicAdd(q.moved_cnt, 1);
      if (slot < 2 * q.nsteps) q.moved[slot] = c0 + c;
    }
  }
}

template <typename T>
__global__ __launch_bounds__(256) void gather_moved_kernel(const T *__restrict__ A, int64_t lda, int64_t m,
                                                           int64_t r0, const int32_t *__restrict__ moved,
                                                           const int32_t *__restrict__ moved_cnt,
                                                           T *__restrict__ tmp,
                                                           const int32_t *__restrict__ jpvt,
                                                           int32_t *__restrict__ jtmp) {
  const int slot = blockIdx.x;
  if (slot >= *moved_cnt) return;
  const int64_t c = r0 + moved[slot];
  for (int64_t r = (int64_t)blockIdx.y * blockDim.x + threadIdx.x; r < m; r += (int64_t)gridDim.y * blockDim.x)
    tmp[r + slot * m] = A[r + c * lda];
  if (blockIdx.y == 0 && threadIdx.x == 0) jtmp[slot] = jpvt[c];
}

template <typename T>
__global__ __launch_bounds__(256) void scatter_moved_kernel(T *__restrict__ A, int64_t lda, int64_t m,
                                                            int64_t r0, const int32_t *__restrict__ moved,
                                                            const int32_t *__restrict__ moved_cnt,
                                                            const int32_t *__restrict__ dest,
                                                            const T *__restrict__ tmp,
                                                            int32_t *__restrict__ jpvt,
                                                            const int32_t *__restrict__ jtmp) {
  const int slot = blockIdx.x;
  if (slot >= *moved_cnt) return;
  const int64_t d = r0 + dest[moved[slot]];
  for (int64_t r = (int64_t)blockIdx.y * blockDim.x + threadIdx.x; r < m; r += (int64_t)gridDim.y * blockDim.x)
    A[r + d * lda] = tmp[r + slot * m];
  if (blockIdx.y == 0 && threadIdx.x == 0) jpvt[d] = jtmp[slot];
}

size_t lds_doubles(int k, int cpw) {
  return (size_t)cpw * k + cpw + k + kQThreads + (size_t)(3 * kQThreads + 2 * cpw + 1) / 2;
}

}  // namespace

int qrcp_small_config(int k, int ncols, int *cpw) {
  if (k < 1 || ncols < 1) return 0;
  int maxc = 0;
  for (int c = 1; c <= 4096; ++c) {
    if (lds_doubles(k, c) > kLdsDoubles) break;
    maxc = c;
  }
  if (maxc < 1) return 0;
  int want = (ncols + 31) / 32;   // aim for about 32 workgroups
  if (want < 1) want = 1;
  const int c = want < maxc ? want : maxc;
  const int nwg = (ncols + c - 1) / c;
  if (nwg > 256) return 0;
  *cpw = c;
  return nwg;
}

size_t qrcp_small_rec_doubles(int nwg) { return (size_t)2 * nwg * 4; }
size_t qrcp_small_cand_doubles(int nwg, int k) { return (size_t)2 * nwg * k; }

hipError_t launch_qrcp_small(hipStream_t s, const QrcpSmall &q) {
  int cpw = 0;
  const int nwg = qrcp_small_config(q.k, q.ncols, &cpw);
  if (nwg == 0) return hipErrorInvalidValue;
  static bool attr_done = false;
  if (!attr_done) {
    hipError_t e = hipFuncSetAttribute((const void *)qrcp_small_kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                                       (int)(kLdsDoubles * sizeof(double)));
    if (e != hipSuccess) return e;
    attr_done = true;
  }
  const size_t lds = lds_doubles(q.k, cpw) * sizeof(double);
  QrcpSmall qq = q;
  GridBarrier gb{q.bar, q.abort_flag, q.limit_ticks};
  void *args[] = {&qq, &cpw, &gb};
  return hipLaunchCooperativeKernel((const void *)qrcp_small_kernel, dim3(nwg), dim3(kQThreads), args,
                                    (unsigned)lds, s);
}

template <typename T>
hipError_t launch_apply_moves(hipStream_t s, T *A, int64_t lda, int64_t m, int64_t r0,
                              const int32_t *moved, const int32_t *moved_cnt, const int32_t *dest,
                              int max_moved, T *tmp, int32_t *jpvt, int32_t *jtmp) {
  if (max_moved <= 0) return hipSuccess;
  int64_t gy = (m + 1023) / 1024;
  if (gy > 64) gy = 64;
  if (gy < 1) gy = 1;
  dim3 grid((unsigned)max_moved, (unsigned)gy);
  hipLaunchKernelGGL(gather_moved_kernel<T>, grid, dim3(256), 0, s, A, lda, m, r0, moved, moved_cnt, tmp, jpvt, jtmp);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(scatter_moved_kernel<T>, grid, dim3(256), 0, s, A, lda, m, r0, moved, moved_cnt, dest, tmp, jpvt,
                     jtmp);
  return hipGetLastError();
}
template hipError_t launch_apply_moves<double>(hipStream_t, double *, int64_t, int64_t, int64_t, const int32_t *,
                                               const int32_t *, const int32_t *, int, double *, int32_t *, int32_t *);
template hipError_t launch_apply_moves<float>(hipStream_t, float *, int64_t, int64_t, int64_t, const int32_t *,
                                              const int32_t *, const int32_t *, int, float *, int32_t *, int32_t *);

}  // namespace rq
