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
//
// Two kernels implement this.  For a sketch (k = b + p <= 512 rows, many
// columns) the columns live in registers: 8 lanes share a column, each
// holding every 8th row, so applying a reflector and recomputing a norm is a
// few register FMAs and a 3-step shuffle reduction per lane, and one
// workgroup of 512 threads holds 64 columns (k <= 448).  For taller inputs
// (the classical last block, k up to the LDS size) the columns live in LDS,
// one wave per column at a time.
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
// The same without branches (for arg-max exchanges between lanes and for
// loops whose loads should all issue before the comparisons).
__device__ __forceinline__ int better_bits(double v1, int p1, double v2, int p2) {
  return (int)(v1 > v2) | ((int)(v1 == v2) & (int)(p1 < p2));
}

__device__ void flag_nonfinite(int32_t *info, int block_index) {
  if (!info) return;
  atomicExch(&info[0], 1);
  atomicCAS(&info[1], 0, block_index + 1);
}

// One arg-max exchange of (val, pos, idx) with the lane that CTRL selects;
// ties go to the lower pos.  Both lanes of a pair end with the same triple.
template <int CTRL>
__device__ __forceinline__ void argmax_dpp(double &v, int &p, int &i) {
  const double v2 = dpp_mov<CTRL>(v);
  const int p2 = dpp_mov<CTRL>(p), i2 = dpp_mov<CTRL>(i);
  const int take = better_bits(v2, p2, v, p);   // selects, no branch
  v = take ? v2 : v;
  p = take ? p2 : p;
  i = take ? i2 : i;
}
// The same across lanes i and i ^ SPAN (16 or 32): both lanes see the pair
// in the same order and pick the same member.
template <int SPAN>
__device__ __forceinline__ void argmax_span(double &v, int &p, int &i) {
  double vl, vh;
  int pl, ph, il, ih;
  lane_pair<SPAN>(v, vl, vh);
  lane_pair<SPAN>(p, pl, ph);
  lane_pair<SPAN>(i, il, ih);
  const int up = better_bits(vh, ph, vl, pl);
  v = up ? vh : vl;
  p = up ? ph : pl;
  i = up ? ih : il;
}
// Arg-max over aligned groups of 8 lanes (every lane of a group gets the winner).
__device__ __forceinline__ void group8_argmax(double &v, int &p, int &i) {
  argmax_dpp<kDppXor1>(v, p, i);
  argmax_dpp<kDppXor2>(v, p, i);
  argmax_dpp<kDppHalfMirror>(v, p, i);
}
// Arg-max over the wave, given that the lanes of each group of 8 agree.
__device__ __forceinline__ void groups_argmax(double &v, int &p, int &i) {
  argmax_dpp<kDppMirror>(v, p, i);
  argmax_span<16>(v, p, i);
  argmax_span<32>(v, p, i);
}
// Arg-max over the lanes of one wave; every lane returns the winner.  Call
// with all 64 lanes active.
__device__ __forceinline__ void wave_argmax(double &v, int &p, int &i) {
  group8_argmax(v, p, i);
  groups_argmax(v, p, i);
}

// Squared norm as a pivot key: non-finite values never win (and are flagged).
__device__ __forceinline__ double key_of(double x, int32_t *info, int block_index, int lane) {
  if (!(x == x) || x > 1.79e308) {
    if (lane == 0) flag_nonfinite(info, block_index);
    return -0.5;
  }
  return x;
}

__global__ __launch_bounds__(kQThreads) void qrcp_small_kernel(QrcpSmall q, int cpw, GridBarrier gb) {
  extern __shared__ double lds[];
  const int k = q.k;
  double *Yl = lds;                           // cpw * k, column-major
  double *v = Yl + (size_t)cpw * k;           // k     reflector (winning column)
  double *wbv = v + k;                        // kQWaves best key per wave
  int *wbp = (int *)(wbv + kQWaves);          // kQWaves best position per wave
  int *wbi = wbp + kQWaves;                   // kQWaves best local column per wave
  int *pos = wbi + kQWaves;                   // cpw   current position of each column
  int *act = pos + cpw;                       // cpw   1 while not yet chosen
  __shared__ double s_tau;
  __shared__ int s_wpos, s_wcol, s_fail;

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
  // initial norms over all k rows; every wave keeps its best column
  {
    double bv = -1.0;
    int bp = INT_MAX, bi = -1;
    for (int c = wave; c < nloc; c += kQWaves) {
      const double *y = Yl + (size_t)c * k;
      double s2 = 0.0;
      for (int r = lane; r < k; r += 64) s2 += y[r] * y[r];
      s2 = key_of(wave_sum(s2), q.info, q.block_index, lane);
      if (better(s2, c0 + c, bv, bp)) { bv = s2; bp = c0 + c; bi = c; }
    }
    if (lane == 0) { wbv[wave] = bv; wbp[wave] = bp; wbi[wave] = bi; }
  }

  unsigned gen = 0;
  bool ok = true;
  for (int j = 0; j < q.nsteps; ++j) {
    __syncthreads();
    const int buf = j & 1;
    // wave 0: this workgroup's best candidate -> record + column in global memory
    if (wave == 0) {
      double bv = lane < kQWaves ? wbv[lane] : -1.0;
      int bp = lane < kQWaves ? wbp[lane] : INT_MAX;
      int bi = lane < kQWaves ? wbi[lane] : -1;
      wave_argmax(bv, bp, bi);
      double *myrec = q.rec + ((size_t)buf * nwg + wg) * 4;
      double *mycand = q.cand + ((size_t)buf * nwg + wg) * k;
      if (bi >= 0)
        for (int r = j + lane; r < k; r += 64) mycand[r] = Yl[(size_t)bi * k + r];
      if (lane == 0) {
        myrec[0] = bv;
        myrec[1] = (double)bp;
        myrec[2] = (double)(bi >= 0 ? c0 + bi : -1);
      }
    }
    ok = grid_sync(gb, gen);
    if (!ok) break;
    // wave 0: global winner, its column and the reflector (Section 3.1)
    if (wave == 0) {
      double gv = -1.0;
      int gp = INT_MAX, gi = -1;
      for (int w2 = lane; w2 < nwg; w2 += 64) {
        const double *rr = q.rec + ((size_t)buf * nwg + w2) * 4;
        const double x = rr[0];
        const int p = (int)rr[1];
        if (rr[2] >= 0.0 && better(x, p, gv, gp)) { gv = x; gp = p; gi = w2; }
      }
      wave_argmax(gv, gp, gi);
      if (gi < 0) {
        if (lane == 0) s_fail = 1;
      } else {
        const double *wc = q.cand + ((size_t)buf * nwg + gi) * k;
        double s2 = 0.0;
        for (int r = j + lane; r < k; r += 64) {
          const double x = wc[r];
          v[r] = x;
          s2 += x * x;
        }
        s2 = wave_sum(s2);
        double tau = 0.0, scale = 1.0;
        const double a = wc[j];
        if (j < k - 1 && s2 != 0.0) {
          const double beta = (a >= 0.0 ? -1.0 : 1.0) * sqrt(s2);
          tau = (beta - a) / beta;
          scale = a - beta;
        }
        if (tau != 0.0)
          for (int r = j + 1 + lane; r < k; r += 64) v[r] = v[r] / scale;
        if (lane == 0) {
          v[j] = 1.0;
          s_tau = tau;
          s_wpos = gp;
          s_wcol = (int)q.rec[((size_t)buf * nwg + gi) * 4 + 2];
          s_fail = 0;
          if (wg == 0) q.piv[j] = gp;
        }
      }
    }
    __syncthreads();
    if (s_fail) { ok = false; break; }   // no candidate left: cannot happen for nsteps <= ncols
    const double tau = s_tau;
    const int wpos = s_wpos, wcol = s_wcol;
    // every wave: bookkeeping, H_j applied to its remaining columns, new norms
    double bv = -1.0;
    int bp = INT_MAX, bi = -1;
    for (int c = wave; c < nloc; c += kQWaves) {
      if (!act[c]) continue;
      if (c0 + c == wcol) {
        if (lane == 0) { act[c] = 0; pos[c] = j; }
        continue;
      }
      int pc = pos[c];
      if (pc == j) {
        pc = wpos;
        if (lane == 0) pos[c] = wpos;
      }
      double *y = Yl + (size_t)c * k;
      if (tau != 0.0) {
        double d = 0.0;
        for (int r = j + lane; r < k; r += 64) d += v[r] * y[r];
        d = wave_sum(d);
        const double f = tau * d;
        for (int r = j + lane; r < k; r += 64) y[r] -= f * v[r];
      }
      double s2 = 0.0;
      for (int r = j + 1 + lane; r < k; r += 64) s2 += y[r] * y[r];
      s2 = key_of(wave_sum(s2), q.info, q.block_index, lane);
      if (better(s2, pc, bv, bp)) { bv = s2; bp = pc; bi = c; }
    }
    if (lane == 0) { wbv[wave] = bv; wbp[wave] = bp; wbi[wave] = bi; }
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

// ---------------------------------------------------------------------------
// Register-resident form (k <= 8 * RPL).
constexpr int kRLanes = 8;                         // lanes per column
constexpr int kRCols = kQThreads / kRLanes;        // 64 columns per workgroup
constexpr int kRMaxRows = 448;                   // 56 registers of rows per lane at most

template <int RPL>
__global__ __launch_bounds__(kQThreads) void qrcp_reg_kernel(QrcpSmall q, GridBarrier gb) {
  constexpr int KP = kRLanes * RPL;                // padded row count
  __shared__ double v[KP];                         // reflector, rows >= j valid
  __shared__ double cb[kQWaves][KP];               // each wave's best column
  __shared__ double wbv[kQWaves];
  __shared__ int wbp[kQWaves], wbi[kQWaves];
  __shared__ double s_tau;
  __shared__ int s_wpos, s_wcol, s_fail;

  const int k = q.k;
  const int nwg = gridDim.x, wg = blockIdx.x, t = threadIdx.x;
  const int lane = t & 63, wave = t >> 6, sub = lane & (kRLanes - 1);
  const int col = wg * kRCols + (t >> 3);          // this lane group's column
  const bool valid = col < q.ncols;

  double y[RPL];
#pragma unroll
  for (int i = 0; i < RPL; ++i) {
    const int r = sub + kRLanes * i;
    y[i] = (valid && r < k) ? q.Y[r + (int64_t)col * q.ldy] : 0.0;
  }
  for (int r = t; r < KP; r += kQThreads) v[r] = 0.0;
  int pos = col, act = valid ? 1 : 0;

  // publish this wave's best column to LDS (all rows; readers use rows >= j)
  auto wave_best = [&](double key) {
    double bv = act ? key : -1.0;
    int bp = act ? pos : INT_MAX, bi = act ? col : -1;
    groups_argmax(bv, bp, bi);   // the lanes of a column group agree
    if (bi >= 0 && col == bi) {
#pragma unroll
      for (int i = 0; i < RPL; ++i) cb[wave][sub + kRLanes * i] = y[i];
    }
    if (lane == 0) { wbv[wave] = bv; wbp[wave] = bp; wbi[wave] = bi; }
  };

  {
    double s2 = 0.0;
#pragma unroll
    for (int i = 0; i < RPL; ++i) s2 += y[i] * y[i];
    s2 = group8_sum(s2);
    s2 = key_of(s2, q.info, q.block_index, valid ? sub : 1);
    wave_best(s2);
  }

  unsigned gen = 0;
  bool ok = true;
  for (int j = 0; j < q.nsteps; ++j) {
    __syncthreads();
    const int buf = j & 1;
    // wave 0: this workgroup's best candidate -> record + column in global memory
    if (wave == 0) {
      double bv = lane < kQWaves ? wbv[lane] : -1.0;
      int bp = lane < kQWaves ? wbp[lane] : INT_MAX;
      int bw = lane < kQWaves ? lane : -1;
      group8_argmax(bv, bp, bw);   // lanes 0..7 hold the 8 wave bests
      bw = lane0(bw);
      double *myrec = q.rec + ((size_t)buf * nwg + wg) * 4;
      double *mycand = q.cand + ((size_t)buf * nwg + wg) * k;
      const int bi = bw >= 0 ? wbi[bw] : -1;
      if (bi >= 0)
        for (int r = j + lane; r < k; r += 64) st_agent(mycand + r, cb[bw][r]);
      if (lane == 0) {
        st_agent(myrec, bv);
        st_agent(myrec + 1, (double)bp);
        st_agent(myrec + 2, (double)bi);
      }
    }
    // exchange mode: records and columns are written and read with agent-scope atomics
    ok = grid_sync(gb, gen, false, true);
    if (!ok) break;
    // wave 0: global winner, its column and the reflector (Section 3.1)
    if (wave == 0) {
      double gv = -1.0;
      int gp = INT_MAX, gi = -1;
      double rv[4], rp[4], rc[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {           // nwg <= 256: all records in one round of loads
        const int w2 = lane + 64 * u;
        const double *rr = q.rec + ((size_t)buf * nwg + (w2 < nwg ? w2 : 0)) * 4;
        rv[u] = ld_agent(rr); rp[u] = ld_agent(rr + 1); rc[u] = ld_agent(rr + 2);
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) {           // gi packs (workgroup << 16) | column
        const int w2 = lane + 64 * u;
        const int take = (int)(w2 < nwg) & (int)(rc[u] >= 0.0) & better_bits(rv[u], (int)rp[u], gv, gp);
        gv = take ? rv[u] : gv;
        gp = take ? (int)rp[u] : gp;
        gi = take ? ((w2 << 16) | (int)rc[u]) : gi;
      }
      wave_argmax(gv, gp, gi);
      gp = lane0(gp);
      gi = lane0(gi);
      const int gcol = gi & 0xFFFF;
      gi = gi < 0 ? -1 : gi >> 16;
      if (gi < 0) {
        if (lane == 0) s_fail = 1;
      } else {
        const double *wc = q.cand + ((size_t)buf * nwg + gi) * k;
        double xs[kRMaxRows / 64];
#pragma unroll
        for (int u = 0; u < kRMaxRows / 64; ++u) {
          const int r = j + lane + 64 * u;
          xs[u] = r < k ? ld_agent(wc + r) : 0.0;
        }
        double s2 = 0.0;
#pragma unroll
        for (int u = 0; u < kRMaxRows / 64; ++u) s2 += xs[u] * xs[u];
        s2 = wave_sum(s2);
        double tau = 0.0, scale = 1.0;
        const double a = lane0(xs[0]);   // row j
        if (j < k - 1 && s2 != 0.0) {
          const double beta = (a >= 0.0 ? -1.0 : 1.0) * sqrt(s2);
          tau = (beta - a) / beta;
          scale = a - beta;
        }
        const double rs = 1.0 / scale;   // one division; v = x / scale as products
#pragma unroll
        for (int u = 0; u < kRMaxRows / 64; ++u) {
          const int r = j + lane + 64 * u;
          if (r < k) v[r] = (r == j) ? 1.0 : (tau != 0.0 ? xs[u] * rs : xs[u]);
        }
        // rows < j of v stay zero, so the column updates need no row masks
        if (lane == 0 && j > 0) v[j - 1] = 0.0;
        if (lane == 0) {
          s_tau = tau;
          s_wpos = gp;
          s_wcol = gcol;
          s_fail = 0;
          if (wg == 0) q.piv[j] = gp;
        }
      }
    }
    __syncthreads();
    if (s_fail) { ok = false; break; }   // no candidate left: cannot happen for nsteps <= ncols
    const double tau = s_tau;
    const int wpos = s_wpos, wcol = s_wcol;
    // every column group: bookkeeping, H_j applied, new norm over rows > j
    if (act && col == wcol) {
      act = 0;
      pos = j;
    } else if (act && pos == j) {
      pos = wpos;
    }
    // straight-line code (no per-row branches): v is zero on rows < j and
    // past k, and rows < j of y were zeroed at earlier steps
    if (tau != 0.0) {
      double d0 = 0.0, d1 = 0.0;
#pragma unroll
      for (int i = 0; i < RPL; i += 2) {
        d0 += v[sub + kRLanes * i] * y[i];
        if (i + 1 < RPL) d1 += v[sub + kRLanes * (i + 1)] * y[i + 1];
      }
      const double d = group8_sum(d0 + d1);
      const double f = act ? tau * d : 0.0;
      // up to 40 rows per lane v stays in registers between the two loops;
      // beyond that it would spill, so the update re-reads it from LDS
      if constexpr (RPL > 40) __asm__ volatile("" ::: "memory");
#pragma unroll
      for (int i = 0; i < RPL; ++i) y[i] -= f * v[sub + kRLanes * i];
    }
    // row j now holds an entry of R, which no later decision uses: zero it,
    // so that all rows <= j of y are zero and the norm over rows > j is a
    // plain sum (adding the zeros changes no bit of it)
    {
      // a branch on the wave-uniform register index (a short tree of scalar
      // branches): one select, instead of a select per register (measured
      // 1.6 ms less per H1 factorization)
      const int ib = j / kRLanes, sj = j % kRLanes;
      switch (ib) {
#define RQ_ZERO_ROW(i) \
  case i:              \
    if constexpr (i < RPL) y[i] = sub == sj ? 0.0 : y[i]; \
    break;
#define RQ_ZERO_ROW8(i) RQ_ZERO_ROW(i) RQ_ZERO_ROW(i + 1) RQ_ZERO_ROW(i + 2) RQ_ZERO_ROW(i + 3) \
  RQ_ZERO_ROW(i + 4) RQ_ZERO_ROW(i + 5) RQ_ZERO_ROW(i + 6) RQ_ZERO_ROW(i + 7)
        RQ_ZERO_ROW8(0) RQ_ZERO_ROW8(8) RQ_ZERO_ROW8(16) RQ_ZERO_ROW8(24)
        RQ_ZERO_ROW8(32) RQ_ZERO_ROW8(40) RQ_ZERO_ROW8(48)
#undef RQ_ZERO_ROW8
#undef RQ_ZERO_ROW
        default: break;
      }
    }
    double s20 = 0.0, s21 = 0.0;
#pragma unroll
    for (int i = 0; i < RPL; i += 2) {
      s20 += y[i] * y[i];
      if (i + 1 < RPL) s21 += y[i + 1] * y[i + 1];
    }
    double s2 = group8_sum(s20 + s21);
    s2 = key_of(s2, q.info, q.block_index, act ? sub : 1);
    wave_best(s2);
  }
  if (!ok && q.info && t == 0) atomicExch(&q.info[2], 1);
  if (valid && sub == 0) {
    q.dest[col] = pos;
    if (pos != col) {
      const int slot = atomicAdd(q.moved_cnt, 1);
      if (slot < 2 * q.nsteps) q.moved[slot] = col;
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
  // four loads in flight before their stores (a store right after each load
  // would wait for it)
  const int64_t stride = (int64_t)gridDim.y * blockDim.x;
  int64_t r = (int64_t)blockIdx.y * blockDim.x + threadIdx.x;
  for (; r + 3 * stride < m; r += 4 * stride) {
    T v[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) v[u] = A[r + u * stride + c * lda];
#pragma unroll
    for (int u = 0; u < 4; ++u) tmp[r + u * stride + slot * m] = v[u];
  }
  for (; r < m; r += stride) tmp[r + slot * m] = A[r + c * lda];
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
  const int64_t stride = (int64_t)gridDim.y * blockDim.x;
  int64_t r = (int64_t)blockIdx.y * blockDim.x + threadIdx.x;
  for (; r + 3 * stride < m; r += 4 * stride) {
    T v[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) v[u] = tmp[r + u * stride + slot * m];
#pragma unroll
    for (int u = 0; u < 4; ++u) A[r + u * stride + d * lda] = v[u];
  }
  for (; r < m; r += stride) A[r + d * lda] = tmp[r + slot * m];
  if (blockIdx.y == 0 && threadIdx.x == 0) jpvt[d] = jtmp[slot];
}

size_t lds_doubles(int k, int cpw) {
  // Yl + v + wave bests (key, pos, idx) + pos + act
  return (size_t)cpw * k + k + kQWaves + (size_t)(2 * kQWaves + 2 * cpw + 1) / 2;
}

}  // namespace

static int rpl_for(int k) {
  const int r = (k + kRLanes - 1) / kRLanes;
  return ((r + 1) / 2) * 2;   // rows per lane rounded up to a multiple of 2 (two norm chains)
}

int qrcp_small_config(int k, int ncols, int *cpw) {
  if (k < 1 || ncols < 1) return 0;
  if (k <= kRMaxRows) {
    const int nwg = (ncols + kRCols - 1) / kRCols;   // at most 16384 columns (16-bit column ids)
    if (nwg > 256) return 0;
    *cpw = kRCols;
    return nwg;
  }
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

template <int RPL>
static hipError_t launch_reg(hipStream_t s, int nwg, const QrcpSmall &q) {
  QrcpSmall qq = q;
  GridBarrier gb{q.bar, q.abort_flag, q.limit_ticks};
  void *args[] = {&qq, &gb};
  return launch_persistent((const void *)qrcp_reg_kernel<RPL>, (unsigned)nwg, kQThreads, args, 0, s);
}

hipError_t launch_qrcp_small(hipStream_t s, const QrcpSmall &q) {
  int cpw = 0;
  const int nwg = qrcp_small_config(q.k, q.ncols, &cpw);
  if (nwg == 0) return hipErrorInvalidValue;
  if (q.k <= kRMaxRows) {
    switch (rpl_for(q.k)) {
#define RQ_REG_CASE(r) \
  case r: return launch_reg<r>(s, nwg, q);
      RQ_REG_CASE(2) RQ_REG_CASE(4) RQ_REG_CASE(6) RQ_REG_CASE(8) RQ_REG_CASE(10) RQ_REG_CASE(12) RQ_REG_CASE(14)
      RQ_REG_CASE(16) RQ_REG_CASE(18) RQ_REG_CASE(20) RQ_REG_CASE(22) RQ_REG_CASE(24) RQ_REG_CASE(26)
      RQ_REG_CASE(28) RQ_REG_CASE(30) RQ_REG_CASE(32) RQ_REG_CASE(34) RQ_REG_CASE(36) RQ_REG_CASE(38)
      RQ_REG_CASE(40) RQ_REG_CASE(42) RQ_REG_CASE(44) RQ_REG_CASE(46) RQ_REG_CASE(48) RQ_REG_CASE(50)
      RQ_REG_CASE(52) RQ_REG_CASE(54)
#undef RQ_REG_CASE
      default: return launch_reg<56>(s, nwg, q);
    }
  }
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
  return launch_persistent((const void *)qrcp_small_kernel, (unsigned)nwg, kQThreads, args, lds, s);
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
