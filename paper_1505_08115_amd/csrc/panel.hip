// Unpivoted Householder QR of the m' x b panel (Fig. 3, the panel step with
// P-hat = I; Sections 3.1-3.2) and the T factor of its compact WY form
// (Section 5.1: H_1 ... H_b = I - V T V^T).
//
// One persistent cooperative launch per panel.  Panel rows are dealt in
// contiguous ranges of rpw rows to workgroups; a workgroup only ever touches
// its own rows, so all cross-workgroup traffic is the reductions.  Columns
// are processed in slabs of kPanelW that live in LDS:
//   * column step j: every workgroup forms partial sums over its rows of
//     g_c = x_j^T x_c (rows >= j) and contributes x_c(j) (owner only), for the
//     remaining slab columns c >= j; one grid barrier; every workgroup sums
//     the partials in the same fixed order.  With alpha = x_j(j),
//     beta = -sign(alpha) |x_j|, tau = (beta - alpha)/beta and
//     v = (x_j - beta e_j)/(alpha - beta), the reflector's action on column c
//     follows from the reduced sums alone: v^T x_c = (g_c - beta x_c(j)) /
//     (alpha - beta).  Degenerate columns follow the conventions of the
//     oracle: tau = 0 for a zero column or a column of length one.  Up to
//     kG = 8 columns share one exchange: the reflectors leave inner products
//     over rows >= j unchanged, so the sums of x_{j+u}^T x_c and the entries
//     of rows j .. j+7 determine all eight reflectors and their action.
//   * after a slab: the partial products V_s^T [V_s | A_rest] are
//     reduce-scattered (two barriers); they give the slab's Gram block
//     V_s^T V_s for its T_s and W = V_s^T A_rest, which updates the rest of
//     the panel as A_rest <- A_rest - V_s (T_s^T W).  (The Gram matrix V^T V
//     of the whole panel, which the T factor needs, is a product of the
//     explicit V formed outside the kernel.)
#include <type_traits>

#include "common.h"

namespace rq {

namespace {

constexpr int W = kPanelW;
typedef double d4 __attribute__((ext_vector_type(4)));
constexpr int kPThreads = 256;
constexpr size_t kLdsDoubles = 20480 - 256;
constexpr int kG = 8;                       // columns per exchange in a column step
constexpr int kGW = kG * W;                 // sums (or row entries) per exchange
constexpr int kNH = kPThreads / kGW;        // workgroup sets in the reduction of the sums
constexpr int kLd = (64 + kNH - 1) / kNH;   // loads in flight per thread in that reduction
static_assert(kPThreads % kGW == 0 && 2 * kGW % 64 == 0, "column-step layout");

// lane l's value in every lane (l wave-uniform)
__device__ __forceinline__ double lane_d(double x, int l) {
  return __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(x), l), __builtin_amdgcn_readlane(__double2loint(x), l));
}

__device__ void flag_nonfinite(int32_t *info, int block_index) {
  if (!info) return;
  atomicExch(&info[0], 1);
  atomicCAS(&info[1], 0, block_index + 1);
}

__global__ __launch_bounds__(kPThreads) void panel_qr_kernel(PanelQR p, int rpw, GridBarrier gb) {
  extern __shared__ double lds[];
  __shared__ double sc_st[5 * kGW + W];     // a separate array: its accesses never alias the slab's
  const int nb = p.nb;
  const int rpw4 = (rpw + 3) & ~3;           // rows padded to the MFMA K step
  const int ldx = rpw4 + 1;                 // odd stride: the 16 lanes of a fragment hit distinct banks
  double *X = lds;                          // W x ldx   slab (own rows), column c at X + c*ldx
  double *Wp = X + (size_t)W * ldx;         // W x nb    reduced V_s^T [V_s | A_rest], row t at Wp + t*nb (columns >= cs)
  double *Ts = Wp + (size_t)W * nb;         // W x W     column-major
  double *sc = sc_st;                       // 5 kGW     reduction scratch
  double *taus = sc + 5 * kGW;              // W

  const int nwg = gridDim.x, wg = blockIdx.x, t = threadIdx.x;
  const int64_t rbeg = (int64_t)wg * rpw;
  const int nrow = (int)max((int64_t)0, min((int64_t)rpw, p.mi - rbeg));
  const int nslab = (nb + W - 1) / W;
  double *part_cs = p.part;                                   // [2][nwg][2 kGW]
  double *part_up = p.part + (size_t)2 * nwg * 2 * kGW;       // [nwg][W*nb]
  unsigned gen = 0;
  bool ok = true;
  int step = 0;

  for (int s = 0; s < nslab && ok; ++s) {
    const int cs = s * W, ws = min(W, nb - cs);
    // eight entries per thread are loaded before any is written to LDS, so
    // the loads are in flight together: a write after each load would wait
    // for it, one memory latency per entry.  Indices are clamped into the
    // slab and the writes are unconditional (a load behind a bounds branch is
    // sunk into it and waits again): past the end, a lane writes the last
    // entry's own value to it once more.
    for (int base = 0, tot = ws * nrow; base < tot; base += 8 * kPThreads) {
      double v[8];
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        const int idx = min(base + t + q * kPThreads, tot - 1), c = idx / nrow, r = idx % nrow;
        v[q] = p.P[(rbeg + r) + (int64_t)(cs + c) * p.ldp];
      }
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        const int idx = min(base + t + q * kPThreads, tot - 1);
        X[(idx / nrow) * ldx + idx % nrow] = v[q];
      }
    }
    // pad rows (nrow .. rpw4) and absent columns (ws .. W) read as zero in the MFMA products
    for (int idx = t; idx < W * (rpw4 - nrow); idx += kPThreads) {
      const int c = idx / (rpw4 - nrow), r = nrow + idx % (rpw4 - nrow);
      X[c * ldx + r] = 0.0;
    }
    for (int idx = t; idx < (W - ws) * nrow; idx += kPThreads) {
      const int c = ws + idx / nrow, r = idx % nrow;
      X[c * ldx + r] = 0.0;
    }
    __syncthreads();
    for (int jj = 0; jj < ws && ok; ++step) {
      const int64_t j = cs + jj;
      const int E = ws - jj;
      const int buf = step & 1;
      // Up to kG columns jj, jj+1, ... share one exchange; column jj+u joins
      // only if it lies in the slab and keeps at least two rows from its
      // diagonal down.  H_j ... H_{j+u-1} act orthogonally on rows >= j, so
      // inner products of transformed columns over those rows are the sums of
      // the original columns: every reflector of the group and its action on
      // the slab follow from the sums over rows >= j of x_{jj+u}^T x_c and the
      // entries of rows j .. j+kG-1.
      const int gc = (int)max((int64_t)1, min((int64_t)min(kG, E), p.mi - j - 1));
      // partial sums over own rows >= j: Gm at sc[u*W + c - jj] (u < kG) and
      // the row entries h at sc[kGW + s*W + c - jj], Gm_u,c = x_{jj+u}^T x_c,
      // h_s,c = x_c(j + s)
      {
        // straight-line passes over 4 rows (the loads first); a column past
        // the slab or the group reads column W - 1 (its sums are not kept) and
        // rows past nrow count as zero
        const int c = jj + (t >> 3), sub = t & 7;
        const int cx = min(c, W - 1) * ldx;
        int gx[kG];
#pragma unroll
        for (int u = 0; u < kG; ++u) gx[u] = min(jj + u, W - 1) * ldx;
        double g[kG];
#pragma unroll
        for (int u = 0; u < kG; ++u) g[u] = 0.0;
        for (int r = (int)max((int64_t)0, j - rbeg) + sub; r < nrow; r += 32) {
          double xc[4], xg[4][kG];
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            const int ri = min(r + 8 * i, nrow - 1);
            xc[i] = X[cx + ri];
#pragma unroll
            for (int u = 0; u < kG; ++u) xg[i][u] = X[gx[u] + ri];
          }
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            const double xi = r + 8 * i < nrow ? xc[i] : 0.0;
#pragma unroll
            for (int u = 0; u < kG; ++u) g[u] += xg[i][u] * xi;
          }
        }
#pragma unroll
        for (int u = 0; u < kG; ++u) g[u] = group8_sum(g[u]);
        if (sub == 0 && c < ws) {
#pragma unroll
          for (int u = 0; u < kG; ++u) {
            const int64_t row = j + u;
            sc[u * W + (c - jj)] = g[u];
            sc[kGW + u * W + (c - jj)] = (row >= rbeg && row < rbeg + nrow) ? X[cx + (int)(row - rbeg)] : 0.0;
          }
        }
        __syncthreads();
        // wave 0 publishes this workgroup's values
        if (t < 64) {
#pragma unroll
          for (int q = 0; q < 2 * kGW / 64; ++q) {
            const int e = t + 64 * q;
            if (e % W < E && (e / W) % kG < gc) st_agent(part_cs + ((size_t)buf * nwg + wg) * 2 * kGW + e, sc[e]);
          }
        }
      }
      // exchange mode: the partials are written and read with agent-scope atomics
      ok = grid_sync(gb, gen, false, true);
      if (!ok) break;
      // fixed-order reduction of the sums Gm: kNH sets of workgroups (w mod
      // kNH), each summed in workgroup order, then the sets in order; thread
      // (set, e) sums entry e.  The row entries h are read once, from the
      // workgroups owning rows j .. j + gc - 1 (every other workgroup's are zero).
      {
        const int e = t % kGW, set = t / kGW;
        const bool live = e % W < E && e / W < gc;
        double acc = 0.0;
        // kLd loads in flight per thread (one round trip at 64 workgroups)
        for (int w0 = set; w0 < nwg; w0 += kNH * kLd) {
          double x[kLd];
#pragma unroll
          for (int u = 0; u < kLd; ++u) {
            const int w2 = w0 + kNH * u;
            const double *src = part_cs + ((size_t)buf * nwg + (w2 < nwg ? w2 : 0)) * 2 * kGW;
            x[u] = (live && w2 < nwg) ? ld_agent(src + e) : 0.0;
          }
#pragma unroll
          for (int u = 0; u < kLd; ++u) acc += x[u];
        }
        if (set == kNH - 1) {
          double h = 0.0;
          if (live) {
            const int owner = (int)((j + e / W) / rpw);
            h = ld_agent(part_cs + ((size_t)buf * nwg + owner) * 2 * kGW + kGW + e);
          }
          sc[kGW + e] = h;
        }
        sc[2 * kGW + set * kGW + e] = acc;
        __syncthreads();
        if (t < kGW) {
          double s = sc[2 * kGW + t];
#pragma unroll
          for (int q = 1; q < kNH; ++q) s += sc[2 * kGW + q * kGW + t];
          sc[t] = s;
        }
        __syncthreads();
      }
      // Every thread forms the group's reflectors from the reduced sums itself
      // (the same operations on the same LDS values, so all threads agree bit
      // for bit): no serial section and no barrier before the column factors.
      // Column u after H_j ... H_{j+u-1}: its entries on rows j .. j+u-1 are R
      // entries, and its inner product with a column c over rows >= j+u is
      // Gm_u,c minus the products of their R entries on those rows.  Each
      // thread carries the group's columns (zg) and, beside them, column
      // jj + t (zc), whose factors f_tt = tau_tt v_tt^T (H_{j+tt-1} ... H_j x_c)
      // go to sc[4 kGW + tt*W + t]; a factor is zero where reflector tt does
      // not act (tt at or past the group's end, or column jj + t at or before
      // jj + tt), so the row updates below apply all kG reflectors blindly.
      double bet[kG], tau[kG], rsv[kG];
      int ng = 1;
      {
        // Lane l of every 8-lane group keeps group column l & 7 (its entries
        // zo on rows j .. j+kG-1 and its sums gmo); reflector tt's data come
        // from lane tt by readlane, so a lane updates only its own group
        // column instead of all of them.  Every lane then takes the same
        // decisions from the same broadcast values.
        const int tc = min(t, W - 1), gl = t & 7;
        double zo[kG], gmo[kG], zc[kG], gmc[kG], vq[kG], rr[kG];
#pragma unroll
        for (int s2 = 0; s2 < kG; ++s2) {
          zc[s2] = sc[kGW + s2 * W + tc];
          gmc[s2] = sc[s2 * W + tc];
          zo[s2] = sc[kGW + s2 * W + gl];
          gmo[s2] = sc[s2 * W + gl];
        }
        bool open = true;
#pragma unroll
        for (int tt = 0; tt < kG; ++tt) {
          // reflector tt from column tt after the earlier ones (lane tt's copy)
          double pz[kG];
#pragma unroll
          for (int s2 = 0; s2 < kG; ++s2) pz[s2] = lane_d(zo[s2], tt);
          const double guu = lane_d(gmo[tt], tt);
          bool act;
          double scale;
          if (tt == 0) {
            const double alpha = pz[0], nrm2 = guu;
            bet[0] = alpha;
            tau[0] = 0.0;
            scale = 1.0;
            if (j < p.mi - 1) {
              if (nrm2 != 0.0) {
                bet[0] = (alpha >= 0.0 ? -1.0 : 1.0) * sqrt(nrm2);
                tau[0] = (bet[0] - alpha) / bet[0];
                scale = alpha - bet[0];
              } else {
                bet[0] = 0.0;
              }
            }
            act = true;
            open = tau[0] != 0.0;
            if (t == 0 && (!(nrm2 == nrm2) || nrm2 > 1.79e308)) flag_nonfinite(p.info, p.block_index);
          } else {
            // column tt joins while its norm over rows >= j+tt, Gm_tt,tt minus
            // the squares of its R entries, keeps more than half of Gm_tt,tt
            // (relative error below 2 u); otherwise it takes a step of its own
            double nrm = guu;
#pragma unroll
            for (int s2 = 0; s2 < tt; ++s2) nrm -= pz[s2] * pz[s2];
            act = open && tt < gc && guu > 0.0 && guu < 1.79e308 && nrm > 0.5 * guu;
            open = act;
            const double y = pz[tt];
            const double b = (y >= 0.0 ? -1.0 : 1.0) * sqrt(act ? nrm : 1.0);
            bet[tt] = act ? b : 0.0;
            tau[tt] = act ? (b - y) / b : 0.0;
            scale = act ? y - b : 1.0;
            if (act) ng = tt + 1;
          }
          // v = (x - beta e_j) / scale is formed as a product with 1/scale (one
          // division per thread instead of one per use)
          rsv[tt] = 1.0 / scale;
#pragma unroll
          for (int s2 = 0; s2 < kG; ++s2) {
            rr[s2] = s2 < tt ? pz[s2] : 0.0;
            vq[s2] = s2 > tt ? pz[s2] * rsv[tt] : 0.0;
          }
          // reflector tt on this lane's group column (when it lies past tt)
          // and on column jj + t
          {
            double ip = gmo[tt];
#pragma unroll
            for (int s2 = 0; s2 < tt; ++s2) ip -= rr[s2] * zo[s2];
            double f = tau[tt] * ((ip - bet[tt] * zo[tt]) * rsv[tt]);
            f = act && gl > tt ? f : 0.0;
            zo[tt] -= f;
#pragma unroll
            for (int s2 = tt + 1; s2 < kG; ++s2) zo[s2] -= f * vq[s2];
          }
          {
            double ip = gmc[tt];
#pragma unroll
            for (int s2 = 0; s2 < tt; ++s2) ip -= rr[s2] * zc[s2];
            double f = tau[tt] * ((ip - bet[tt] * zc[tt]) * rsv[tt]);
            f = act && t > tt ? f : 0.0;
            if (t < W) sc[4 * kGW + tt * W + t] = f;
            zc[tt] -= f;
#pragma unroll
            for (int s2 = tt + 1; s2 < kG; ++s2) zc[s2] -= f * vq[s2];
          }
        }
      }
      if (t == 0) {
#pragma unroll
        for (int u = 0; u < kG; ++u)
          if (u < ng) {
            taus[jj + u] = tau[u];
            if (wg == 0) p.tau[j + u] = tau[u];
          }
      }
      // Row updates: G threads per row (G = 1 when a workgroup has more than
      // 128 rows; then a thread takes rows t and t + 256, rpw being below
      // 512), thread (r, g) takes the columns c = jj + 1 + g, jj + 1 + g + G,
      // ...  The group columns' entries of the row are read before the
      // barrier: their owners overwrite them with R entries and reflectors.
      const int G = max(1, min(kPThreads / max(nrow, 1), 8));
      const int nitem = nrow * G;
      double xg[2][kG];
#pragma unroll
      for (int q = 0; q < 2; ++q) {
        const int idx = t + q * kPThreads, r = idx % max(nrow, 1);
#pragma unroll
        for (int u = 0; u < kG; ++u) xg[q][u] = X[min(jj + u, W - 1) * ldx + r];
      }
      __syncthreads();
#pragma unroll
      for (int q = 0; q < 2; ++q) {
        const int idx = t + q * kPThreads;
        if (idx >= nitem) continue;
        const int r = idx % nrow, ug = idx / nrow;
        const int64_t rg = rbeg + r;
        if (rg < j) continue;
        // the row's reflector entries a[u] = v_{j+u}(r): zero above row j+u
        // and past the group, one on row j+u, and below it the row's entry of
        // column jj+u after the earlier reflectors of the group, times 1/scale
        double a[kG];
        if (rg == j) {
          a[0] = tau[0] != 0.0 ? 1.0 : 0.0;
          if (ug == 0) X[jj * ldx + r] = bet[0];
        } else if (tau[0] != 0.0) {
          a[0] = xg[q][0] * rsv[0];
          if (ug == 0) X[jj * ldx + r] = a[0];
        } else {
          a[0] = 0.0;
        }
#pragma unroll
        for (int u = 1; u < kG; ++u) {
          double y = xg[q][u];
#pragma unroll
          for (int tt = 0; tt < u; ++tt) y -= sc[4 * kGW + tt * W + u] * a[tt];
          a[u] = u >= ng || rg < j + u ? 0.0 : (rg == j + u ? 1.0 : y * rsv[u]);
        }
        // four columns at a time: loads first (clamped to the slab), then
        // the updates x_c -= f_tt,c a[tt] in the order of the column-by-column
        // form, then the stores; a group column takes its R entry on its
        // diagonal row and its reflector below it
        for (int c0 = jj + 1 + ug; c0 < ws; c0 += 4 * G) {
          double xv[4], fv[kG][4];
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            const int c = min(c0 + i * G, ws - 1);
            xv[i] = X[c * ldx + r];
#pragma unroll
            for (int tt = 0; tt < kG; ++tt) fv[tt][i] = sc[4 * kGW + tt * W + c - jj];
          }
#pragma unroll
          for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int tt = 0; tt < kG; ++tt) xv[i] -= fv[tt][i] * a[tt];
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            const int c = c0 + i * G, u = c - jj;
            if (c >= ws) continue;
            double out = xv[i];
#pragma unroll
            for (int uu = 1; uu < kG; ++uu)
              if (uu == u && uu < ng && rg >= j + uu) out = rg == j + uu ? bet[uu] : a[uu];
            X[c * ldx + r] = out;
          }
        }
      }
      __syncthreads();
      jj += ng;
    }
    if (!ok) break;
    // write the slab back (R and the stored vectors) and the explicit V;
    // then turn X into the explicit unit-lower V_s
    for (int idx = t; idx < ws * nrow; idx += kPThreads) {
      const int c = idx / nrow, r = idx % nrow;
      const int64_t rg = rbeg + r, jc = cs + c;
      const double x = X[c * ldx + r];
      p.P[rg + jc * p.ldp] = x;
      const double ve = rg > jc ? x : (rg == jc ? 1.0 : 0.0);
      p.V[rg + jc * p.ldv] = ve;
    }
    // V^T rows (slab columns fastest: 32 contiguous values per row), then X <- explicit V_s
    if (p.VT) {
      __syncthreads();
      for (int idx = t; idx < ws * nrow; idx += kPThreads) {
        const int c = idx % ws, r = idx / ws;
        const int64_t rg = rbeg + r, jc = cs + c;
        const double x = X[c * ldx + r];
        p.VT[jc + rg * p.ldvt] = rg > jc ? x : (rg == jc ? 1.0 : 0.0);
      }
    }
    __syncthreads();
    for (int idx = t; idx < ws * nrow; idx += kPThreads) {
      const int c = idx / nrow, r = idx % nrow;
      const int64_t rg = rbeg + r, jc = cs + c;
      const double x = X[c * ldx + r];
      X[c * ldx + r] = rg > jc ? x : (rg == jc ? 1.0 : 0.0);
    }
    __syncthreads();
    // partial products V_s^T Z over own rows, Z = [V_s | A_rest] (columns
    // cs .. nb), on the matrix cores (v_mfma_f64_16x16x4: A[i][k] from lane
    // i + 16k, B[k][j] from lane j + 16k, D[i][j] in lane j + 16 (i%4),
    // register i/4).  Wave w owns the 16-column blocks cs/16 + w, + 4, ... of
    // the 32 x (nb - cs) output; its lanes load Z straight from V (the slab's
    // explicit V written above) or P (A_rest), up to 32 loads in flight;
    // V_s^T comes from LDS.  Batches have a fixed size (32, 16, ...,
    // 1 steps of K), so the loads and MFMAs of a batch are straight-line code.
    const int nz = nb - cs;   // columns of Z = [V_s | A_rest]
    double *mypart = part_up + (size_t)wg * W * nb;
    const int lane = t & 63, wave = t >> 6, li = lane & 15, lk = lane >> 4;
    {
      const int nbk = (nb + 15) / 16, KS = rpw4 / 4, nr1 = max(nrow - 1, 0);
      for (int jb = cs / 16 + wave; jb < nbk; jb += kPThreads / 64) {
        const int col = 16 * jb + li;
        // columns past nb load column nb - 1 (their outputs are never stored);
        // a workgroup without rows loads row 0 of P (its X is all zero)
        const int cl = min(col, nb - 1);
        const double *src = nrow == 0 ? p.P
                                      : (cl < cs + ws ? p.V + rbeg + (int64_t)cl * p.ldv
                                                      : p.P + rbeg + (int64_t)cl * p.ldp);
        d4 acc[2][2];
#pragma unroll
        for (int a = 0; a < 2; ++a) acc[a][0] = acc[a][1] = d4{0.0, 0.0, 0.0, 0.0};
        int kb = 0;
        // every batch but the last has an even size, so step kb + u goes to chain u & 1
        auto batch = [&](auto nbc) {
          constexpr int NB = decltype(nbc)::value;
          double bz[NB];
#pragma unroll
          for (int u = 0; u < NB; ++u) {
            // rows past nrow load row nrow - 1: their V_s^T rows in X are zero
            bz[u] = src[min(4 * (kb + u) + lk, nr1)];
          }
          __builtin_amdgcn_sched_barrier(0);   // all loads of the batch issue before its MFMAs
#pragma unroll
          for (int u = 0; u < NB; ++u) {
            const int r = 4 * (kb + u) + lk;
            acc[0][u & 1] = __builtin_amdgcn_mfma_f64_16x16x4f64(X[li * ldx + r], bz[u], acc[0][u & 1], 0, 0, 0);
            acc[1][u & 1] = __builtin_amdgcn_mfma_f64_16x16x4f64(X[(16 + li) * ldx + r], bz[u], acc[1][u & 1], 0, 0, 0);
          }
          kb += NB;
        };
        while (KS - kb >= 32) batch(std::integral_constant<int, 32>{});
        if (KS - kb >= 16) batch(std::integral_constant<int, 16>{});
        if (KS - kb >= 8) batch(std::integral_constant<int, 8>{});
        if (KS - kb >= 4) batch(std::integral_constant<int, 4>{});
        if (KS - kb >= 2) batch(std::integral_constant<int, 2>{});
        if (KS - kb >= 1) batch(std::integral_constant<int, 1>{});
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            const int i = 16 * a + 4 * q + lk;
            if (i < ws && col < nb) st_agent(mypart + i * nz + (col - cs), acc[a][0][q] + acc[a][1][q]);
          }
      }
    }
    ok = grid_sync(gb, gen, true, true);   // exchange mode, every wave stored partials
    if (!ok) break;
    {
      // reduce-scatter: this workgroup sums elements [beg, end) over all
      // workgroups' partials; G threads share an element, thread g taking a
      // contiguous range of workgroups with its loads issued 16 at a time, and
      // the G range sums are added in range order (a fixed order)
      const int E = ws * nz;
      const int per = (E + nwg - 1) / nwg;
      const int beg = wg * per, end = min(E, beg + per);
      const int G = per >= kPThreads ? 1 : (per >= kPThreads / 2 ? 2 : (per >= kPThreads / 4 ? 4 : 8));
      const int wper = (nwg + G - 1) / G;
      const int g = t % G;
      const int w0 = g * wper, w1 = min(nwg, w0 + wper);
      for (int e0 = beg; e0 < end; e0 += kPThreads / G) {
        const int e = e0 + t / G;
        double acc = 0.0;
        if (e < end)
          for (int wb = w0; wb < w1; wb += 16) {
            double x[16];
#pragma unroll
            for (int u = 0; u < 16; ++u) x[u] = wb + u < w1 ? ld_agent(part_up + (size_t)(wb + u) * W * nb + e) : 0.0;
#pragma unroll
            for (int u = 0; u < 16; ++u) acc += x[u];
          }
        sc[t] = acc;
        __syncthreads();
        if (g == 0 && e < end) {
          double tot = sc[t];
          for (int h = 1; h < G; ++h) tot += sc[t + h];
          st_agent(p.red + e, tot);
        }
        __syncthreads();
      }
    }
    ok = grid_sync(gb, gen, true, true);
    if (!ok) break;
    // the reduced rows V_s^T [V_s | A_rest] -> LDS (row tt at Wp + tt*nb,
    // columns cs .. nb), 16 loads in flight
    for (int base = 0; base < ws * nz; base += 16 * kPThreads) {
      double x[16];
#pragma unroll
      for (int u = 0; u < 16; ++u) {
        const int idx = base + t + u * kPThreads;
        x[u] = idx < ws * nz ? ld_agent(p.red + idx) : 0.0;
      }
#pragma unroll
      for (int u = 0; u < 16; ++u) {
        const int idx = base + t + u * kPThreads;
        if (idx < ws * nz) Wp[(idx / nz) * nb + cs + idx % nz] = x[u];
      }
    }
    for (int idx = ws * nb + t; idx < W * nb; idx += kPThreads) Wp[idx] = 0.0;   // rows ws .. W of a ragged slab
    // the recurrence below reads rows of Wp that other waves stored
    __syncthreads();
    // T_s by the recurrence T(r, tt) = -tau_tt sum_{r<=u<tt} T(r, u) v_u^T v_tt,
    // which involves only row r.  Eight lanes share a row (all 256 threads:
    // 32 rows x 8): lane `part` keeps T(r, u) for u = part + 8i in registers
    // and sums those terms, a group sum over the 8 lanes completes each entry,
    // and the lane owning column tt keeps it.  Entries not yet formed are zero,
    // so every sum may run over all u; the loads of v_u^T v_tt do not depend
    // on T and run ahead of the 32-step chain.
    {
      const int r = t >> 3, part = t & 7;
      double tr[W / 8];
#pragma unroll
      for (int i = 0; i < W / 8; ++i) tr[i] = 0.0;
#pragma unroll
      for (int tt = 0; tt < W; ++tt) {
        double a = 0.0;
#pragma unroll
        for (int i = 0; i < W / 8; ++i) {
          const int u = part + 8 * i;
          const double g = Wp[u * nb + cs + tt];
          a += u < tt ? tr[i] * g : 0.0;
        }
        a = group8_sum(a);
        const double ta = taus[tt];
        const bool live = r < ws && tt < ws && tt >= r;
        const double v = !live ? 0.0 : (tt == r ? ta : -ta * a);
        if (part == (tt & 7)) tr[tt >> 3] = v;
      }
#pragma unroll
      for (int i = 0; i < W / 8; ++i) Ts[r + (part + 8 * i) * W] = tr[i];
    }
    __syncthreads();
    const int rest = nb - (cs + ws);
    if (rest > 0) {
      // A_rest -= V_s (T_s^T W) is applied as (V_s T_s^T) W: X <- X T_s^T on
      // the matrix cores, one wave per 16-row block (it reads all its rows
      // before writing them, so the update is in place), W stays as reduced
      {
        const int rb = (nrow + 15) / 16;
        for (int blk = wave; blk < rb; blk += kPThreads / 64) {
          const int r0 = 16 * blk;
          const int ra = min(r0 + li, rpw4 - 1);
          d4 acc0 = {0.0, 0.0, 0.0, 0.0}, acc1 = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
          for (int k0 = 0; k0 < W; k0 += 4) {
            const double a = X[(k0 + lk) * ldx + ra];
            acc0 = __builtin_amdgcn_mfma_f64_16x16x4f64(a, Ts[li + (k0 + lk) * W], acc0, 0, 0, 0);
            acc1 = __builtin_amdgcn_mfma_f64_16x16x4f64(a, Ts[16 + li + (k0 + lk) * W], acc1, 0, 0, 0);
          }
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            const int r = r0 + 4 * q + lk;
            if (r < nrow) {
              X[li * ldx + r] = acc0[q];
              X[(16 + li) * ldx + r] = acc1[q];
            }
          }
        }
      }
      __syncthreads();
      // A_rest(own rows) -= (V_s T_s^T) W on the matrix cores, computed transposed
      // (D[i][j] = sum_tt W(tt, c0 + i) X(r0 + j, tt)) so that each lane
      // holds consecutive rows of one column of P: 16 x 16 blocks dealt to waves
      {
        // eight blocks per pass: their 32 loads of P (unconditional, clamped to
        // a valid element; values loaded for absent elements are never stored)
        // are issued before the pass's MFMAs
        const int rb = (nrow + 15) / 16, cb = (rest + 15) / 16, nblk = rb * cb;
        constexpr int NW = kPThreads / 64, GB = 8;
        const int nr1 = nrow - 1;
        for (int b0 = wave * GB; b0 < nblk; b0 += NW * GB) {
          double pv[GB][4];
#pragma unroll
          for (int u = 0; u < GB; ++u) {
            const int blk = b0 + u;
            const int r = 16 * (blk % rb) + li, c0 = 16 * (blk / rb);
#pragma unroll
            for (int q = 0; q < 4; ++q) {
              const int c = c0 + 4 * q + lk;
              pv[u][q] = p.P[(rbeg + min(r, nr1)) + (int64_t)(cs + ws + min(c, rest - 1)) * p.ldp];
            }
          }
          __builtin_amdgcn_sched_barrier(0);
          d4 acc[GB];
#pragma unroll
          for (int u = 0; u < GB; ++u) acc[u] = d4{0.0, 0.0, 0.0, 0.0};
          // all W steps (rows tt >= ws of W are zero, and so are columns tt >= ws
          // of X T_s^T): straight-line MFMAs whose LDS operands load ahead
#pragma unroll
          for (int k0 = 0; k0 < W; k0 += 4) {
            const int tt = k0 + lk;
#pragma unroll
            for (int u = 0; u < GB; ++u) {
              const int blk = min(b0 + u, nblk - 1);
              const int r0 = 16 * (blk % rb), c0 = 16 * (blk / rb);
              const int ca = cs + ws + min(c0 + li, rest - 1);
              const double a = Wp[tt * nb + ca];                         // rows tt >= ws are zero
              const double bv = X[tt * ldx + min(r0 + li, rpw4 - 1)];   // zero for tt >= ws and pad rows
              acc[u] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, bv, acc[u], 0, 0, 0);
            }
          }
#pragma unroll
          for (int u = 0; u < GB; ++u) {
            const int blk = b0 + u;
            const int r = 16 * (blk % rb) + li, c0 = 16 * (blk / rb);
#pragma unroll
            for (int q = 0; q < 4; ++q) {
              const int c = c0 + 4 * q + lk;
              if (blk < nblk && r < nrow && c < rest)
                p.P[(rbeg + r) + (int64_t)(cs + ws + c) * p.ldp] = pv[u][q] - acc[u][q];
            }
          }
        }
      }
    }
    __syncthreads();
  }
  if (!ok && p.info && t == 0) atomicExch(&p.info[2], 1);
}

size_t panel_lds_doubles(int rpw, int nb) {
  const size_t ld = (size_t)((rpw + 3) & ~3) + 1;   // the kernel's padded stride
  return (size_t)W * ld + (size_t)W * nb + W * W;
}

// T (nb x nb, upper triangular) of the compact WY form from tau and the Gram
// matrix S = V^T V (Section 5.1), by recursive doubling over blocks of W
// columns.  A diagonal block follows the column recurrence T(r, j) = -tau_j
// sum_{r<=u<j} T(r, u) S(u, j), T(j, j) = tau_j, which only involves row r.
// Two neighbouring diagonal parts T_1 (columns [c0, c0+h)) and T_2 (columns
// [c0+h, c0+2h)) combine as T = [T_1, -T_1 S_12 T_2; 0, T_2] (the product of
// the two groups of reflectors), so one launch per level h = W, 2W, 4W, ...
// fills the off-diagonal blocks of all pairs at once; each workgroup owns one
// W x W tile (r, c) of one T_12 = -T_1 (S_12 T_2): it forms the column block
// X = S_12 T_2(:, c) and then -T_1(r, :) X.  No grid-wide wait: a level only
// reads the levels before it.  The strictly lower part of T is written as zero.
constexpr int kTThreads = 256;
constexpr int kTLd = W + 1;        // row stride of staged W x W blocks (odd: no bank conflicts)

__global__ __launch_bounds__(kTThreads) void wy_t_diag_kernel(int nb, const double *__restrict__ tau,
                                                              const double *__restrict__ S, double *__restrict__ T,
                                                              int64_t ldt) {
  __shared__ double Sd[W * kTLd];
  const int t = threadIdx.x, J = blockIdx.x, cJ = J * W;
  const int ws = min(W, nb - cJ);
  // every staged entry is loaded before any is written to LDS, so the loads
  // are in flight together (a write after each load would wait for it)
  static_assert(W * W % kTThreads == 0, "staging loops without a tail");
  double sv[W * W / kTThreads];
#pragma unroll
  for (int q = 0; q < W * W / kTThreads; ++q) {
    const int idx = t + q * kTThreads, u = idx % W, j = idx / W;
    sv[q] = (u < ws && j < ws) ? S[(cJ + u) + (int64_t)(cJ + j) * nb] : 0.0;
  }
#pragma unroll
  for (int q = 0; q < W * W / kTThreads; ++q) {
    const int idx = t + q * kTThreads;
    Sd[(idx % W) * kTLd + idx / W] = sv[q];
  }
  // zeros left of the diagonal block (rows cJ .. cJ + ws)
  for (int idx = t; idx < ws * cJ; idx += kTThreads) {
    const int r = idx % ws, col = idx / ws;
    T[(cJ + r) + (int64_t)col * ldt] = 0.0;
  }
  __syncthreads();
  // eight lanes per row: lane `part` keeps T(r, u) for u = part + 8i and sums
  // those terms; a group sum completes each entry
  const int r = t >> 3, part = t & 7;
  double tr[W / 8];
#pragma unroll
  for (int i = 0; i < W / 8; ++i) tr[i] = 0.0;
#pragma unroll
  for (int tt = 0; tt < W; ++tt) {
    double a = 0.0;
#pragma unroll
    for (int i = 0; i < W / 8; ++i) {
      const int u = part + 8 * i;
      a += u < tt ? tr[i] * Sd[u * kTLd + tt] : 0.0;
    }
    a = group8_sum(a);
    const double ta = tt < ws ? tau[cJ + tt] : 0.0;
    const bool live = r < ws && tt < ws && tt >= r;
    const double v = !live ? 0.0 : (tt == r ? ta : -ta * a);
    if (part == (tt & 7)) tr[tt >> 3] = v;
  }
#pragma unroll
  for (int i = 0; i < W / 8; ++i) {
    const int col = part + 8 * i;
    if (r < ws && col < ws) T[(cJ + r) + (int64_t)(cJ + col) * ldt] = tr[i];
  }
}

// One level of the doubling: h = W * 2^(level-1); workgroup -> (pair p, tile
// row tr, tile column tc) of T_12 = T(c0 : c0+h, c0+h : c0+2h), c0 = 2 h p.
// Entries past nb are zero in S, T and tau, so ragged edges need no cases
// beyond the bounds of the loads and stores.
template <int RPT>   // rows of X per thread: h / 8
__global__ __launch_bounds__(kTThreads) void wy_t_level_kernel(int nb, const double *__restrict__ S,
                                                               double *__restrict__ T, int64_t ldt) {
  extern __shared__ double sh[];
  constexpr int h = 8 * RPT;
  const int t = threadIdx.x;
  const int nt = h / W;                       // tiles per side of T_12
  const int p = blockIdx.x / (nt * nt), tr = (blockIdx.x / nt) % nt, tc = blockIdx.x % nt;
  const int c0 = 2 * h * p, c1 = c0 + h;      // T_1 columns [c0, c1), T_2 columns [c1, c1 + h)
  if (c1 >= nb) return;                       // no right half: nothing to combine
  double *X = sh;                             // h x W: X = S_12 T_2(:, tile tc), row i at X + i*kTLd
  double *Bs = X + (size_t)h * kTLd;          // W x W staged block of T_2, then of T_1
  double *As = Bs + W * kTLd;                 // h x W staged block column of S_12
  auto Tg = [&](int i, int j) -> double { return (i < nb && j < nb) ? T[i + (int64_t)j * ldt] : 0.0; };
  auto Sg = [&](int i, int j) -> double { return (i < nb && j < nb) ? S[i + (int64_t)j * nb] : 0.0; };
  // X(i, cc) = sum_{b <= tc} sum_k S_12(i, W b + k) T_2(W b + k, W tc + cc): thread (row group, column cc)
  const int cc = t & (W - 1), rg = t >> 5;    // 8 row groups of RPT rows
  double acc[RPT];
#pragma unroll
  for (int q = 0; q < RPT; ++q) acc[q] = 0.0;
  // staged entries are loaded into registers before any LDS write, so each
  // thread's loads are in flight together
  constexpr int nBq = W * W / kTThreads, nAq = h * W / kTThreads;
  static_assert(W * W % kTThreads == 0 && h * W % kTThreads == 0, "staging loops without a tail");
  for (int bb = 0; bb <= tc; ++bb) {
    double rb[nBq], ra[nAq];
#pragma unroll
    for (int q = 0; q < nBq; ++q) {
      const int idx = t + q * kTThreads;
      rb[q] = Tg(c1 + W * bb + idx % W, c1 + W * tc + idx / W);
    }
#pragma unroll
    for (int q = 0; q < nAq; ++q) {
      const int idx = t + q * kTThreads;
      ra[q] = Sg(c0 + idx % h, c1 + W * bb + idx / h);
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < nBq; ++q) {
      const int idx = t + q * kTThreads;
      Bs[(idx % W) * kTLd + idx / W] = rb[q];
    }
#pragma unroll
    for (int q = 0; q < nAq; ++q) {
      const int idx = t + q * kTThreads;
      As[(idx % h) * kTLd + idx / h] = ra[q];
    }
    __syncthreads();
    for (int k = 0; k < W; ++k) {
      const double bv = Bs[k * kTLd + cc];
#pragma unroll
      for (int q = 0; q < RPT; ++q) acc[q] += As[(rg * RPT + q) * kTLd + k] * bv;
    }
  }
#pragma unroll
  for (int q = 0; q < RPT; ++q) X[(rg * RPT + q) * kTLd + cc] = acc[q];
  // tile (tr, tc) of T_12 = -sum_{a >= tr} T_1(W tr + i, W a + k) X(W a + k, cc): thread (rows 4 rq .. 4 rq + 3, cc)
  const int rq = t >> 5;
  double o[4] = {0.0, 0.0, 0.0, 0.0};
  for (int a = tr; a < nt; ++a) {
    double rb[nBq];
#pragma unroll
    for (int q = 0; q < nBq; ++q) {
      const int idx = t + q * kTThreads;
      rb[q] = Tg(c0 + W * tr + idx % W, c0 + W * a + idx / W);
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < nBq; ++q) {
      const int idx = t + q * kTThreads;
      Bs[(idx % W) * kTLd + idx / W] = rb[q];
    }
    __syncthreads();
    for (int k = 0; k < W; ++k) {
      const double xv = X[(W * a + k) * kTLd + cc];
#pragma unroll
      for (int q = 0; q < 4; ++q) o[q] += Bs[(4 * rq + q) * kTLd + k] * xv;
    }
  }
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int i = c0 + W * tr + 4 * rq + q, j = c1 + W * tc + cc;
    if (i < nb && j < nb) T[i + (int64_t)j * ldt] = -o[q];
  }
}

}  // namespace

int panel_config(int64_t mi, int nb, int *rpw) {
  if (mi < 1 || nb < 1 || nb > 512) return 0;
  int64_t nwg = (mi + 31) / 32;
  if (nwg > 64) nwg = 64;
  for (;; ++nwg) {
    if (nwg > 256) return 0;
    const int64_t r = (mi + nwg - 1) / nwg;
    // the row update of a column step gives a thread at most two rows
    if (r <= 2 * kPThreads && panel_lds_doubles((int)r, nb) <= kLdsDoubles - (5 * kGW + W)) {
      *rpw = (int)r;
      return (int)((mi + r - 1) / r);
    }
  }
}

size_t panel_part_doubles(int nwg, int nb) { return (size_t)2 * nwg * 2 * kGW + (size_t)nwg * W * nb; }

hipError_t launch_panel_qr(hipStream_t s, const PanelQR &p) {
  int rpw = 0;
  const int nwg = panel_config(p.mi, p.nb, &rpw);
  if (nwg == 0) return hipErrorInvalidValue;
  static bool attr_done = false;
  if (!attr_done) {
    hipError_t e = hipFuncSetAttribute((const void *)panel_qr_kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                                       (int)((kLdsDoubles - (5 * kGW + W)) * sizeof(double)));
    if (e != hipSuccess) return e;
    attr_done = true;
  }
  const size_t lds = panel_lds_doubles(rpw, p.nb) * sizeof(double);
  PanelQR pp = p;
  GridBarrier gb{p.bar, p.abort_flag, p.limit_ticks};
  void *args[] = {&pp, &rpw, &gb};
  return launch_persistent((const void *)panel_qr_kernel, (unsigned)nwg, kPThreads, args, lds, s);
}

hipError_t launch_wy_t(hipStream_t s, int nb, const double *tau, const double *S, double *T, int64_t ldt) {
  if (nb <= 0) return hipSuccess;
  if (nb > 512) return hipErrorInvalidValue;
  const int nslab = (nb + W - 1) / W;
  hipLaunchKernelGGL(wy_t_diag_kernel, dim3(nslab), dim3(kTThreads), 0, s, nb, tau, S, T, ldt);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  for (int h = W; h < nb; h *= 2) {
    const int nt = h / W, npair = (nb + 2 * h - 1) / (2 * h);
    const size_t lds = ((size_t)h * kTLd + W * kTLd + (size_t)h * kTLd) * sizeof(double);
    const void *fn = h == W ? (const void *)wy_t_level_kernel<W / 8>
                   : h == 2 * W ? (const void *)wy_t_level_kernel<2 * W / 8>
                   : h == 4 * W ? (const void *)wy_t_level_kernel<4 * W / 8>
                                : (const void *)wy_t_level_kernel<8 * W / 8>;
    static bool attr_done[4] = {false, false, false, false};
    const int li = h == W ? 0 : h == 2 * W ? 1 : h == 4 * W ? 2 : 3;
    if (!attr_done[li]) {
      e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)(kLdsDoubles * sizeof(double)));
      if (e != hipSuccess) return e;
      attr_done[li] = true;
    }
    const dim3 grid((unsigned)(npair * nt * nt)), block(kTThreads);
    if (li == 0) hipLaunchKernelGGL(wy_t_level_kernel<W / 8>, grid, block, lds, s, nb, S, T, ldt);
    else if (li == 1) hipLaunchKernelGGL(wy_t_level_kernel<2 * W / 8>, grid, block, lds, s, nb, S, T, ldt);
    else if (li == 2) hipLaunchKernelGGL(wy_t_level_kernel<4 * W / 8>, grid, block, lds, s, nb, S, T, ldt);
    else hipLaunchKernelGGL(wy_t_level_kernel<8 * W / 8>, grid, block, lds, s, nb, S, T, ldt);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

}  // namespace rq
