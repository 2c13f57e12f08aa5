// C ABI of librqrcp: argument checking, workspace planning and the host loop
// over blocks of the blocked randomized QR (Fig. 3).  Every step runs in the
// kernels of this library on the handle's stream; the host only computes
// offsets and enqueues launches, so nothing here waits for the GPU.
#include <algorithm>
#include <cstdio>
#include <cstring>
#include <string>
#include <type_traits>
#include <mutex>
#include <vector>

#include "common.h"
#include "misc.h"

// Workspace of the allocation-free entry point (rqrcp_factor_noalloc): one
// array per device, held until the process ends.  Host code uses the device
// address that hipGetSymbolAddress returns for the current device (kept per
// device by rqrcp_create), never the array's name.
static __device__ __align__(256) unsigned char scratch[RQRCP_NOALLOC_WORK_BYTES];

namespace {
std::mutex g_scratch_mu;
std::vector<void *> g_scratch_ptr;   // device address of `scratch`, per device (nullptr until set up)

// Once per device, with that device current: the address of its copy of `scratch`.
hipError_t scratch_setup(int dev, void **out) {
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if ((int)g_scratch_ptr.size() <= dev) g_scratch_ptr.resize(dev + 1, nullptr);
  if (!g_scratch_ptr[dev]) {
    void *ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch_ptr[dev] = ptr;
  }
  *out = g_scratch_ptr[dev];
  return hipSuccess;
}
}  // namespace

struct rqrcp_timing_rec {
  int kclass;
  hipEvent_t start, stop;
  double flops, bytes;
};

struct rqrcp_ctx {
  hipStream_t stream = nullptr;
  hipStream_t side = nullptr;          // library-owned, default priority: work that overlaps the main stream
  hipEvent_t fork_ev = nullptr, join_ev = nullptr;
  // Library-owned non-blocking stream (default priority): the sketch product
  // of the next block and the trailing update run there with their grids
  // capped at half the CUs, so that the persistent panel and pivoted-QR
  // kernels beside them find their CUs free.
  hipStream_t aux = nullptr;
  int ncu = 0;
  hipEvent_t ev_moves = nullptr, ev_ypre = nullptr, ev_vt = nullptr, ev_upd = nullptr, ev_w = nullptr;
  hipEvent_t ev_diag = nullptr;   // the diagonalised block's work on the side stream
  // device int32[4]: the info word of factorizations given no opts.info, so
  // that a give-up of a grid-wide wait is never lost (read by rqrcp_check)
  int32_t *own_info = nullptr;
  void *scratch = nullptr;    // this device's `scratch` (rqrcp_factor_noalloc)
  int device = 0;
  uint64_t limit_ticks = 0;   // grid-barrier wait limit (about 2 s of the device clock)
  std::string last_error;
  bool timing = false;
  uint32_t timing_mask = 0xFFFFFFFFu;   // classes bracketed while timing is on
  std::vector<hipEvent_t> free_events;
  std::vector<hipEvent_t> all_events;
  std::vector<rqrcp_timing_rec> recs;
};

namespace rq {
namespace {

thread_local std::string g_last_error;

rqrcp_status_t fail(rqrcp_handle_t h, rqrcp_status_t st, const std::string &msg) {
  if (h) h->last_error = msg;
  g_last_error = msg;
  return st;
}

rqrcp_status_t fail_hip(rqrcp_handle_t h, hipError_t e, const char *where) {
  std::string m = std::string(where) + ": " + hipGetErrorString(e);
  return fail(h, RQRCP_ERR_HIP, m);
}

inline size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }
inline int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }

struct Bump {
  size_t off = 0;
  size_t take(size_t bytes) {
    const size_t o = off;
    off = align256(off + bytes);
    return o;
  }
};

constexpr int kSlotWords = 512;   // per cooperative launch: barrier state + abort word
constexpr int kAbortWord = 448;
static_assert(kBarrierWords < kAbortWord && kAbortWord < kSlotWords, "barrier slot layout");

struct GemmShape {
  int64_t M, N, K;
};

// Partial-product room for a GEMM of this shape, whichever engine (tiled or
// all-rows) and transposition the call uses.
size_t gemm_part_doubles(int64_t M, int64_t N, int64_t K) {
  if (M <= 0 || N <= 0 || K <= 0) return 0;
  int sp = 1;
  for (int tb = 0; tb < 2; ++tb) {
    GemmF64 g{};
    g.M = M; g.N = N; g.K = K; g.tb = tb != 0;
    sp = std::max(sp, gemm_f64_splits(g));
  }
  return sp > 1 ? (size_t)sp * M * N : 0;
}

// S = V^T V (cols x cols, ld cols) for the T factor of the reflectors in the
// explicit unit-lower V (rows x cols, ld ldv).
hipError_t launch_gram(hipStream_t s, const double *V, int64_t ldv, int64_t rows, int64_t cols, double *S,
                       double *part) {
  GemmF64 g{true, false, cols, cols, rows, V, ldv, V, ldv, S, cols, 1.0, 0.0};
  return launch_gemm_f64(s, g, part);
}

// The same for an FP32 product (the all-rows engine takes more rows in FP32).
size_t gemm_part_floats(int64_t M, int64_t N, int64_t K) {
  if (M <= 0 || N <= 0 || K <= 0) return 0;
  int sp = 1;
  for (int tb = 0; tb < 2; ++tb) {
    GemmF32 g{};
    g.M = M; g.N = N; g.K = K; g.tb = tb != 0;
    sp = std::max(sp, gemm_splits<float>(g));
  }
  return sp > 1 ? (size_t)sp * M * N : 0;
}

struct FactorPlan {
  int64_t m = 0, n = 0, b = 0, p = 0, k = 0, ks = 0, nblocks = 0;
  bool ortho = false, fixed = false, classical_tail = false, f32 = false, mixed = false;
  int power = 0;   // steps of the power iteration on every sketched block
  bool panel_pivot = false;   // in-block pivot P-hat by QRCP of the panel's R'
  bool diag = false;          // diagonalised blocks (Section 6.2)
  // FP32-storage buffers
  size_t Pw = 0, V32 = 0, VT32 = 0, Vt32 = 0, W32 = 0, gpart32 = 0, Gb = 0, spart = 0, G32 = 0, Y32 = 0, VS32 = 0, TS32 = 0;
  size_t gpart32_aux = 0;   // split-K room of the FP32 trailing update on the auxiliary stream
  int nslots = 0;
  // byte offsets into the workspace
  size_t G = 0, Y = 0, YT = 0, Vb = 0, VT = 0, Vt = 0, Wb = 0, gpart = 0, Sg = 0, ppart = 0, pred = 0, qrec = 0, qcand = 0,
         piv = 0, dest = 0, moved = 0, mcnt = 0, tmp = 0, jtmp = 0, bars = 0, Acopy = 0, total = 0;
  size_t Y_doubles = 0;
  // overlapped schedule (FP64 storage, permutation pivots, sampled blocks)
  bool pipe = false;
  size_t GVb = 0, gpart_aux = 0;
  size_t vtpart = 0;   // split-K buffer of V T^T (on the side stream, beside W)
  size_t W2 = 0;       // T^T W (overlapped schedule)
  size_t Z = 0;        // Y X^T of the power iteration
  size_t Pc = 0, Rp = 0;   // saved panel and its R' (in-block pivoting)
  size_t svdw = 0;         // working columns of the SVD of blocks above 64 columns
  size_t r22 = 0;          // FP32 storage: the block's triangle widened for its SVD
  size_t scal = 0;         // one word for the power-of-two scaling of FP32 power steps
};

bool block_is_classical_tail(const FactorPlan &P, int64_t i) {
  return P.classical_tail && i == P.nblocks - 1;
}

rqrcp_status_t make_plan(rqrcp_handle_t h, rqrcp_dtype_t dt, int64_t m, int64_t n, const rqrcp_opts_t *o,
                         FactorPlan *out) {
  if (!o) return fail(h, RQRCP_ERR_ARG, "opts is NULL");
  if (dt != RQRCP_F64 && dt != RQRCP_F32) return fail(h, RQRCP_ERR_ARG, "dt: unknown storage type");
  if (n < 1) return fail(h, RQRCP_ERR_ARG, "n must be >= 1");
  if (m < n) return fail(h, RQRCP_ERR_ARG, "m must be >= n (the method assumes m >= n)");
  if (o->block < 1) return fail(h, RQRCP_ERR_ARG, "opts.block must be >= 1");
  if (o->oversample < 0) return fail(h, RQRCP_ERR_ARG, "opts.oversample must be >= 0");
  if (o->rank < 0 || o->rank > n) return fail(h, RQRCP_ERR_ARG, "opts.rank must be in [0, n]");
  if (o->pivot != RQRCP_PIVOT_PERM && o->pivot != RQRCP_PIVOT_ORTHO)
    return fail(h, RQRCP_ERR_ARG, "opts.pivot: unknown value");
  if (o->precision != RQRCP_PREC_PLAIN && o->precision != RQRCP_PREC_MIXED)
    return fail(h, RQRCP_ERR_ARG, "opts.precision: unknown value");
  if (o->precision == RQRCP_PREC_MIXED && dt != RQRCP_F32)
    return fail(h, RQRCP_ERR_ARG, "opts.precision: MIXED needs F32 storage");
  if (o->tail != RQRCP_TAIL_CLASSICAL && o->tail != RQRCP_TAIL_SAMPLED)
    return fail(h, RQRCP_ERR_ARG, "opts.tail: unknown value");
  if (o->fixed_pivots != 0 && o->fixed_pivots != 1) return fail(h, RQRCP_ERR_ARG, "opts.fixed_pivots must be 0 or 1");
  if (o->fixed_pivots && o->pivot == RQRCP_PIVOT_ORTHO)
    return fail(h, RQRCP_ERR_UNSUPPORTED, "opts.fixed_pivots applies to the permutation form only");
  if (o->power < 0 || o->power > 8) return fail(h, RQRCP_ERR_ARG, "opts.power must be in [0, 8]");
  if (o->panel_pivot != 0 && o->panel_pivot != 1) return fail(h, RQRCP_ERR_ARG, "opts.panel_pivot must be 0 or 1");
  if (o->diagonalize != 0 && o->diagonalize != 1) return fail(h, RQRCP_ERR_ARG, "opts.diagonalize must be 0 or 1");
  if (o->diagonalize && o->pivot != RQRCP_PIVOT_ORTHO)
    return fail(h, RQRCP_ERR_UNSUPPORTED, "opts.diagonalize: orthonormal pivoting only");
  if (o->diagonalize && o->block > svd_small_max_block())
    return fail(h, RQRCP_ERR_UNSUPPORTED, "opts.diagonalize: block at most 256");
  if (o->panel_pivot && !o->fixed_pivots && o->pivot != RQRCP_PIVOT_PERM)
    return fail(h, RQRCP_ERR_UNSUPPORTED, "opts.panel_pivot: the permutation form only");
  FactorPlan P;
  P.f32 = dt == RQRCP_F32;
  P.mixed = o->precision == RQRCP_PREC_MIXED;
  P.m = m; P.n = n; P.b = o->block; P.p = o->oversample;
  P.k = o->rank == 0 ? n : o->rank;
  P.ks = P.b + P.p;
  P.nblocks = cdiv(P.k, P.b);
  P.ortho = o->pivot == RQRCP_PIVOT_ORTHO;
  P.fixed = o->fixed_pivots != 0;
  P.power = P.fixed ? 0 : o->power;
  P.panel_pivot = !P.fixed && o->panel_pivot != 0;
  P.diag = o->diagonalize != 0;
  P.classical_tail = !P.ortho && !P.fixed && o->tail == RQRCP_TAIL_CLASSICAL && P.k == n;
  if (P.b > 512) return fail(h, RQRCP_ERR_UNSUPPORTED, "opts.block: at most 512");
  if (P.ks > 512 && !P.fixed) return fail(h, RQRCP_ERR_UNSUPPORTED, "block + oversample: at most 512");

  size_t Yd = 0, gpart = 0, ppart = 0, gpart32 = 0, spart = 0, vtp = 0;
  int qnwg = 0;
  int64_t qk = 1;
  for (int64_t i = 0; i < P.nblocks; ++i) {
    const int64_t r0 = i * P.b, bi = std::min(P.b, P.k - r0), mi = m - r0, ni = n - r0;
    int rpw = 0;
    const int pn = panel_config(mi, (int)bi, &rpw);
    if (pn == 0) return fail(h, RQRCP_ERR_UNSUPPORTED, "panel too large for the panel kernel");
    ppart = std::max(ppart, panel_part_doubles(pn, (int)bi));
    vtp = std::max(vtp, gemm_part_doubles(mi, bi, bi));
    vtp = std::max(vtp, gemm_part_doubles(bi, bi, mi));      // V^T V beside W
    gpart = std::max(gpart, gemm_part_doubles(bi, bi, mi));  // V^T V of the last block
    if (P.diag) {   // U'^T C and A12 V' run on the side stream as well
      vtp = std::max(vtp, gemm_part_doubles(bi, ni - bi, bi));
      vtp = std::max(vtp, gemm_part_doubles(r0, bi, bi));
    }
    if (!P.fixed) {
      if (block_is_classical_tail(P, i)) {
        int cpw = 0;
        const int qn = qrcp_small_config((int)mi, (int)ni, &cpw);
        if (qn == 0) return fail(h, RQRCP_ERR_UNSUPPORTED, "last block too large for the pivoted-QR kernel");
        qnwg = std::max(qnwg, qn);
        qk = std::max(qk, mi);
        Yd = std::max(Yd, (size_t)(mi * ni));
      } else {
        Yd = std::max(Yd, (size_t)(P.ks * ni));
        const int64_t yrows = P.ortho ? bi : P.ks;
        gpart = std::max(gpart, gemm_part_doubles(yrows, ni, mi));
        if (P.power > 0) {
          gpart = std::max(gpart, gemm_part_doubles(yrows, mi, ni));
          gpart32 = std::max(gpart32, gemm_part_floats(yrows, mi, ni));
          gpart32 = std::max(gpart32, gemm_part_floats(yrows, ni, mi));
        }
        if (P.f32 && P.mixed) spart = std::max(spart, sample_bf16_part_floats(yrows, ni, mi));
        if (P.f32 && !P.mixed) gpart32 = std::max(gpart32, gemm_part_doubles(yrows, ni, mi));
        if (P.ortho) {
          gpart = std::max(gpart, gemm_part_doubles(m, bi, bi));
          gpart32 = std::max(gpart32, gemm_part_doubles(m, bi, bi));
          gpart32 = std::max(gpart32, gemm_part_doubles(m, bi, ni));
          gpart32 = std::max(gpart32, gemm_part_doubles(m, ni, bi));
          const int pn2 = panel_config(ni, (int)bi, &rpw);
          if (pn2 == 0) return fail(h, RQRCP_ERR_UNSUPPORTED, "sketch too large for the panel kernel");
          ppart = std::max(ppart, panel_part_doubles(pn2, (int)bi));
          gpart = std::max(gpart, gemm_part_doubles(bi, bi, ni));   // V_S^T V_S
          gpart = std::max(gpart, gemm_part_doubles(m, bi, ni));
          gpart = std::max(gpart, gemm_part_doubles(m, ni, bi));
        } else {
          int cpw = 0;
          const int qn = qrcp_small_config((int)P.ks, (int)ni, &cpw);
          if (qn == 0) return fail(h, RQRCP_ERR_UNSUPPORTED, "sketch too large for the pivoted-QR kernel");
          qnwg = std::max(qnwg, qn);
          qk = std::max(qk, P.ks);
          if (P.panel_pivot) {
            const int qp = qrcp_small_config((int)bi, (int)bi, &cpw);
            if (qp == 0) return fail(h, RQRCP_ERR_UNSUPPORTED, "block too large for the pivoted QR of the panel's R'");
            qnwg = std::max(qnwg, qp);
            qk = std::max(qk, bi);
          }
        }
      }
    }
    gpart = std::max(gpart, gemm_part_doubles(mi, bi, bi));
    if (P.diag) gpart = std::max(gpart, gemm_part_doubles(r0, bi, bi));   // A12 V'
    if (ni > bi) {
      gpart = std::max(gpart, gemm_part_doubles(bi, ni - bi, mi));
      gpart = std::max(gpart, gemm_part_doubles(bi, ni, mi));        // [S | W] = V^T [V | C]
      gpart = std::max(gpart, gemm_part_doubles(mi, ni - bi, bi));
      gpart = std::max(gpart, gemm_part_doubles(bi, ni - bi, bi));   // T^T W and U'^T C
      gpart32 = std::max(gpart32, gemm_part_doubles(bi, ni - bi, mi));
      gpart32 = std::max(gpart32, gemm_part_doubles(mi, ni - bi, bi));
    }
  }
  if (!P.f32) gpart32 = 0;
  // the next block's sketch product and this block's trailing update may run
  // on the auxiliary stream (own split-K room), the correction G V on the main
  P.pipe = (!P.f32 || P.mixed) && !P.ortho && !P.fixed;
  size_t gpaux = 0, gpaux32 = 0;
  if (P.pipe)
    for (int64_t i = 0; i + 1 < P.nblocks; ++i) {
      const int64_t r0 = i * P.b, bi = std::min(P.b, P.k - r0), mi = m - r0, ni = n - r0;
      if (block_is_classical_tail(P, i + 1) || ni <= bi) continue;
      gpaux = std::max(gpaux, gemm_part_doubles(P.ks, ni - bi, mi - bi));
      gpaux = std::max(gpaux, gemm_part_doubles(mi, ni - bi, bi));
      gpaux = std::max(gpaux, gemm_part_doubles(P.ks, bi, mi - bi));   // G V
      gpart = std::max(gpart, gemm_part_doubles(P.ks, bi, mi - bi));
      gpart = std::max(gpart, gemm_part_doubles(P.ks, ni - bi, bi));
      gpart = std::max(gpart, gemm_part_doubles(bi, ni - bi, bi));     // T^T W
      if (P.f32) {
        gpart = std::max(gpart, gemm_part_doubles(P.ks, bi, bi));       // (G V) T^T
        gpaux32 = std::max(gpaux32, gemm_part_floats(mi, ni - bi, bi));  // the FP32 update beside the QR
      }
    }
  P.Y_doubles = Yd;
  // cooperative launches per block: pivoted QR of the sketch (or the
  // orthonormal form's panel), the panel, and with P-hat one more of each
  P.nslots = (int)((P.panel_pivot ? 5 : 3) * P.nblocks + (P.diag ? P.nblocks : 0) + 4);
  Bump w;
  const size_t d = sizeof(double);
  P.G = w.take((o->G || P.fixed) ? 0 : (size_t)P.ks * m * d);
  P.Y = w.take(Yd * d);
  P.YT = w.take(P.ortho ? (size_t)n * P.b * d : 0);
  P.Vb = w.take((size_t)m * P.b * d);
  P.VT = w.take((size_t)m * P.b * d);
  P.Vt = w.take((size_t)m * P.b * d);
  // S (b x b) directly in front of W (b x n): at b = 256 one launch forms
  // [S | W] = V^T [V | C] with leading dimension b
  P.Sg = w.take((size_t)P.b * (P.b + n) * d);
  P.Wb = P.Sg + (size_t)P.b * P.b * d;
  P.gpart = w.take(gpart * d);
  P.ppart = w.take(ppart * d);
  P.pred = w.take((size_t)kPanelW * P.b * d);
  P.qrec = w.take(qrcp_small_rec_doubles(qnwg) * d);
  P.qcand = w.take(qrcp_small_cand_doubles(qnwg, (int)qk) * d);
  P.piv = w.take((size_t)P.b * 4);
  P.dest = w.take((size_t)n * 4);
  P.moved = w.take((size_t)2 * P.b * 4);
  P.mcnt = w.take(4 * 64);
  const size_t es = P.f32 ? 4 : 8;   // storage element size
  P.tmp = w.take(P.ortho || P.fixed ? 0 : (size_t)m * 2 * P.b * es);
  P.jtmp = w.take((size_t)2 * P.b * 4);
  P.bars = w.take((size_t)P.nslots * kSlotWords * 4);
  P.Acopy = w.take(P.fixed ? (size_t)m * n * es : 0);
  P.GVb = w.take(P.pipe ? (size_t)P.ks * P.b * d : 0);
  P.gpart_aux = w.take(gpaux * d);
  P.vtpart = w.take(vtp * d);
  P.W2 = w.take(P.f32 ? 0 : (size_t)P.b * n * d);
  P.Z = w.take(P.power > 0 ? (size_t)P.ks * m * d : 0);
  P.Pc = w.take(P.panel_pivot && !P.f32 ? (size_t)m * P.b * d : 0);
  P.Rp = w.take(P.panel_pivot ? (size_t)P.b * P.b * d : 0);
  P.svdw = w.take(P.diag ? svd_small_work_doubles((int)P.b) * d : 0);
  P.r22 = w.take(P.diag && P.f32 ? (size_t)P.b * P.b * d : 0);
  P.scal = w.take(P.f32 && P.power > 0 ? 256 : 0);
  if (P.f32) {
    P.Pw = w.take((size_t)m * P.b * d);
    P.V32 = w.take((size_t)m * P.b * 4);
    P.VT32 = w.take((size_t)m * P.b * 4);
    P.Vt32 = w.take((size_t)m * P.b * 4);
    P.W32 = w.take((size_t)P.b * n * 4);
    P.gpart32 = w.take(gpart32 * 4);
    const bool sampled = !P.fixed;
    P.Gb = w.take(sampled && P.mixed ? (size_t)P.ks * m * 2 : 0);
    P.spart = w.take(spart * 4);
    P.G32 = w.take(sampled && !P.mixed ? (size_t)P.ks * m * 4 : 0);
    P.Y32 = w.take(sampled && (!P.mixed || P.power > 0) ? (size_t)P.ks * n * 4 : 0);
    P.VS32 = w.take(P.ortho ? (size_t)n * P.b * 4 : 0);
    P.TS32 = w.take(P.ortho ? (size_t)P.b * P.b * 4 : 0);
    P.gpart32_aux = w.take(gpaux32 * 4);
  }
  P.total = w.off + 256;
  *out = P;
  return RQRCP_OK;
}

template <typename T>
T *at(void *base, size_t off) {
  return reinterpret_cast<T *>(static_cast<char *>(base) + off);
}

hipEvent_t take_event(rqrcp_handle_t h) {
  if (h->free_events.empty()) {
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    h->all_events.push_back(e);
    return e;
  }
  hipEvent_t e = h->free_events.back();
  h->free_events.pop_back();
  return e;
}

// Brackets the launches of one kernel class with events when timing is on.
struct ScopedTimer {
  rqrcp_handle_t h;
  int kclass;
  double flops, bytes;
  hipEvent_t start = nullptr;
  hipStream_t stream;
  ScopedTimer(rqrcp_handle_t hh, int kc, double f, double b, hipStream_t st = nullptr)
      : h(hh), kclass(kc), flops(f), bytes(b), stream(st ? st : hh->stream) {
    if (h->timing && ((h->timing_mask >> kc) & 1u)) {
      start = take_event(h);
      if (start) (void)hipEventRecord(start, stream);
    }
  }
  ~ScopedTimer() {
    if (!start) return;
    hipEvent_t stop = take_event(h);
    if (!stop) return;
    (void)hipEventRecord(stop, stream);
    h->recs.push_back({kclass, start, stop, flops, bytes});
  }
};

double qrcp_flops(double k, double ncols, double steps) {
  double f = 0.0;
  for (double t = 0; t < steps; t += 1.0) f += 4.0 * (k - t) * (ncols - t);
  return f;
}

}  // namespace
}  // namespace rq

using namespace rq;

extern "C" {

void rqrcp_default_opts(rqrcp_opts_t *o) {
  if (!o) return;
  std::memset(o, 0, sizeof(*o));
  o->block = 128;
  o->oversample = 10;
  o->rank = 0;
  o->pivot = RQRCP_PIVOT_PERM;
  o->precision = RQRCP_PREC_PLAIN;
  o->tail = RQRCP_TAIL_CLASSICAL;
}

const char *rqrcp_status_string(rqrcp_status_t s) {
  switch (s) {
    case RQRCP_OK: return "RQRCP_OK";
    case RQRCP_ERR_ARG: return "RQRCP_ERR_ARG: invalid argument";
    case RQRCP_ERR_WORKSPACE: return "RQRCP_ERR_WORKSPACE: workspace missing or too small";
    case RQRCP_ERR_HIP: return "RQRCP_ERR_HIP: HIP runtime error";
    case RQRCP_ERR_UNSUPPORTED: return "RQRCP_ERR_UNSUPPORTED: outside the supported range";
    case RQRCP_ERR_NONFINITE: return "RQRCP_ERR_NONFINITE: non-finite values";
    case RQRCP_ERR_TIMEOUT: return "RQRCP_ERR_TIMEOUT: a grid-wide wait gave up, results invalid";
  }
  return "unknown status";
}

const char *rqrcp_last_error(rqrcp_handle_t h) { return h ? h->last_error.c_str() : g_last_error.c_str(); }

rqrcp_status_t rqrcp_create(rqrcp_handle_t *h, void *hip_stream) {
  if (!h) return fail(nullptr, RQRCP_ERR_ARG, "h is NULL");
  *h = nullptr;
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return fail_hip(nullptr, e, "hipGetDevice");
  hipDeviceProp_t prop;
  e = hipGetDeviceProperties(&prop, dev);
  if (e != hipSuccess) return fail_hip(nullptr, e, "hipGetDeviceProperties");
  if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0)
    return fail(nullptr, RQRCP_ERR_UNSUPPORTED, std::string("device is ") + prop.gcnArchName + ", need gfx950");
  if (!prop.cooperativeLaunch) return fail(nullptr, RQRCP_ERR_UNSUPPORTED, "device lacks cooperative launch");
  int khz = 0;
  e = hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev);
  if (e != hipSuccess) return fail_hip(nullptr, e, "hipDeviceGetAttribute(WallClockRate)");
  rqrcp_ctx *c = new rqrcp_ctx();
  c->stream = static_cast<hipStream_t>(hip_stream);
  e = hipStreamCreateWithFlags(&c->side, hipStreamNonBlocking);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&c->fork_ev, hipEventDisableTiming);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&c->join_ev, hipEventDisableTiming);
  if (e == hipSuccess) e = hipStreamCreateWithFlags(&c->aux, hipStreamNonBlocking);
  hipEvent_t *evs[6] = {&c->ev_moves, &c->ev_ypre, &c->ev_vt, &c->ev_upd, &c->ev_w, &c->ev_diag};
  for (hipEvent_t *ev : evs)
    if (e == hipSuccess) e = hipEventCreateWithFlags(ev, hipEventDisableTiming);
  if (e == hipSuccess) e = hipMalloc(reinterpret_cast<void **>(&c->own_info), 4 * sizeof(int32_t));
  if (e == hipSuccess) e = hipMemset(c->own_info, 0, 4 * sizeof(int32_t));
  if (e == hipSuccess) e = scratch_setup(dev, &c->scratch);
  if (e != hipSuccess) {
    if (c->own_info) (void)hipFree(c->own_info);
    for (hipEvent_t *ev : evs)
      if (*ev) (void)hipEventDestroy(*ev);
    if (c->join_ev) (void)hipEventDestroy(c->join_ev);
    if (c->fork_ev) (void)hipEventDestroy(c->fork_ev);
    if (c->side) (void)hipStreamDestroy(c->side);
    if (c->aux) (void)hipStreamDestroy(c->aux);
    delete c;
    return fail_hip(nullptr, e, "side stream / events / info word / scratch address");
  }
  c->ncu = prop.multiProcessorCount;
  c->device = dev;
  c->limit_ticks = (uint64_t)(khz > 0 ? khz : 100000) * 2000ull;
  *h = c;
  return RQRCP_OK;
}

rqrcp_status_t rqrcp_set_stream(rqrcp_handle_t h, void *hip_stream) {
  if (!h) return fail(nullptr, RQRCP_ERR_ARG, "h is NULL");
  h->stream = static_cast<hipStream_t>(hip_stream);
  return RQRCP_OK;
}

rqrcp_status_t rqrcp_destroy(rqrcp_handle_t h) {
  if (!h) return RQRCP_OK;
  if (h->side) (void)hipStreamSynchronize(h->side);
  if (h->aux) (void)hipStreamSynchronize(h->aux);
  for (hipEvent_t e : h->all_events) (void)hipEventDestroy(e);
  if (h->fork_ev) (void)hipEventDestroy(h->fork_ev);
  if (h->join_ev) (void)hipEventDestroy(h->join_ev);
  for (hipEvent_t e : {h->ev_moves, h->ev_ypre, h->ev_vt, h->ev_upd, h->ev_w, h->ev_diag})
    if (e) (void)hipEventDestroy(e);
  if (h->side) (void)hipStreamDestroy(h->side);
  if (h->aux) (void)hipStreamDestroy(h->aux);
  if (h->own_info) {
    (void)hipStreamSynchronize(h->stream);
    (void)hipFree(h->own_info);
  }
  delete h;
  return RQRCP_OK;
}

rqrcp_status_t rqrcp_check(rqrcp_handle_t h, int32_t *info_host) {
  if (!h) return fail(nullptr, RQRCP_ERR_ARG, "h is NULL");
  int32_t w[4] = {0, 0, 0, 0};
  hipError_t e = hipMemcpyAsync(w, h->own_info, sizeof(w), hipMemcpyDeviceToHost, h->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
  if (e != hipSuccess) return fail_hip(h, e, "reading the info word");
  if (info_host) std::memcpy(info_host, w, sizeof(w));
  if (w[2]) return fail(h, RQRCP_ERR_TIMEOUT, "a grid-wide wait gave up: the factorization's results are invalid");
  if (w[0])
    return fail(h, RQRCP_ERR_NONFINITE, "a non-finite norm was met in block " + std::to_string(w[1] - 1));
  return RQRCP_OK;
}

rqrcp_status_t rqrcp_timing_enable(rqrcp_handle_t h, int enable) {
  if (!h) return fail(nullptr, RQRCP_ERR_ARG, "h is NULL");
  h->timing = enable != 0;
  return RQRCP_OK;
}

rqrcp_status_t rqrcp_timing_classes(rqrcp_handle_t h, uint32_t mask) {
  if (!h) return fail(nullptr, RQRCP_ERR_ARG, "h is NULL");
  h->timing_mask = mask;
  return RQRCP_OK;
}

rqrcp_status_t rqrcp_timing_read(rqrcp_handle_t h, int kclass, int64_t *launches, double *ms, double *flops,
                                 double *bytes) {
  if (!h) return fail(nullptr, RQRCP_ERR_ARG, "h is NULL");
  if (kclass < 0 || kclass >= RQRCP_K_COUNT) return fail(h, RQRCP_ERR_ARG, "kclass: unknown kernel class");
  int64_t cnt = 0;
  double tms = 0.0, tf = 0.0, tb = 0.0;
  std::vector<rqrcp_timing_rec> keep;
  for (const auto &r : h->recs) {
    if (r.kclass != kclass) { keep.push_back(r); continue; }
    float e = 0.f;
    hipError_t st = hipEventElapsedTime(&e, r.start, r.stop);
    if (st != hipSuccess) return fail_hip(h, st, "hipEventElapsedTime (synchronise the stream first)");
    ++cnt; tms += e; tf += r.flops; tb += r.bytes;
    h->free_events.push_back(r.start);
    h->free_events.push_back(r.stop);
  }
  h->recs.swap(keep);
  if (launches) *launches = cnt;
  if (ms) *ms = tms;
  if (flops) *flops = tf;
  if (bytes) *bytes = tb;
  return RQRCP_OK;
}

rqrcp_status_t rqrcp_factor_sizes(rqrcp_dtype_t dt, int64_t m, int64_t n, const rqrcp_opts_t *o, size_t *tau_elems,
                                  size_t *T_elems, size_t *S_elems, size_t *work_bytes) {
  FactorPlan P;
  rqrcp_status_t st = make_plan(nullptr, dt, m, n, o, &P);
  if (st != RQRCP_OK) return st;
  if (tau_elems) *tau_elems = (size_t)P.k;
  if (T_elems) *T_elems = (size_t)P.nblocks * P.b * P.b;
  if (S_elems) {
    size_t vs = 0;
    for (int64_t i = 0; i < P.nblocks; ++i) vs += (size_t)(n - i * P.b) * P.b;
    *S_elems = P.ortho ? vs + (size_t)P.nblocks * P.b + (size_t)P.nblocks * P.b * P.b * (P.diag ? 3 : 1) : 0;
  }
  if (work_bytes) *work_bytes = P.total;
  return RQRCP_OK;
}

rqrcp_status_t rqrcp_sketch(rqrcp_handle_t h, uint64_t seed, int64_t block, int64_t nsample, int64_t row0,
                            int64_t nrows, double *G, int64_t ldg) {
  if (!h) return fail(nullptr, RQRCP_ERR_ARG, "h is NULL");
  if (!G) return fail(h, RQRCP_ERR_ARG, "G is NULL");
  if (block < 0 || nsample < 0 || row0 < 0 || nrows < 0) return fail(h, RQRCP_ERR_ARG, "negative size or index");
  if (ldg < std::max<int64_t>(1, nsample)) return fail(h, RQRCP_ERR_ARG, "ldg < nsample");
  hipError_t e = launch_sketch(h->stream, seed, block, nsample, row0, nrows, G, ldg);
  if (e != hipSuccess) return fail_hip(h, e, "sketch");
  return RQRCP_OK;
}

#define CHK(call, where)                                  \
  do {                                                    \
    hipError_t e_ = (call);                               \
    if (e_ != hipSuccess) return fail_hip(h, e_, where);  \
  } while (0)

}  // extern "C"

namespace rq {
namespace {

// The per-block loop of Fig. 3 for storage type T (double: FP64 throughout;
// float: FP64 panel, T and pivoted QR of the sketch, FP32 matrix-core GEMMs,
// BF16 sketch product in the mixed mode).
template <typename T>
rqrcp_status_t factor_impl(rqrcp_handle_t h, const FactorPlan &P, const rqrcp_opts_t *o, T *A, int64_t lda,
                           int32_t *jpvt, double *tau, double *Tout, double *S, void *work) {
  constexpr bool F32 = std::is_same<T, float>::value;
  hipStream_t s = h->stream;
  const int64_t m = P.m, n = P.n, b = P.b, ks = P.ks;
  double *G = at<double>(work, P.G), *Y = at<double>(work, P.Y), *YT = at<double>(work, P.YT);
  double *Vb = at<double>(work, P.Vb), *VT = at<double>(work, P.VT), *Vt = at<double>(work, P.Vt);
  double *Wb = at<double>(work, P.Wb);
  double *gpart = at<double>(work, P.gpart), *Sg = at<double>(work, P.Sg);
  double *ppart = at<double>(work, P.ppart), *pred = at<double>(work, P.pred);
  double *qrec = at<double>(work, P.qrec), *qcand = at<double>(work, P.qcand);
  int32_t *piv = at<int32_t>(work, P.piv), *dest = at<int32_t>(work, P.dest);
  int32_t *moved = at<int32_t>(work, P.moved), *mcnt = at<int32_t>(work, P.mcnt);
  T *tmp = at<T>(work, P.tmp);
  int32_t *jtmp = at<int32_t>(work, P.jtmp);
  unsigned *bars = at<unsigned>(work, P.bars);
  // FP32-storage buffers
  double *Pw = at<double>(work, P.Pw);
  float *V32 = at<float>(work, P.V32), *VT32 = at<float>(work, P.VT32), *Vt32 = at<float>(work, P.Vt32);
  float *W32 = at<float>(work, P.W32);
  float *gpart32 = at<float>(work, P.gpart32), *spart = at<float>(work, P.spart);
  float *gpart32_aux = at<float>(work, P.gpart32_aux);
  float *G32 = at<float>(work, P.G32), *Y32 = at<float>(work, P.Y32);
  float *VS32 = at<float>(work, P.VS32), *TS32 = at<float>(work, P.TS32);
  void *Gb = at<void>(work, P.Gb);
  double *GVb = at<double>(work, P.GVb), *gpart_aux = at<double>(work, P.gpart_aux);
  double *vtpart = at<double>(work, P.vtpart);
  double *W2 = at<double>(work, P.W2);
  double *Z = at<double>(work, P.Z);
  double *Pc = at<double>(work, P.Pc), *Rp = at<double>(work, P.Rp);
  double *svdw = at<double>(work, P.svdw);
  double *r22 = at<double>(work, P.r22);
  float *Z32 = at<float>(work, P.Z);   // FP32 storage: Y X^T of the power iteration
  unsigned *scal = at<unsigned>(work, P.scal);
  int32_t *info = o->info;
  hipStream_t aux = P.pipe ? h->aux : nullptr;

  std::vector<size_t> vs_off(P.nblocks, 0);
  size_t vs_total = 0;
  for (int64_t i = 0; i < P.nblocks; ++i) {
    vs_off[i] = vs_total;
    vs_total += (size_t)(n - i * b) * b;
  }
  double *tauS = P.ortho ? S + vs_total : nullptr;
  double *TS = P.ortho ? tauS + P.nblocks * b : nullptr;
  double *UVd = P.diag ? TS + (size_t)P.nblocks * b * b : nullptr;   // U'_i, V'_i per block

  CHK(launch_zero_u32(s, bars, (size_t)P.nslots * kSlotWords), "zero barrier state");
  CHK(launch_zero_u32(s, Tout, (size_t)P.nblocks * b * b * 2), "zero T");
  if (info) CHK(launch_zero_u32(s, info, 4), "zero info");
  if (P.ortho)
    CHK(launch_zero_u32(s, S, (vs_total + P.nblocks * b + (size_t)P.nblocks * b * b * (P.diag ? 3 : 1)) * 2),
        "zero S");
  if (P.fixed) {
    T *Ac = at<T>(work, P.Acopy);
    CHK(launch_copy2d_t(s, A, lda, Ac, m, m, n), "copy A");
    CHK(launch_gather_cols_t(s, Ac, m, m, n, jpvt, n, A, lda), "permute A by jpvt");
  } else {
    CHK(launch_iota(s, jpvt, n), "jpvt identity");
  }
  int slot = 0;
  auto next_slot = [&](unsigned **bar, int **ab) {
    unsigned *base = bars + (size_t)slot * kSlotWords;
    ++slot;
    *bar = base;
    *ab = reinterpret_cast<int *>(base + kAbortWord);
  };
  auto run_qrcp = [&](double *Yp, int64_t ldy, int64_t k, int64_t ncols, int64_t steps, int64_t i) -> hipError_t {
    hipError_t e = launch_zero_u32(s, mcnt, 1);
    if (e != hipSuccess) return e;
    QrcpSmall q{};
    q.Y = Yp; q.ldy = ldy; q.k = (int)k; q.ncols = (int)ncols; q.nsteps = (int)steps;
    q.piv = piv; q.dest = dest; q.moved = moved; q.moved_cnt = mcnt;
    q.rec = qrec; q.cand = qcand; q.info = info; q.block_index = (int)i; q.limit_ticks = h->limit_ticks;
    next_slot(&q.bar, &q.abort_flag);
    return launch_qrcp_small(s, q);
  };
  // offset of block i's sketch in opts.G: every earlier block was sampled
  auto goff_of = [&](int64_t i) {
    size_t off = 0;
    for (int64_t j = 0; j < i; ++j) off += (size_t)ks * (m - j * b);
    return off;
  };
  // Overlapped schedule (FP64, permutation pivots).  The sketch of block i+1
  // is Y_{i+1} = G_{i+1} C'(b_i:, :) with C' = C - (V T^T) W the updated
  // trailing matrix; it equals G_{i+1} C(b_i:, :) - (G_{i+1} (V T^T)(b_i:, :)) W,
  // whose first product reads C before the update and runs on the auxiliary
  // stream during the panel, and whose correction is two thin products on
  // the main stream.  The trailing update of block i then runs on the
  // auxiliary stream during the pivoted QR of block i+1, and block i+1's
  // column moves wait for it.  (Same quantity, other rounding order.)
  bool y_ready = false;       // Y already holds this block's sketch product
  bool upd_pending = false;   // the previous block's update runs on the auxiliary stream
  auto join_update = [&]() -> hipError_t {
    if (!upd_pending) return hipSuccess;
    upd_pending = false;
    return hipStreamWaitEvent(s, h->ev_upd, 0);
  };
  // the previous block's diagonalisation runs on the side stream beside this
  // block's sketch and its QR; it must end before S_i touches the rows above
  bool diag_pending = false;
  auto join_diag = [&]() -> hipError_t {
    if (!diag_pending) return hipSuccess;
    diag_pending = false;
    return hipStreamWaitEvent(s, h->ev_diag, 0);
  };

  for (int64_t i = 0; i < P.nblocks; ++i) {
    const int64_t r0 = i * b, bi = std::min(b, P.k - r0), mi = m - r0, ni = n - r0;
    T *X = A + r0 + r0 * lda;
    const bool pipe_next =
        aux && !P.fixed && i + 1 < P.nblocks && !block_is_classical_tail(P, i + 1) && ni > bi;
    if (!P.fixed) {
      if (block_is_classical_tail(P, i)) {
        CHK(join_update(), "wait for the trailing update");
        // last block of Fig. 3: classical QRCP of the remaining block
        {
          ScopedTimer tq(h, RQRCP_K_QRCP, qrcp_flops((double)mi, (double)ni, (double)bi), 16.0 * mi * ni);
          CHK(launch_to_f64(s, X, lda, Y, mi, mi, ni), "copy last block");
          CHK(run_qrcp(Y, mi, mi, ni, bi, i), "pivoted QR of the last block");
        }
        ScopedTimer tm(h, RQRCP_K_MOVES, 0.0, 32.0 * bi * m);
        CHK(launch_apply_moves<T>(s, A, lda, m, r0, moved, mcnt, dest, (int)(2 * bi), tmp, jpvt, jtmp),
            "move columns");
      } else {
        const int64_t yrows = P.ortho ? bi : ks;
        if (!y_ready) {
          const double *Gi;
          if (o->G) {
            Gi = o->G + goff_of(i);
          } else {
            ScopedTimer tg(h, RQRCP_K_SKETCH, 0.0, 8.0 * ks * mi);
            CHK(launch_sketch(s, o->seed, i, ks, r0, mi, G, ks), "sketch");
            Gi = G;
          }
          // Y_i = G_i X_i (Section 4.1, eq. defY).  The orthonormal variant runs
          // the QR of Y_i^T without pivoting, whose first b_i reflectors depend
          // only on the first b_i rows of Y_i: only those are formed.
          {
            ScopedTimer ts(h, RQRCP_K_SAMPLE_GEMM, 2.0 * yrows * ni * mi,
                           (double)sizeof(T) * mi * ni + 8.0 * (yrows * mi + yrows * ni));
            if constexpr (!F32) {
              GemmF64 gy{false, false, yrows, ni, mi, Gi, ks, X, lda, Y, ks, 1.0, 0.0};
              CHK(launch_gemm_f64(s, gy, gpart), "sketch product");
            } else if (P.mixed) {
              CHK(launch_g_to_bf16(s, Gi, ks, yrows, mi, Gb, mi), "sketch to BF16");
              CHK(launch_sample_bf16(s, yrows, ni, mi, Gb, mi, X, lda, spart, Y, ks), "BF16 sketch product");
            } else {
              CHK(launch_copy_f64_f32(s, Gi, ks, G32, ks, yrows, mi), "sketch to FP32");
              GemmF32 gy{false, false, yrows, ni, mi, G32, ks, X, lda, Y32, ks, 1.f, 0.f};
              CHK(launch_gemm<float>(s, gy, gpart32), "FP32 sketch product");
              CHK(launch_copy_f32_f64(s, Y32, ks, Y, ks, yrows, ni), "sketch to FP64");
            }
          }
        }
        // Section 6.3: q steps of the power iteration in the row form of the
        // sample, Y_i := (Y_i X_i^T) X_i, so that Y_i = G_i X_i (X_i^T X_i)^q
        // (also on a sample that the previous block formed and corrected:
        // its update ran on this stream, so X_i is the updated block)
        if constexpr (!F32) {
          for (int q = 0; q < P.power; ++q) {
            ScopedTimer tp(h, RQRCP_K_SAMPLE_GEMM, 4.0 * yrows * ni * mi,
                           16.0 * mi * ni + 16.0 * yrows * (mi + ni));
            GemmF64 gz{false, true, yrows, mi, ni, Y, ks, X, lda, Z, ks, 1.0, 0.0};
            CHK(launch_gemm_f64(s, gz, gpart), "power iteration Y X^T");
            GemmF64 gy{false, false, yrows, ni, mi, Z, ks, X, lda, Y, ks, 1.0, 0.0};
            CHK(launch_gemm_f64(s, gy, gpart), "power iteration (Y X^T) X");
          }
        } else if (P.power > 0) {
          // FP32 storage: the steps on FP32 matrix cores from an FP32 copy of
          // the sketch, which is scaled by a power of two before each step
          // (its entries grow like |X|^2q, beyond FP32's range for large q;
          // a scalar factor changes no pivot and no S_i)
          CHK(launch_copy_f64_f32(s, Y, ks, Y32, ks, yrows, ni), "sketch to FP32");
          for (int q = 0; q < P.power; ++q) {
            ScopedTimer tp(h, RQRCP_K_SAMPLE_GEMM, 4.0 * yrows * ni * mi,
                           8.0 * mi * ni + 8.0 * yrows * (mi + ni));
            CHK(launch_normalise_pow2(s, Y32, ks, yrows, ni, scal), "scale the sketch");
            GemmF32 gz{false, true, yrows, mi, ni, Y32, ks, X, lda, Z32, ks, 1.f, 0.f};
            CHK(launch_gemm<float>(s, gz, gpart32), "power iteration Y X^T");
            GemmF32 gy{false, false, yrows, ni, mi, Z32, ks, X, lda, Y32, ks, 1.f, 0.f};
            CHK(launch_gemm<float>(s, gy, gpart32), "power iteration (Y X^T) X");
          }
          CHK(launch_copy_f32_f64(s, Y32, ks, Y, ks, yrows, ni), "sketch to FP64");
        }
        y_ready = false;
        if (!P.ortho) {
          {
            ScopedTimer tq(h, RQRCP_K_QRCP, qrcp_flops((double)ks, (double)ni, (double)bi), 8.0 * ks * ni);
            CHK(run_qrcp(Y, ks, ks, ni, bi, i), "pivoted QR of the sketch");
          }
          CHK(join_update(), "wait for the trailing update");
          ScopedTimer tm(h, RQRCP_K_MOVES, 0.0, 32.0 * bi * m);
          CHK(launch_apply_moves<T>(s, A, lda, m, r0, moved, mcnt, dest, (int)(2 * bi), tmp, jpvt, jtmp),
              "move columns");
        } else {
          // Section 4.2: unpivoted QR of Y_i^T, first b_i steps -> S_i = I - VS TS VS^T
          double *VS = S + vs_off[i];
          double *TSi = TS + (size_t)i * b * b;
          ScopedTimer to(h, RQRCP_K_ORTHO, 2.0 * ni * bi * bi + 4.0 * m * ni * bi + 2.0 * m * bi * bi,
                         (double)sizeof(T) * 3.0 * m * ni + 24.0 * ni * bi);
          CHK(launch_transpose(s, Y, ks, YT, ni, bi, ni), "transpose sketch");
          PanelQR pq{};
          pq.P = YT; pq.ldp = ni; pq.mi = ni; pq.nb = (int)bi;
          pq.tau = tauS + i * b; pq.V = VS; pq.ldv = ni;
          pq.part = ppart; pq.red = pred; pq.info = info; pq.block_index = (int)i; pq.limit_ticks = h->limit_ticks;
          next_slot(&pq.bar, &pq.abort_flag);
          CHK(launch_panel_qr(s, pq), "QR of the sketch");
          CHK(launch_gram(s, VS, ni, ni, bi, Sg, gpart), "V_S^T V_S");
          CHK(launch_wy_t(s, (int)bi, tauS + i * b, Sg, TSi, b), "T of the sketch reflectors");
          // A(0:m, r0:n) <- A(0:m, r0:n) (I - VS TS VS^T), all m rows
          CHK(join_diag(), "wait for the previous block's diagonalisation");
          T *Ac = A + r0 * lda;
          if constexpr (!F32) {
            GemmF64 g1{false, false, m, bi, ni, Ac, lda, VS, ni, Vb, m, 1.0, 0.0};
            CHK(launch_gemm_f64(s, g1, gpart), "A VS");
            GemmF64 g2{false, false, m, bi, bi, Vb, m, TSi, b, Vt, m, 1.0, 0.0};
            CHK(launch_gemm_f64(s, g2, gpart), "(A VS) TS");
            GemmF64 g3{false, true, m, ni, bi, Vt, m, VS, ni, Ac, lda, -1.0, 1.0};
            CHK(launch_gemm_f64(s, g3, gpart), "A -= (A VS TS) VS^T");
          } else {
            CHK(launch_copy_f64_f32(s, VS, ni, VS32, ni, ni, bi), "VS to FP32");
            CHK(launch_copy_f64_f32(s, TSi, b, TS32, b, bi, bi), "TS to FP32");
            GemmF32 g1{false, false, m, bi, ni, Ac, lda, VS32, ni, V32, m, 1.f, 0.f};
            CHK(launch_gemm<float>(s, g1, gpart32), "A VS");
            GemmF32 g2{false, false, m, bi, bi, V32, m, TS32, b, Vt32, m, 1.f, 0.f};
            CHK(launch_gemm<float>(s, g2, gpart32), "(A VS) TS");
            GemmF32 g3{false, true, m, ni, bi, Vt32, m, VS32, ni, Ac, lda, -1.f, 1.f};
            CHK(launch_gemm<float>(s, g3, gpart32), "A -= (A VS TS) VS^T");
          }
        }
      }
    }
    // next block's sketch and the product G_{i+1} C(b_i:, :) on the auxiliary
    // stream: C is final here (moved, not yet updated), and the panel does
    // not touch it
    const double *Gn = nullptr;
    // Workgroups of the auxiliary products: those beside the panel take the
    // CUs it leaves (the panel holds pw, one workgroup per CU, its LDS filling
    // the CU), so that the next block's sample product ends with the panel
    // rather than beside W; those beside the pivoted QR of the sketch (at
    // most 128 workgroups) take half the CUs
    int prw = 0;
    const int pw = panel_config(mi, (int)bi, &prw);
    const int beside_panel = pw > 0 && pw <= h->ncu / 2 ? h->ncu - pw : h->ncu / 2, beside_qrcp = h->ncu / 2;
    if constexpr (F32) if (pipe_next) {
      // FP32 storage (mixed): the BF16 sketch product of block i+1 from the
      // moved, not yet updated C, beside the panel
      CHK(hipEventRecord(h->ev_moves, s), "fork event");
      CHK(hipStreamWaitEvent(aux, h->ev_moves, 0), "auxiliary stream wait");
      const int64_t mn = mi - bi, nn = ni - bi;
      if (o->G) {
        Gn = o->G + goff_of(i + 1);
      } else {
        ScopedTimer tg(h, RQRCP_K_SKETCH, 0.0, 8.0 * ks * mn, aux);
        CHK(launch_sketch(aux, o->seed, i + 1, ks, r0 + bi, mn, G, ks, beside_panel), "sketch");
        Gn = G;
      }
      ScopedTimer ts(h, RQRCP_K_SAMPLE_GEMM, 2.0 * ks * nn * mn, 4.0 * mn * nn + 2.0 * ks * mn + 8.0 * ks * nn, aux);
      CHK(launch_g_to_bf16(aux, Gn, ks, ks, mn, Gb, mn, beside_panel), "sketch to BF16");
      CHK(launch_sample_bf16(aux, ks, nn, mn, Gb, mn, X + bi + bi * lda, lda, spart, Y, ks, beside_panel),
          "BF16 sketch product of the next block");
    }
    if constexpr (!F32) if (pipe_next) {
      CHK(hipEventRecord(h->ev_moves, s), "fork event");
      CHK(hipStreamWaitEvent(aux, h->ev_moves, 0), "auxiliary stream wait");
      const int64_t mn = mi - bi, nn = ni - bi;
      if (o->G) {
        Gn = o->G + goff_of(i + 1);
      } else {
        ScopedTimer tg(h, RQRCP_K_SKETCH, 0.0, 8.0 * ks * mn, aux);
        CHK(launch_sketch(aux, o->seed, i + 1, ks, r0 + bi, mn, G, ks, beside_panel), "sketch");
        Gn = G;
      }
      {
        ScopedTimer ts(h, RQRCP_K_SAMPLE_GEMM, 2.0 * ks * nn * mn, 8.0 * (mn * nn + ks * mn + ks * nn), aux);
        GemmF64 gy{false, false, ks, nn, mn, Gn, ks, X + bi + bi * lda, lda, Y, ks, 1.0, 0.0};
        gy.max_wg = beside_panel;
        CHK(launch_gemm_f64(aux, gy, gpart_aux), "sketch product of the next block");
      }
    }
    // Fig. 3's in-block pivot P-hat (permutation form): a QR with column
    // pivoting of the panel.  Its pivot order depends on the columns only
    // through their Gram matrix, which the triangular factor R' of an
    // unpivoted QR of the panel shares (the Remark of Section 2), so the
    // order is read off a QRCP of the b_i x b_i R'; the saved panel is then
    // restored, its columns (all m rows) and jpvt permuted, and the pivoted
    // panel factored below like any other.
    if (P.panel_pivot && !block_is_classical_tail(P, i)) {
      {
        ScopedTimer tp(h, RQRCP_K_PANEL, 2.0 * mi * bi * bi - 2.0 * bi * bi * bi / 3.0, 40.0 * mi * bi);
        // FP64 storage factors a saved copy's original in place and restores
        // it; FP32 storage factors an FP64 copy and leaves the panel alone
        PanelQR pq{};
        if constexpr (F32) {
          CHK(launch_copy_f32_f64(s, X, lda, Pw, mi, mi, bi), "panel to FP64");
          pq.P = Pw; pq.ldp = mi;
        } else {
          CHK(launch_copy2d(s, X, lda, Pc, mi, mi, bi), "save the panel");
          pq.P = X; pq.ldp = lda;
        }
        pq.mi = mi; pq.nb = (int)bi;
        pq.tau = tau + r0; pq.V = Vb; pq.ldv = mi;
        pq.VT = nullptr; pq.ldvt = b;
        pq.part = ppart; pq.red = pred; pq.info = info; pq.block_index = (int)i; pq.limit_ticks = h->limit_ticks;
        next_slot(&pq.bar, &pq.abort_flag);
        CHK(launch_panel_qr(s, pq), "unpivoted QR of the panel");
        CHK(launch_extract_r(s, pq.P, pq.ldp, bi, bi, Rp, bi), "R' of the panel");
      }
      {
        ScopedTimer tq(h, RQRCP_K_QRCP, qrcp_flops((double)bi, (double)bi, (double)bi), 8.0 * bi * bi);
        CHK(run_qrcp(Rp, bi, bi, bi, bi, i), "pivoted QR of R'");
      }
      ScopedTimer tm(h, RQRCP_K_MOVES, 0.0, 16.0 * mi * bi + 32.0 * bi * m);
      if constexpr (!F32) CHK(launch_copy2d(s, Pc, mi, X, lda, mi, bi), "restore the panel");
      CHK(launch_apply_moves<T>(s, A, lda, m, r0, moved, mcnt, dest, (int)(2 * bi), tmp, jpvt, jtmp),
          "move the panel's columns");
    }
    // panel: unpivoted Householder QR of A(r0:m, r0:r0+bi) in FP64
    {
      ScopedTimer tp(h, RQRCP_K_PANEL, 2.0 * mi * bi * bi - 2.0 * bi * bi * bi / 3.0, 24.0 * mi * bi);
      PanelQR pq{};
      if constexpr (F32) {
        CHK(launch_copy_f32_f64(s, X, lda, Pw, mi, mi, bi), "panel to FP64");
        pq.P = Pw; pq.ldp = mi;
      } else {
        pq.P = X; pq.ldp = lda;
      }
      pq.mi = mi; pq.nb = (int)bi;
      pq.tau = tau + r0; pq.V = Vb; pq.ldv = mi;
      pq.VT = VT; pq.ldvt = b;
      pq.part = ppart; pq.red = pred; pq.info = info; pq.block_index = (int)i; pq.limit_ticks = h->limit_ticks;
      next_slot(&pq.bar, &pq.abort_flag);
      CHK(launch_panel_qr(s, pq), "panel QR");
      if constexpr (F32) CHK(launch_copy_f64_f32(s, Pw, mi, X, lda, mi, bi), "panel to FP32");
    }
    double *Ti = Tout + (size_t)i * b * b;
    if (ni <= bi) {
      ScopedTimer tt(h, RQRCP_K_TFACTOR, (double)bi * bi * bi / 3.0, 16.0 * bi * bi);
      CHK(launch_gram(s, Vb, mi, mi, bi, Sg, gpart), "V^T V");
      CHK(launch_wy_t(s, (int)bi, tau + r0, Sg, Ti, b), "T factor");
    } else {
      // C <- (I - V T V^T)^T C = C - (V T^T) (V^T C)   (Section 5.1).  W = V^T C
      // does not need T: T is formed on the side stream meanwhile (one
      // workgroup per block row would leave most of the chip idle).
      T *C = X + bi * lda;
      const double nc = (double)(ni - bi);
      // FP64 applies the update as C - V (T^T W) (every block, so that a
      // fixed-pivot refactorization repeats the forward's operations): in the
      // overlapped schedule the correction of the next sketch is then
      // (G V(b_i:, :)) (T^T W), whose first factor needs only V and runs on
      // the auxiliary stream beside W; no V T^T is formed
      const bool reassoc = !F32;
      // At b = 256 in FP64, S = V^T V comes from W's own launch as two more
      // 128-column tiles ([S | W] = V^T [V | C], S directly in front of W):
      // nothing can share a CU with W's workgroups, so S beside W on the side
      // stream waited for W's last workgroups, and T after it
      const bool fuse_s = reassoc && bi == b && b == 256;
      if (!fuse_s) {
        CHK(hipEventRecord(h->fork_ev, s), "fork event");
        CHK(hipStreamWaitEvent(h->side, h->fork_ev, 0), "side stream wait");
        {
          ScopedTimer tt(h, RQRCP_K_TFACTOR, (double)bi * bi * bi / 3.0, 16.0 * bi * bi, h->side);
          CHK(launch_gram(h->side, Vb, mi, mi, bi, Sg, vtpart), "V^T V");
          CHK(launch_wy_t(h->side, (int)bi, tau + r0, Sg, Ti, b), "T factor");
        }
        if (!reassoc) {
          // V T^T right after T, also beside W (its own split-K buffer)
          ScopedTimer t1(h, RQRCP_K_VT_GEMM, 2.0 * mi * bi * bi, 8.0 * (2.0 * mi * bi + bi * bi), h->side);
          GemmF64 gv{false, true, mi, bi, bi, Vb, mi, Ti, b, Vt, mi, 1.0, 0.0};
          CHK(launch_gemm_f64(h->side, gv, vtpart), "V T^T");
          if constexpr (F32) CHK(launch_copy_f64_f32(h->side, Vt, mi, Vt32, mi, mi, bi), "V T^T to FP32");
        }
        CHK(hipEventRecord(h->join_ev, h->side), "join event");
      }
      {
        ScopedTimer t2(h, RQRCP_K_W_GEMM, 2.0 * bi * nc * mi,
                       (double)sizeof(T) * (mi * nc + mi * bi + bi * nc));
        if constexpr (!F32) {
          if (fuse_s) {
            GemmF64 gw{false, false, bi, ni, mi, VT, b, C, lda, Sg, bi, 1.0, 0.0};
            gw.wprod = true;
            gw.B2 = Vb; gw.ldb2 = mi; gw.n2 = bi;
            CHK(launch_gemm_f64(s, gw, gpart), "V^T [V | C]");
          } else {
            GemmF64 gw{false, false, bi, ni - bi, mi, VT, b, C, lda, Wb, bi, 1.0, 0.0};
            gw.wprod = true;
            CHK(launch_gemm_f64(s, gw, gpart), "V^T C");
          }
        } else {
          CHK(launch_copy_f64_f32(s, VT, b, VT32, b, bi, mi), "V^T to FP32");
          GemmF32 gw{false, false, bi, ni - bi, mi, VT32, b, C, lda, W32, bi, 1.f, 0.f};
          CHK(launch_gemm<float>(s, gw, gpart32), "V^T C");
        }
      }
      if (pipe_next) {
          // G_{i+1} V(b_i:, :) on the auxiliary stream after W (beside T^T W;
          // beside W itself it slowed W by a sixth)
          CHK(hipEventRecord(h->ev_w, s), "W event");
          CHK(hipStreamWaitEvent(aux, h->ev_w, 0), "auxiliary stream wait for W");
          const int64_t mn = mi - bi;
          ScopedTimer tc(h, RQRCP_K_SAMPLE_GEMM, 2.0 * ks * bi * mn, 8.0 * (ks * mn + mn * bi + ks * bi), aux);
          GemmF64 g1{false, false, ks, bi, mn, Gn, ks, Vb + bi, mi, GVb, ks, 1.0, 0.0};
          g1.max_wg = beside_qrcp;
          CHK(launch_gemm_f64(aux, g1, gpart_aux), "G V");
          CHK(hipEventRecord(h->ev_ypre, aux), "correction factor event");
        }
      if (fuse_s) {
        ScopedTimer tt(h, RQRCP_K_TFACTOR, (double)bi * bi * bi / 3.0, 16.0 * bi * bi);
        CHK(launch_wy_t(s, (int)bi, tau + r0, Sg, Ti, b), "T factor");
      } else {
        CHK(hipStreamWaitEvent(s, h->join_ev, 0), reassoc ? "join T" : "join T and V T^T");
      }
      if constexpr (!F32) {
        ScopedTimer t1(h, RQRCP_K_VT_GEMM, 2.0 * bi * bi * nc, 8.0 * (bi * bi + 2.0 * bi * nc));
        GemmF64 gw2{true, false, bi, ni - bi, bi, Ti, b, Wb, bi, W2, bi, 1.0, 0.0};
        CHK(launch_gemm_f64(s, gw2, gpart), "T^T W");
      }
      if (pipe_next) {
        if constexpr (!F32) {
          // the update on the auxiliary stream, the next sketch's correction here
          if (P.power > 0) {
            // the next block's power steps read the updated block: the update
            // runs here, on the whole chip
            ScopedTimer t3(h, RQRCP_K_UPDATE_GEMM, 2.0 * mi * nc * bi,
                           (double)sizeof(T) * (2.0 * mi * nc + mi * bi + bi * nc));
            GemmF64 gu{false, false, mi, ni - bi, bi, Vb, mi, W2, bi, C, lda, -1.0, 1.0, true};
            CHK(launch_gemm_f64(s, gu, gpart), "C -= V (T^T W)");
          } else {
            CHK(hipEventRecord(h->ev_vt, s), "update fork event");
            CHK(hipStreamWaitEvent(aux, h->ev_vt, 0), "auxiliary stream wait");
            {
              ScopedTimer t3(h, RQRCP_K_UPDATE_GEMM, 2.0 * mi * nc * bi,
                             (double)sizeof(T) * (2.0 * mi * nc + mi * bi + bi * nc), aux);
              GemmF64 gu{false, false, mi, ni - bi, bi, Vb, mi, W2, bi, C, lda, -1.0, 1.0, true};
              gu.max_wg = beside_qrcp;
              CHK(launch_gemm_f64(aux, gu, gpart_aux), "C -= V (T^T W)");
            }
            CHK(hipEventRecord(h->ev_upd, aux), "update event");
            upd_pending = true;
          }
          CHK(hipStreamWaitEvent(s, h->ev_ypre, 0), "wait for the next sketch product and G V");
          ScopedTimer tc(h, RQRCP_K_SAMPLE_GEMM, 2.0 * ks * bi * nc, 8.0 * (ks * bi + 2.0 * ks * nc + bi * nc));
          GemmF64 g2{false, false, ks, ni - bi, bi, GVb, ks, W2, bi, Y, ks, -1.0, 1.0};
          CHK(launch_gemm_f64(s, g2, gpart), "Y -= (G V) (T^T W)");
          y_ready = true;
        } else {
          // FP32 storage: the update C -= (V T^T) W on the auxiliary stream;
          // the correction of the next sketch here, in FP64, as
          // ((G V) T^T) W with W widened from FP32
          if (P.power > 0) {
            ScopedTimer t3(h, RQRCP_K_UPDATE_GEMM, 2.0 * mi * nc * bi,
                           (double)sizeof(T) * (2.0 * mi * nc + mi * bi + bi * nc));
            GemmF32 gu{false, false, mi, ni - bi, bi, Vt32, mi, W32, bi, C, lda, -1.f, 1.f, true};
            CHK(launch_gemm<float>(s, gu, gpart32), "C -= (V T^T) W");
          } else {
            CHK(hipEventRecord(h->ev_vt, s), "update fork event");
            CHK(hipStreamWaitEvent(aux, h->ev_vt, 0), "auxiliary stream wait");
            {
              ScopedTimer t3(h, RQRCP_K_UPDATE_GEMM, 2.0 * mi * nc * bi,
                             (double)sizeof(T) * (2.0 * mi * nc + mi * bi + bi * nc), aux);
              GemmF32 gu{false, false, mi, ni - bi, bi, Vt32, mi, W32, bi, C, lda, -1.f, 1.f, true};
              gu.max_wg = beside_qrcp;
              CHK(launch_gemm<float>(aux, gu, gpart32_aux), "C -= (V T^T) W");
            }
            CHK(hipEventRecord(h->ev_upd, aux), "update event");
            upd_pending = true;
          }
          CHK(hipStreamWaitEvent(s, h->ev_ypre, 0), "wait for the next sketch product and G V");
          ScopedTimer tc(h, RQRCP_K_SAMPLE_GEMM, 2.0 * ks * bi * nc + 2.0 * ks * bi * bi,
                         8.0 * (ks * bi + 2.0 * ks * nc + bi * nc) + 4.0 * bi * nc);
          CHK(launch_copy_f32_f64(s, W32, bi, Wb, bi, bi, ni - bi), "W to FP64");
          // (G V) T^T into Vt (V T^T went to FP32 on the side stream, joined above)
          GemmF64 g1{false, true, ks, bi, bi, GVb, ks, Ti, b, Vt, ks, 1.0, 0.0};
          CHK(launch_gemm_f64(s, g1, gpart), "(G V) T^T");
          GemmF64 g2{false, false, ks, ni - bi, bi, Vt, ks, Wb, bi, Y, ks, -1.0, 1.0};
          CHK(launch_gemm_f64(s, g2, gpart), "Y -= ((G V) T^T) W");
          y_ready = true;
        }
      } else {
        ScopedTimer t3(h, RQRCP_K_UPDATE_GEMM, 2.0 * mi * nc * bi,
                       (double)sizeof(T) * (2.0 * mi * nc + mi * bi + bi * nc));
        if constexpr (!F32) {
          GemmF64 gu{false, false, mi, ni - bi, bi, Vb, mi, W2, bi, C, lda, -1.0, 1.0, true};
          CHK(launch_gemm_f64(s, gu, gpart), "C -= V (T^T W)");
        } else {
          GemmF32 gu{false, false, mi, ni - bi, bi, Vt32, mi, W32, bi, C, lda, -1.f, 1.f, true};
          CHK(launch_gemm<float>(s, gu, gpart32), "C -= (V T^T) W");
        }
      }
    }
    // Section 6.2: R22 = U' D V'^T; U-tilde = Q-tilde diag(U', I) puts U'^T on
    // the block's rows right of it, V' multiplies its columns above it, and
    // the triangle becomes D (orthonormal pivoting; in FP64, on widened copies
    // with FP32 storage).  None of it is read by the next block's sketch,
    // power steps or QR of the sketch (rows and columns past this block; their
    // own buffers), so it runs on the side stream beside them
    if (P.diag) {
      double *Ud = UVd + (size_t)i * 2 * b * b, *Vd = Ud + (size_t)b * b;
      hipStream_t sd = h->side;
      CHK(hipEventRecord(h->fork_ev, s), "fork event");
      CHK(hipStreamWaitEvent(sd, h->fork_ev, 0), "side stream wait");
      {
        ScopedTimer td(h, RQRCP_K_OTHER, 22.0 * bi * bi * bi + 2.0 * bi * bi * (ni - bi + r0),
                       16.0 * bi * (ni - bi + r0) + 24.0 * bi * bi, sd);
        if constexpr (!F32) {
          SvdSmall sv{X, lda, (int)bi, Ud, b, Vd, b, svdw, nullptr, nullptr, info, h->limit_ticks};
          next_slot(&sv.bar, &sv.abort_flag);
          CHK(launch_svd_small(sd, sv), "SVD of the block's triangle");
          if (ni > bi) {
            GemmF64 gu{true, false, bi, ni - bi, bi, Ud, b, X + bi * lda, lda, Wb, bi, 1.0, 0.0};
            CHK(launch_gemm_f64(sd, gu, vtpart), "U'^T times the block's rows");
            CHK(launch_copy2d(sd, Wb, bi, X + bi * lda, lda, bi, ni - bi), "rows of the block");
          }
          if (r0 > 0) {
            GemmF64 gv{false, false, r0, bi, bi, A + r0 * lda, lda, Vd, b, Vt, r0, 1.0, 0.0};
            CHK(launch_gemm_f64(sd, gv, vtpart), "columns above the block times V'");
            CHK(launch_copy2d(sd, Vt, r0, A + r0 * lda, lda, r0, bi), "columns above the block");
          }
        } else {
          // the block (its reflectors below the triangle come back unchanged:
          // FP32 -> FP64 -> FP32 is exact, and the SVD writes only the triangle)
          CHK(launch_copy_f32_f64(sd, X, lda, r22, b, bi, bi), "triangle to FP64");
          SvdSmall sv{r22, b, (int)bi, Ud, b, Vd, b, svdw, nullptr, nullptr, info, h->limit_ticks};
          next_slot(&sv.bar, &sv.abort_flag);
          CHK(launch_svd_small(sd, sv), "SVD of the block's triangle");
          CHK(launch_copy_f64_f32(sd, r22, b, X, lda, bi, bi), "triangle to FP32");
          if (ni > bi) {
            CHK(launch_copy_f32_f64(sd, X + bi * lda, lda, Vt, bi, bi, ni - bi), "rows of the block to FP64");
            GemmF64 gu{true, false, bi, ni - bi, bi, Ud, b, Vt, bi, Wb, bi, 1.0, 0.0};
            CHK(launch_gemm_f64(sd, gu, vtpart), "U'^T times the block's rows");
            CHK(launch_copy_f64_f32(sd, Wb, bi, X + bi * lda, lda, bi, ni - bi), "rows of the block");
          }
          if (r0 > 0) {
            CHK(launch_copy_f32_f64(sd, A + r0 * lda, lda, Vt, r0, r0, bi), "columns above the block to FP64");
            GemmF64 gv{false, false, r0, bi, bi, Vt, r0, Vd, b, Wb, r0, 1.0, 0.0};
            CHK(launch_gemm_f64(sd, gv, vtpart), "columns above the block times V'");
            CHK(launch_copy_f64_f32(sd, Wb, r0, A + r0 * lda, lda, r0, bi), "columns above the block");
          }
        }
      }
      CHK(hipEventRecord(h->ev_diag, sd), "diagonalisation event");
      diag_pending = true;
    }
  }
  CHK(join_diag(), "wait for the last diagonalisation");
  CHK(join_update(), "wait for the trailing update");
  (void)piv;
  return RQRCP_OK;
}

// Checks of rqrcp_factor's arguments other than the workspace.
rqrcp_status_t factor_args(rqrcp_handle_t h, rqrcp_dtype_t dt, int64_t m, int64_t n, void *Av, int64_t lda,
                           int32_t *jpvt, double *tau, double *T, double *S, const rqrcp_opts_t *o,
                           FactorPlan *P) {
  rqrcp_status_t st = make_plan(h, dt, m, n, o, P);
  if (st != RQRCP_OK) return st;
  if (!Av) return fail(h, RQRCP_ERR_ARG, "A is NULL");
  if (lda < m) return fail(h, RQRCP_ERR_ARG, "lda must be >= m");
  if (!jpvt) return fail(h, RQRCP_ERR_ARG, "jpvt is NULL");
  if (!tau) return fail(h, RQRCP_ERR_ARG, "tau is NULL");
  if (!T) return fail(h, RQRCP_ERR_ARG, "T is NULL");
  if (P->ortho && !S) return fail(h, RQRCP_ERR_ARG, "S is NULL (required for ORTHO)");
  if (!P->ortho && S) return fail(h, RQRCP_ERR_ARG, "S must be NULL for PERM");
  return RQRCP_OK;
}

}  // namespace
}  // namespace rq

extern "C" {

rqrcp_status_t rqrcp_factor_noalloc(rqrcp_handle_t h, rqrcp_dtype_t dt, int64_t m, int64_t n, void *Av,
                                    int64_t lda, int32_t *jpvt, double *tau, double *T, double *S,
                                    const rqrcp_opts_t *o) {
  if (!h) return fail(nullptr, RQRCP_ERR_ARG, "h is NULL");
  FactorPlan P;
  rqrcp_status_t st = factor_args(h, dt, m, n, Av, lda, jpvt, tau, T, S, o, &P);
  if (st != RQRCP_OK) return st;
  if (P.total > (size_t)RQRCP_NOALLOC_WORK_BYTES)
    return fail(h, RQRCP_ERR_WORKSPACE,
                "this problem needs " + std::to_string(P.total) + " bytes of workspace; rqrcp_factor_noalloc has " +
                    std::to_string((size_t)RQRCP_NOALLOC_WORK_BYTES) + " (use rqrcp_factor with a workspace)");
  if (!h->scratch) return fail(h, RQRCP_ERR_HIP, "no scratch address for this device");
  int dev = -1;
  const hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return fail_hip(h, e, "hipGetDevice");
  if (dev != h->device) return fail(h, RQRCP_ERR_ARG, "the current device is not the handle's device");
  // every region of the workspace is written before it is read, and the
  // parts that must start at zero (barrier state) are cleared by fill kernels
  rqrcp_opts_t oc = *o;
  if (!oc.info) oc.info = h->own_info;
  if (dt == RQRCP_F64)
    return factor_impl<double>(h, P, &oc, static_cast<double *>(Av), lda, jpvt, tau, T, S, h->scratch);
  return factor_impl<float>(h, P, &oc, static_cast<float *>(Av), lda, jpvt, tau, T, S, h->scratch);
}

rqrcp_status_t rqrcp_factor(rqrcp_handle_t h, rqrcp_dtype_t dt, int64_t m, int64_t n, void *Av, int64_t lda,
                            int32_t *jpvt, double *tau, double *T, double *S, const rqrcp_opts_t *o, void *work,
                            size_t work_bytes) {
  if (!h) return fail(nullptr, RQRCP_ERR_ARG, "h is NULL");
  FactorPlan P;
  rqrcp_status_t st = factor_args(h, dt, m, n, Av, lda, jpvt, tau, T, S, o, &P);
  if (st != RQRCP_OK) return st;
  if (!work) return fail(h, RQRCP_ERR_WORKSPACE, "work is NULL");
  if (work_bytes < P.total) return fail(h, RQRCP_ERR_WORKSPACE, "work_bytes smaller than rqrcp_factor_sizes");
  if (reinterpret_cast<uintptr_t>(work) % 256) return fail(h, RQRCP_ERR_WORKSPACE, "work must be 256-byte aligned");
  rqrcp_opts_t oc = *o;
  if (!oc.info) oc.info = h->own_info;   // flags stay readable through rqrcp_check
  if (dt == RQRCP_F64) return factor_impl<double>(h, P, &oc, static_cast<double *>(Av), lda, jpvt, tau, T, S, work);
  return factor_impl<float>(h, P, &oc, static_cast<float *>(Av), lda, jpvt, tau, T, S, work);
}

// ---------------------------------------------------------------------------
// Q, P, truncation and the backward pass

// FP32 storage in the products below: the FP32 operands are widened into FP64
// copies at the front of the workspace, the FP64 sequence runs on them and the
// results are rounded back (FP32 storage, FP64 arithmetic).
static size_t shadow_bytes(rqrcp_dtype_t dt, size_t doubles) {
  return dt == RQRCP_F32 ? ((doubles * 8 + 255) / 256) * 256 : 0;
}

static size_t apply_q_work_f64(int64_t m, int64_t k, int64_t b, int64_t ncol) {
  if (m < 1 || k < 1 || b < 1 || ncol < 0) return 0;
  size_t gp = 0;
  for (int64_t r0 = 0; r0 < k; r0 += b) {
    const int64_t bi = std::min(b, k - r0), mi = m - r0;
    gp = std::max(gp, gemm_part_doubles(bi, ncol, mi));
    gp = std::max(gp, gemm_part_doubles(bi, ncol, bi));
    gp = std::max(gp, gemm_part_doubles(mi, ncol, bi));
  }
  Bump w;
  w.take((size_t)m * b * 8);
  w.take((size_t)b * ncol * 8);
  w.take((size_t)b * ncol * 8);
  w.take(gp * 8);
  return w.off + 256;
}

size_t rqrcp_diag_offset(int64_t n, int64_t k, int64_t b) {
  if (n < 1 || k < 1 || b < 1) return 0;
  const int64_t nb = cdiv(k, b);
  size_t vs_total = 0;
  for (int64_t i = 0; i < nb; ++i) vs_total += (size_t)(n - i * b) * b;
  return vs_total + (size_t)nb * b + (size_t)nb * b * b;
}

size_t rqrcp_apply_q_work_bytes(rqrcp_dtype_t dt, int64_t m, int64_t k, int64_t b, int64_t ncol) {
  const size_t base = apply_q_work_f64(m, k, b, ncol);
  if (base == 0) return 0;
  return shadow_bytes(dt, (size_t)m * k) + shadow_bytes(dt, (size_t)m * ncol) + base;
}

// The U'_i of a diagonalised factorization (Section 6.2) act on the rows of
// block i only, which the reflectors of later blocks do not touch, so
// Q = H_0 U~_0 H_1 U~_1 ... = (H_0 H_1 ...) (U~_0 U~_1 ...): Q C applies every
// U'_i to its rows first, Q^T C applies every U'_i^T last.
static rqrcp_status_t apply_q_impl(rqrcp_handle_t h, int trans, int64_t m, int64_t k, int64_t b, const double *VR,
                                   int64_t ldvr, const double *T, const double *UV, int64_t ncol, double *C,
                                   int64_t ldc, void *work) {
  hipStream_t s = h->stream;
  Bump w;
  double *Vb = at<double>(work, w.take((size_t)m * b * 8));
  double *W1 = at<double>(work, w.take((size_t)b * ncol * 8));
  double *W2 = at<double>(work, w.take((size_t)b * ncol * 8));
  size_t gp = 0;
  for (int64_t r0 = 0; r0 < k; r0 += b) {
    const int64_t bi = std::min(b, k - r0), mi = m - r0;
    gp = std::max(gp, gemm_part_doubles(bi, ncol, mi));
    gp = std::max(gp, gemm_part_doubles(bi, ncol, bi));
    gp = std::max(gp, gemm_part_doubles(mi, ncol, bi));
  }
  double *part = at<double>(work, w.take(gp * 8));
  const int64_t nb = cdiv(k, b);
  auto apply_u = [&]() -> rqrcp_status_t {
    for (int64_t i = 0; i < nb; ++i) {
      const int64_t r0 = i * b, bi = std::min(b, k - r0);
      const double *Ui = UV + (size_t)i * 2 * b * b;
      GemmF64 gu{trans ? true : false, false, bi, ncol, bi, Ui, b, C + r0, ldc, W1, bi, 1.0, 0.0};
      CHK(launch_gemm_f64(s, gu, part), trans ? "U'^T C" : "U' C");
      CHK(launch_copy2d(s, W1, bi, C + r0, ldc, bi, ncol), "rows of the block");
    }
    return RQRCP_OK;
  };
  if (UV && !trans) {
    rqrcp_status_t st = apply_u();
    if (st != RQRCP_OK) return st;
  }
  for (int64_t t = 0; t < nb; ++t) {
    const int64_t i = trans ? t : nb - 1 - t;
    const int64_t r0 = i * b, bi = std::min(b, k - r0), mi = m - r0;
    const double *Ti = T + (size_t)i * b * b;
    CHK(launch_extract_v(s, VR + r0 + r0 * ldvr, ldvr, mi, bi, Vb, mi), "extract V");
    double *Cs = C + r0;
    GemmF64 g1{true, false, bi, ncol, mi, Vb, mi, Cs, ldc, W1, bi, 1.0, 0.0};
    CHK(launch_gemm_f64(s, g1, part), "V^T C");
    // Q_i^T C = C - V T^T V^T C ; Q_i C = C - V T V^T C
    GemmF64 g2{trans ? true : false, false, bi, ncol, bi, Ti, b, W1, bi, W2, bi, 1.0, 0.0};
    CHK(launch_gemm_f64(s, g2, part), "T W");
    GemmF64 g3{false, false, mi, ncol, bi, Vb, mi, W2, bi, Cs, ldc, -1.0, 1.0};
    CHK(launch_gemm_f64(s, g3, part), "C -= V (T W)");
  }
  if (UV && trans) return apply_u();
  return RQRCP_OK;
}

rqrcp_status_t rqrcp_apply_q(rqrcp_handle_t h, rqrcp_dtype_t dt, int trans, int64_t m, int64_t k, int64_t b,
                             const void *VR, int64_t ldvr, const double *T, const double *UV, int64_t ncol,
                             void *C, int64_t ldc, void *work, size_t work_bytes) {
  if (!h) return fail(nullptr, RQRCP_ERR_ARG, "h is NULL");
  if (dt != RQRCP_F64 && dt != RQRCP_F32) return fail(h, RQRCP_ERR_ARG, "dt: unknown storage type");
  if (trans != 0 && trans != 1) return fail(h, RQRCP_ERR_ARG, "trans must be 0 or 1");
  if (m < 1 || k < 1 || k > m || b < 1) return fail(h, RQRCP_ERR_ARG, "need 1 <= k <= m and b >= 1");
  if (!VR || !T || !C) return fail(h, RQRCP_ERR_ARG, "VR, T and C must not be NULL");
  if (ldvr < m || ldc < m) return fail(h, RQRCP_ERR_ARG, "ldvr and ldc must be >= m");
  if (ncol < 0) return fail(h, RQRCP_ERR_ARG, "ncol must be >= 0");
  if (ncol == 0) return RQRCP_OK;
  if (!work || work_bytes < rqrcp_apply_q_work_bytes(dt, m, k, b, ncol))
    return fail(h, RQRCP_ERR_WORKSPACE, "work missing or smaller than rqrcp_apply_q_work_bytes");
  if (dt == RQRCP_F64)
    return apply_q_impl(h, trans, m, k, b, static_cast<const double *>(VR), ldvr, T, UV, ncol,
                        static_cast<double *>(C), ldc, work);
  hipStream_t s = h->stream;
  Bump w;
  double *V64 = at<double>(work, w.take(shadow_bytes(dt, (size_t)m * k)));
  double *C64 = at<double>(work, w.take(shadow_bytes(dt, (size_t)m * ncol)));
  CHK(launch_copy_f32_f64(s, static_cast<const float *>(VR), ldvr, V64, m, m, k), "V to FP64");
  CHK(launch_copy_f32_f64(s, static_cast<const float *>(C), ldc, C64, m, m, ncol), "C to FP64");
  rqrcp_status_t st = apply_q_impl(h, trans, m, k, b, V64, m, T, UV, ncol, C64, m, at<void>(work, w.off));
  if (st != RQRCP_OK) return st;
  CHK(launch_copy_f64_f32(s, C64, m, static_cast<float *>(C), ldc, m, ncol), "C to FP32");
  return RQRCP_OK;
}

static size_t apply_p_work_f64(int64_t nrow, int64_t n, int64_t k, int64_t b) {
  if (nrow < 0 || n < 1 || b < 1) return 0;
  size_t gp = 0;
  for (int64_t r0 = 0; r0 < k; r0 += b) {
    const int64_t bi = std::min(b, k - r0), ni = n - r0;
    gp = std::max(gp, gemm_part_doubles(nrow, bi, ni));
    gp = std::max(gp, gemm_part_doubles(nrow, bi, bi));
    gp = std::max(gp, gemm_part_doubles(nrow, ni, bi));
  }
  Bump w;
  w.take((size_t)nrow * n * 8);
  w.take((size_t)nrow * b * 8);
  w.take((size_t)nrow * b * 8);
  w.take(gp * 8);
  return w.off + 256;
}

size_t rqrcp_apply_p_work_bytes(rqrcp_dtype_t dt, int64_t nrow, int64_t n, int64_t k, int64_t b) {
  const size_t base = apply_p_work_f64(nrow, n, k, b);
  if (base == 0) return 0;
  return shadow_bytes(dt, (size_t)nrow * n) + base;
}

// The V'_i of a diagonalised factorization act on the columns of block i
// only, which the S_j of later blocks do not touch, so
// P = S_0 V~_0 S_1 V~_1 ... = (S_0 S_1 ...) (V~_0 V~_1 ...): C P applies
// every V'_i to its columns last, C P^T applies every V'_i^T first.
static rqrcp_status_t apply_p_impl(rqrcp_handle_t h, int trans, int64_t nrow, int64_t n, int64_t k, int64_t b,
                                   const int32_t *jpvt, const double *S, int diag, double *C, int64_t ldc,
                                   void *work) {
  hipStream_t s = h->stream;
  Bump w;
  double *tmpc = at<double>(work, w.take((size_t)nrow * n * 8));
  double *Z1 = at<double>(work, w.take((size_t)nrow * b * 8));
  double *Z2 = at<double>(work, w.take((size_t)nrow * b * 8));
  size_t gp = 0;
  for (int64_t r0 = 0; r0 < k; r0 += b) {
    const int64_t bi = std::min(b, k - r0), ni = n - r0;
    gp = std::max(gp, gemm_part_doubles(nrow, bi, ni));
    gp = std::max(gp, gemm_part_doubles(nrow, bi, bi));
    gp = std::max(gp, gemm_part_doubles(nrow, ni, bi));
  }
  double *part = at<double>(work, w.take(gp * 8));
  if (!S) {
    CHK(launch_copy2d(s, C, ldc, tmpc, nrow, nrow, n), "copy C");
    if (!trans) CHK(launch_gather_cols(s, tmpc, nrow, nrow, n, jpvt, n, C, ldc), "C P");
    else CHK(launch_scatter_cols(s, tmpc, nrow, nrow, jpvt, n, C, ldc, n, false), "C P^T");
    return RQRCP_OK;
  }
  const int64_t nb = cdiv(k, b);
  std::vector<size_t> vs_off(nb);
  size_t vs_total = 0;
  for (int64_t i = 0; i < nb; ++i) { vs_off[i] = vs_total; vs_total += (size_t)(n - i * b) * b; }
  const double *TS = S + vs_total + nb * b;
  const double *UV = diag ? TS + (size_t)nb * b * b : nullptr;
  auto apply_v = [&]() -> rqrcp_status_t {
    for (int64_t i = 0; i < nb; ++i) {
      const int64_t r0 = i * b, bi = std::min(b, k - r0);
      const double *Vi = UV + (size_t)i * 2 * b * b + (size_t)b * b;
      GemmF64 gv{false, trans ? true : false, nrow, bi, bi, C + r0 * ldc, ldc, Vi, b, Z1, nrow, 1.0, 0.0};
      CHK(launch_gemm_f64(s, gv, part), trans ? "C V'^T" : "C V'");
      CHK(launch_copy2d(s, Z1, nrow, C + r0 * ldc, ldc, nrow, bi), "columns of the block");
    }
    return RQRCP_OK;
  };
  if (UV && trans) {
    rqrcp_status_t st = apply_v();
    if (st != RQRCP_OK) return st;
  }
  for (int64_t t = 0; t < nb; ++t) {
    const int64_t i = trans ? nb - 1 - t : t;
    const int64_t r0 = i * b, bi = std::min(b, k - r0), ni = n - r0;
    const double *VS = S + vs_off[i];
    const double *TSi = TS + (size_t)i * b * b;
    double *Cc = C + r0 * ldc;
    GemmF64 g1{false, false, nrow, bi, ni, Cc, ldc, VS, ni, Z1, nrow, 1.0, 0.0};
    CHK(launch_gemm_f64(s, g1, part), "C VS");
    GemmF64 g2{false, trans ? true : false, nrow, bi, bi, Z1, nrow, TSi, b, Z2, nrow, 1.0, 0.0};
    CHK(launch_gemm_f64(s, g2, part), "(C VS) TS");
    GemmF64 g3{false, true, nrow, ni, bi, Z2, nrow, VS, ni, Cc, ldc, -1.0, 1.0};
    CHK(launch_gemm_f64(s, g3, part), "C -= (..) VS^T");
  }
  if (UV && !trans) return apply_v();
  return RQRCP_OK;
}

rqrcp_status_t rqrcp_apply_p(rqrcp_handle_t h, rqrcp_dtype_t dt, int trans, int64_t nrow, int64_t n, int64_t k,
                             int64_t b, const int32_t *jpvt, const double *S, int diagonalized, void *C, int64_t ldc,
                             void *work, size_t work_bytes) {
  if (!h) return fail(nullptr, RQRCP_ERR_ARG, "h is NULL");
  if (dt != RQRCP_F64 && dt != RQRCP_F32) return fail(h, RQRCP_ERR_ARG, "dt: unknown storage type");
  if (trans != 0 && trans != 1) return fail(h, RQRCP_ERR_ARG, "trans must be 0 or 1");
  if (nrow < 0 || n < 1 || b < 1 || k < 1 || k > n) return fail(h, RQRCP_ERR_ARG, "need nrow >= 0, 1 <= k <= n, b >= 1");
  if (!C || (!S && !jpvt)) return fail(h, RQRCP_ERR_ARG, "C and one of jpvt / S must be given");
  if (diagonalized != 0 && diagonalized != 1) return fail(h, RQRCP_ERR_ARG, "diagonalized must be 0 or 1");
  if (diagonalized && !S) return fail(h, RQRCP_ERR_ARG, "diagonalized needs S (orthonormal pivoting)");
  if (ldc < std::max<int64_t>(1, nrow)) return fail(h, RQRCP_ERR_ARG, "ldc must be >= nrow");
  if (nrow == 0) return RQRCP_OK;
  if (!work || work_bytes < rqrcp_apply_p_work_bytes(dt, nrow, n, k, b))
    return fail(h, RQRCP_ERR_WORKSPACE, "work missing or smaller than rqrcp_apply_p_work_bytes");
  if (dt == RQRCP_F64)
    return apply_p_impl(h, trans, nrow, n, k, b, jpvt, S, diagonalized, static_cast<double *>(C), ldc, work);
  hipStream_t s = h->stream;
  Bump w;
  double *C64 = at<double>(work, w.take(shadow_bytes(dt, (size_t)nrow * n)));
  CHK(launch_copy_f32_f64(s, static_cast<const float *>(C), ldc, C64, nrow, nrow, n), "C to FP64");
  rqrcp_status_t st = apply_p_impl(h, trans, nrow, n, k, b, jpvt, S, diagonalized, C64, nrow, at<void>(work, w.off));
  if (st != RQRCP_OK) return st;
  CHK(launch_copy_f64_f32(s, C64, nrow, static_cast<float *>(C), ldc, nrow, n), "C to FP32");
  return RQRCP_OK;
}

// Q(:, 0:k) = Q applied to the first k columns of the identity, from a
// factorization with kf >= k reflector columns.  Reflector j acts on rows
// >= j, where those columns are zero once j >= k, so only the first k
// reflectors matter; a diagonalised block's U'_i spreads columns r0..k-1 of
// the block holding column k - 1 over all its rows, so there that block's
// reflectors are all needed (blocks past it still act on zero rows only).
static int64_t qk_columns(int64_t k, int64_t kf, int64_t b, bool diag) {
  return diag ? std::min(kf, cdiv(k, b) * b) : k;
}
static size_t lowrank_work_f64(int64_t m, int64_t n, int64_t k, int64_t b) {
  if (m < 1 || n < 1 || k < 1 || b < 1) return 0;
  Bump w;
  w.take((size_t)m * k * 8);                               // Q_k
  w.take((size_t)k * n * 8);                               // R_k P^T
  w.take(std::max(apply_q_work_f64(m, qk_columns(k, n, b, true), b, k), apply_p_work_f64(k, n, n, b)));
  w.take(gemm_part_doubles(m, n, k) * 8);
  return w.off + 256;
}

// FP32 storage: the reflector columns and the rows of R_k widened to FP64,
// Q_k and R_k P^* formed in FP64 as above, then rounded to FP32 for the
// m x n x k product on FP32 matrix cores, which writes A_k directly.
static size_t lowrank_work_f32(int64_t m, int64_t n, int64_t k, int64_t b) {
  if (m < 1 || n < 1 || k < 1 || b < 1) return 0;
  const int64_t kq = qk_columns(k, n, b, true);
  Bump w;
  w.take((size_t)m * kq * 8);                              // F(:, 0:kq) in FP64
  w.take((size_t)k * n * 8);                               // F(0:k, :) in FP64
  w.take((size_t)m * k * 4);                               // Q_k in FP32
  w.take((size_t)k * n * 4);                               // R_k P^* in FP32
  w.take(gemm_part_floats(m, n, k) * 4);
  w.take(lowrank_work_f64(m, n, k, b));
  return w.off + 256;
}

size_t rqrcp_lowrank_work_bytes(rqrcp_dtype_t dt, int64_t m, int64_t n, int64_t k, int64_t b) {
  return dt == RQRCP_F32 ? lowrank_work_f32(m, n, k, b) : lowrank_work_f64(m, n, k, b);
}

static rqrcp_status_t form_qk(rqrcp_handle_t h, int64_t m, int64_t k, int64_t kf, int64_t b, const double *VR,
                              int64_t ldvr, const double *T, const double *UV, double *Qk, void *work) {
  CHK(launch_set_identity(h->stream, Qk, m, m, k), "identity");
  return apply_q_impl(h, 0, m, qk_columns(k, kf, b, UV != nullptr), b, VR, ldvr, T, UV, k, Qk, m, work);
}

// Q_k (m x k) and R_k P^* (k x n) in FP64 from a factorization whose
// reflectors (first columns) are read at Fv, ld ldv, and whose rows 0:k of R
// at Fr, ld ldr; A_k = Q_k (R_k P^*) follows.
static rqrcp_status_t lowrank_factors(rqrcp_handle_t h, int64_t m, int64_t n, int64_t k, int64_t kf, int64_t b,
                                      const double *Fv, int64_t ldv, const double *Fr, int64_t ldr,
                                      const int32_t *jpvt, const double *T, const double *S, int diag, double *Qk,
                                      double *RP, void *sub) {
  // U'_i, V'_i of a diagonalised factorization: after the V_S blocks, tau_S
  // and the T_S blocks in S
  const double *UV = diag ? S + rqrcp_diag_offset(n, kf, b) : nullptr;
  CHK(launch_extract_r(h->stream, Fr, ldr, k, n, RP, k), "extract R_k");
  rqrcp_status_t st = apply_p_impl(h, 1, k, n, kf, b, jpvt, S, diag, RP, k, sub);
  if (st != RQRCP_OK) return st;
  return form_qk(h, m, k, kf, b, Fv, ldv, T, UV, Qk, sub);
}

static rqrcp_status_t lowrank_impl(rqrcp_handle_t h, int64_t m, int64_t n, int64_t k, int64_t kf, int64_t b,
                                   const double *F, int64_t ldvr, const int32_t *jpvt, const double *T,
                                   const double *S, int diag, double *Ak, int64_t ldak, void *work) {
  Bump w;
  double *Qk = at<double>(work, w.take((size_t)m * k * 8));
  double *RP = at<double>(work, w.take((size_t)k * n * 8));
  void *sub = at<void>(work, w.take(std::max(apply_q_work_f64(m, qk_columns(k, n, b, true), b, k),
                                             apply_p_work_f64(k, n, n, b))));
  double *part = at<double>(work, w.take(gemm_part_doubles(m, n, k) * 8));
  rqrcp_status_t st = lowrank_factors(h, m, n, k, kf, b, F, ldvr, F, ldvr, jpvt, T, S, diag, Qk, RP, sub);
  if (st != RQRCP_OK) return st;
  GemmF64 g{false, false, m, n, k, Qk, m, RP, k, Ak, ldak, 1.0, 0.0};
  CHK(launch_gemm_f64(h->stream, g, part), "Q_k (R_k P^*)");
  return RQRCP_OK;
}

static rqrcp_status_t lowrank_f32(rqrcp_handle_t h, int64_t m, int64_t n, int64_t k, int64_t kf, int64_t b,
                                  const float *F, int64_t ldvr, const int32_t *jpvt, const double *T,
                                  const double *S, int diag, float *Ak, int64_t ldak, void *work) {
  hipStream_t s = h->stream;
  const int64_t kq = qk_columns(k, kf, b, diag != 0);
  Bump w;
  double *Fv = at<double>(work, w.take((size_t)m * qk_columns(k, n, b, true) * 8));
  double *Fr = at<double>(work, w.take((size_t)k * n * 8));
  float *Qk32 = at<float>(work, w.take((size_t)m * k * 4));
  float *RP32 = at<float>(work, w.take((size_t)k * n * 4));
  float *part32 = at<float>(work, w.take(gemm_part_floats(m, n, k) * 4));
  void *rest = at<void>(work, w.off);
  Bump w2;
  double *Qk = at<double>(rest, w2.take((size_t)m * k * 8));
  double *RP = at<double>(rest, w2.take((size_t)k * n * 8));
  void *sub = at<void>(rest, w2.take(std::max(apply_q_work_f64(m, qk_columns(k, n, b, true), b, k),
                                              apply_p_work_f64(k, n, n, b))));
  CHK(launch_copy_f32_f64(s, F, ldvr, Fv, m, m, kq), "reflector columns to FP64");
  CHK(launch_copy_f32_f64(s, F, ldvr, Fr, k, k, n), "rows of R_k to FP64");
  rqrcp_status_t st = lowrank_factors(h, m, n, k, kf, b, Fv, m, Fr, k, jpvt, T, S, diag, Qk, RP, sub);
  if (st != RQRCP_OK) return st;
  CHK(launch_copy_f64_f32(s, Qk, m, Qk32, m, m, k), "Q_k to FP32");
  CHK(launch_copy_f64_f32(s, RP, k, RP32, k, k, n), "R_k P^* to FP32");
  GemmF32 g{false, false, m, n, k, Qk32, m, RP32, k, Ak, ldak, 1.f, 0.f};
  CHK(launch_gemm<float>(s, g, part32), "Q_k (R_k P^*) in FP32");
  return RQRCP_OK;
}

rqrcp_status_t rqrcp_lowrank(rqrcp_handle_t h, rqrcp_dtype_t dt, int64_t m, int64_t n, int64_t k, int64_t kf,
                             int64_t b, const void *VR, int64_t ldvr, const int32_t *jpvt, const double *T,
                             const double *S, int diagonalized, void *Ak, int64_t ldak, void *work,
                             size_t work_bytes) {
  if (!h) return fail(nullptr, RQRCP_ERR_ARG, "h is NULL");
  if (dt != RQRCP_F64 && dt != RQRCP_F32) return fail(h, RQRCP_ERR_ARG, "dt: unknown storage type");
  if (m < n || n < 1 || k < 1 || k > n || b < 1) return fail(h, RQRCP_ERR_ARG, "need m >= n >= k >= 1, b >= 1");
  if (kf < k || kf > n) return fail(h, RQRCP_ERR_ARG, "kf (rank of the factorization) must satisfy k <= kf <= n");
  if (!VR || !T || !Ak || (!S && !jpvt)) return fail(h, RQRCP_ERR_ARG, "VR, T, Ak and jpvt (or S) are required");
  if (diagonalized != 0 && diagonalized != 1) return fail(h, RQRCP_ERR_ARG, "diagonalized must be 0 or 1");
  if (diagonalized && !S) return fail(h, RQRCP_ERR_ARG, "diagonalized needs S (orthonormal pivoting)");
  if (ldvr < m || ldak < m) return fail(h, RQRCP_ERR_ARG, "ldvr and ldak must be >= m");
  if (!work || work_bytes < rqrcp_lowrank_work_bytes(dt, m, n, k, b))
    return fail(h, RQRCP_ERR_WORKSPACE, "work missing or smaller than rqrcp_lowrank_work_bytes");
  if (dt == RQRCP_F64)
    return lowrank_impl(h, m, n, k, kf, b, static_cast<const double *>(VR), ldvr, jpvt, T, S, diagonalized,
                        static_cast<double *>(Ak), ldak, work);
  return lowrank_f32(h, m, n, k, kf, b, static_cast<const float *>(VR), ldvr, jpvt, T, S, diagonalized,
                     static_cast<float *>(Ak), ldak, work);
}

static size_t backward_work_f64(int64_t m, int64_t n, int64_t k, int64_t b) {
  if (m < 1 || n < 1 || k < 1 || b < 1) return 0;
  Bump w;
  w.take((size_t)m * k * 8);   // Q_k
  w.take((size_t)k * n * 8);   // R_k
  w.take((size_t)n * k * 8);   // P R_k^T, then Gbar^T Q_k
  w.take((size_t)m * k * 8);   // M
  w.take((size_t)k * k * 8);   // Q_k^T M
  w.take((size_t)k * k * 8);   // R_11^{-1}
  w.take((size_t)m * k * 8);   // Z
  w.take((size_t)k * n * 8);   // Q_k^T Gbar
  w.take(apply_q_work_f64(m, k, b, k));
  size_t gp = 0;
  gp = std::max(gp, gemm_part_doubles(m, k, n));
  gp = std::max(gp, gemm_part_doubles(n, k, m));
  gp = std::max(gp, gemm_part_doubles(k, k, m));
  gp = std::max(gp, gemm_part_doubles(m, k, k));
  gp = std::max(gp, gemm_part_doubles(k, n, m));
  gp = std::max(gp, gemm_part_doubles(m, n, k));
  w.take(gp * 8);
  return w.off + 256;
}

// FP32 storage: Q_k (FP64 from the widened reflector columns), R_k and
// R_11^{-1} in FP64, rounded to FP32; the products with the m x n operands
// (A, dA_k, dA) run on FP32 matrix cores straight on the caller's FP32 data.
static size_t backward_work_f32(int64_t m, int64_t n, int64_t k, int64_t b) {
  if (m < 1 || n < 1 || k < 1 || b < 1) return 0;
  Bump w;
  w.take((size_t)m * k * 8);   // F(:, 0:k) in FP64
  w.take((size_t)k * n * 8);   // F(0:k, :) in FP64
  w.take((size_t)m * k * 8);   // Q_k
  w.take((size_t)k * n * 8);   // R_k
  w.take((size_t)n * k * 8);   // P R_k^T
  w.take((size_t)k * k * 8);   // R_11^{-1}
  w.take(apply_q_work_f64(m, k, b, k));
  w.take((size_t)m * k * 4);   // Q_k in FP32
  w.take((size_t)n * k * 4);   // P R_k^T, then dA_k^T Q_k, in FP32
  w.take((size_t)m * k * 4);   // M
  w.take((size_t)k * k * 4);   // Q_k^T M
  w.take((size_t)k * k * 4);   // R_11^{-1} in FP32
  w.take((size_t)m * k * 4);   // Z
  w.take((size_t)k * n * 4);   // Q_k^T dA_k
  size_t gp = 0;
  gp = std::max(gp, gemm_part_floats(m, k, n));
  gp = std::max(gp, gemm_part_floats(n, k, m));
  gp = std::max(gp, gemm_part_floats(k, k, m));
  gp = std::max(gp, gemm_part_floats(m, k, k));
  gp = std::max(gp, gemm_part_floats(k, n, m));
  gp = std::max(gp, gemm_part_floats(m, n, k));
  w.take(gp * 4);
  return w.off + 256;
}

size_t rqrcp_lowrank_backward_work_bytes(rqrcp_dtype_t dt, int64_t m, int64_t n, int64_t k, int64_t b) {
  return dt == RQRCP_F32 ? backward_work_f32(m, n, k, b) : backward_work_f64(m, n, k, b);
}

static rqrcp_status_t backward_impl(rqrcp_handle_t h, int64_t m, int64_t n, int64_t k, int64_t b, const double *A,
                                    int64_t lda, const double *F, int64_t ldvr, const int32_t *jpvt, const double *T,
                                    const double *Gb, int64_t ldg, double *dA, int64_t ldda, void *work) {
  hipStream_t s = h->stream;
  Bump w;
  double *Qk = at<double>(work, w.take((size_t)m * k * 8));
  double *Rk = at<double>(work, w.take((size_t)k * n * 8));
  double *NK = at<double>(work, w.take((size_t)n * k * 8));
  double *M = at<double>(work, w.take((size_t)m * k * 8));
  double *KK = at<double>(work, w.take((size_t)k * k * 8));
  double *Ri = at<double>(work, w.take((size_t)k * k * 8));
  double *Z = at<double>(work, w.take((size_t)m * k * 8));
  double *KN = at<double>(work, w.take((size_t)k * n * 8));
  void *sub = at<void>(work, w.take(apply_q_work_f64(m, k, b, k)));
  size_t gp = 0;
  gp = std::max(gp, gemm_part_doubles(m, k, n));
  gp = std::max(gp, gemm_part_doubles(n, k, m));
  gp = std::max(gp, gemm_part_doubles(k, k, m));
  gp = std::max(gp, gemm_part_doubles(m, k, k));
  gp = std::max(gp, gemm_part_doubles(k, n, m));
  gp = std::max(gp, gemm_part_doubles(m, n, k));
  double *part = at<double>(work, w.take(gp * 8));

  rqrcp_status_t st = form_qk(h, m, k, k, b, F, ldvr, T, nullptr, Qk, sub);
  if (st != RQRCP_OK) return st;
  CHK(launch_extract_r(s, F, ldvr, k, n, Rk, k), "extract R_k");
  // P R_k^T (n x k): row jpvt[j] is column j of R_k
  CHK(launch_scatter_rows_t(s, Rk, k, k, jpvt, n, NK, n), "P R_k^T");
  // M = Gbar (P R_k^T)
  GemmF64 g1{false, false, m, k, n, Gb, ldg, NK, n, M, m, 1.0, 0.0};
  CHK(launch_gemm_f64(s, g1, part), "Gbar P R_k^T");
  // M += A (Gbar^T Q_k)
  GemmF64 g2{true, false, n, k, m, Gb, ldg, Qk, m, NK, n, 1.0, 0.0};
  CHK(launch_gemm_f64(s, g2, part), "Gbar^T Q_k");
  GemmF64 g3{false, false, m, k, n, A, lda, NK, n, M, m, 1.0, 1.0};
  CHK(launch_gemm_f64(s, g3, part), "A (Gbar^T Q_k)");
  // M <- (I - Q_k Q_k^T) M
  GemmF64 g4{true, false, k, k, m, Qk, m, M, m, KK, k, 1.0, 0.0};
  CHK(launch_gemm_f64(s, g4, part), "Q_k^T M");
  GemmF64 g5{false, false, m, k, k, Qk, m, KK, k, M, m, -1.0, 1.0};
  CHK(launch_gemm_f64(s, g5, part), "M -= Q_k (Q_k^T M)");
  // Z = M R_11^{-T}
  CHK(launch_tri_inv_upper(s, Rk, k, k, Ri, k), "R_11^{-1}");
  GemmF64 g6{false, true, m, k, k, M, m, Ri, k, Z, m, 1.0, 0.0};
  CHK(launch_gemm_f64(s, g6, part), "M R_11^{-T}");
  // dA = Q_k (Q_k^T Gbar), then dA(:, jpvt[0:k]) += Z
  GemmF64 g7{true, false, k, n, m, Qk, m, Gb, ldg, KN, k, 1.0, 0.0};
  CHK(launch_gemm_f64(s, g7, part), "Q_k^T Gbar");
  GemmF64 g8{false, false, m, n, k, Qk, m, KN, k, dA, ldda, 1.0, 0.0};
  CHK(launch_gemm_f64(s, g8, part), "Q_k (Q_k^T Gbar)");
  CHK(launch_scatter_cols(s, Z, m, m, jpvt, k, dA, ldda, n, true), "scatter Z");
  return RQRCP_OK;
}

// The same sequence as backward_impl with FP32 operands (see backward_work_f32).
static rqrcp_status_t backward_f32(rqrcp_handle_t h, int64_t m, int64_t n, int64_t k, int64_t b, const float *A,
                                   int64_t lda, const float *F, int64_t ldvr, const int32_t *jpvt, const double *T,
                                   const float *Gb, int64_t ldg, float *dA, int64_t ldda, void *work) {
  hipStream_t s = h->stream;
  Bump w;
  double *Fv = at<double>(work, w.take((size_t)m * k * 8));
  double *Fr = at<double>(work, w.take((size_t)k * n * 8));
  double *Qk = at<double>(work, w.take((size_t)m * k * 8));
  double *Rk = at<double>(work, w.take((size_t)k * n * 8));
  double *NK = at<double>(work, w.take((size_t)n * k * 8));
  double *Ri = at<double>(work, w.take((size_t)k * k * 8));
  void *sub = at<void>(work, w.take(apply_q_work_f64(m, k, b, k)));
  float *Qk32 = at<float>(work, w.take((size_t)m * k * 4));
  float *NK32 = at<float>(work, w.take((size_t)n * k * 4));
  float *M = at<float>(work, w.take((size_t)m * k * 4));
  float *KK = at<float>(work, w.take((size_t)k * k * 4));
  float *Ri32 = at<float>(work, w.take((size_t)k * k * 4));
  float *Z = at<float>(work, w.take((size_t)m * k * 4));
  float *KN = at<float>(work, w.take((size_t)k * n * 4));
  size_t gp = 0;
  gp = std::max(gp, gemm_part_floats(m, k, n));
  gp = std::max(gp, gemm_part_floats(n, k, m));
  gp = std::max(gp, gemm_part_floats(k, k, m));
  gp = std::max(gp, gemm_part_floats(m, k, k));
  gp = std::max(gp, gemm_part_floats(k, n, m));
  gp = std::max(gp, gemm_part_floats(m, n, k));
  float *part = at<float>(work, w.take(gp * 4));

  CHK(launch_copy_f32_f64(s, F, ldvr, Fv, m, m, k), "reflector columns to FP64");
  CHK(launch_copy_f32_f64(s, F, ldvr, Fr, k, k, n), "rows of R_k to FP64");
  rqrcp_status_t st = form_qk(h, m, k, k, b, Fv, m, T, nullptr, Qk, sub);
  if (st != RQRCP_OK) return st;
  CHK(launch_copy_f64_f32(s, Qk, m, Qk32, m, m, k), "Q_k to FP32");
  CHK(launch_extract_r(s, Fr, k, k, n, Rk, k), "extract R_k");
  CHK(launch_scatter_rows_t(s, Rk, k, k, jpvt, n, NK, n), "P R_k^T");
  CHK(launch_copy_f64_f32(s, NK, n, NK32, n, n, k), "P R_k^T to FP32");
  GemmF32 g1{false, false, m, k, n, Gb, ldg, NK32, n, M, m, 1.f, 0.f};
  CHK(launch_gemm<float>(s, g1, part), "Gbar P R_k^T");
  GemmF32 g2{true, false, n, k, m, Gb, ldg, Qk32, m, NK32, n, 1.f, 0.f};
  CHK(launch_gemm<float>(s, g2, part), "Gbar^T Q_k");
  GemmF32 g3{false, false, m, k, n, A, lda, NK32, n, M, m, 1.f, 1.f};
  CHK(launch_gemm<float>(s, g3, part), "A (Gbar^T Q_k)");
  GemmF32 g4{true, false, k, k, m, Qk32, m, M, m, KK, k, 1.f, 0.f};
  CHK(launch_gemm<float>(s, g4, part), "Q_k^T M");
  GemmF32 g5{false, false, m, k, k, Qk32, m, KK, k, M, m, -1.f, 1.f};
  CHK(launch_gemm<float>(s, g5, part), "M -= Q_k (Q_k^T M)");
  CHK(launch_tri_inv_upper(s, Rk, k, k, Ri, k), "R_11^{-1}");
  CHK(launch_copy_f64_f32(s, Ri, k, Ri32, k, k, k), "R_11^{-1} to FP32");
  GemmF32 g6{false, true, m, k, k, M, m, Ri32, k, Z, m, 1.f, 0.f};
  CHK(launch_gemm<float>(s, g6, part), "M R_11^{-T}");
  GemmF32 g7{true, false, k, n, m, Qk32, m, Gb, ldg, KN, k, 1.f, 0.f};
  CHK(launch_gemm<float>(s, g7, part), "Q_k^T Gbar");
  GemmF32 g8{false, false, m, n, k, Qk32, m, KN, k, dA, ldda, 1.f, 0.f};
  CHK(launch_gemm<float>(s, g8, part), "Q_k (Q_k^T Gbar)");
  CHK(launch_scatter_cols_f32(s, Z, m, m, jpvt, k, dA, ldda, n, true), "scatter Z");
  return RQRCP_OK;
}

rqrcp_status_t rqrcp_lowrank_backward(rqrcp_handle_t h, rqrcp_dtype_t dt, int64_t m, int64_t n, int64_t k, int64_t b,
                                      const void *Av, int64_t lda, const void *VR, int64_t ldvr, const int32_t *jpvt,
                                      const double *T, const void *dAkv, int64_t ldg, void *dAv, int64_t ldda,
                                      void *work, size_t work_bytes) {
  if (!h) return fail(nullptr, RQRCP_ERR_ARG, "h is NULL");
  if (dt != RQRCP_F64 && dt != RQRCP_F32) return fail(h, RQRCP_ERR_ARG, "dt: unknown storage type");
  if (m < n || n < 1 || k < 1 || k > n || b < 1) return fail(h, RQRCP_ERR_ARG, "need m >= n >= k >= 1, b >= 1");
  if (k > 8192) return fail(h, RQRCP_ERR_UNSUPPORTED, "k: at most 8192 in the backward");
  if (!Av || !VR || !jpvt || !T || !dAkv || !dAv) return fail(h, RQRCP_ERR_ARG, "a required pointer is NULL");
  if (lda < m || ldvr < m || ldg < m || ldda < m) return fail(h, RQRCP_ERR_ARG, "leading dimensions must be >= m");
  if (!work || work_bytes < rqrcp_lowrank_backward_work_bytes(dt, m, n, k, b))
    return fail(h, RQRCP_ERR_WORKSPACE, "work missing or smaller than rqrcp_lowrank_backward_work_bytes");
  if (dt == RQRCP_F64)
    return backward_impl(h, m, n, k, b, static_cast<const double *>(Av), lda, static_cast<const double *>(VR), ldvr,
                         jpvt, T, static_cast<const double *>(dAkv), ldg, static_cast<double *>(dAv), ldda, work);
  return backward_f32(h, m, n, k, b, static_cast<const float *>(Av), lda, static_cast<const float *>(VR), ldvr,
                      jpvt, T, static_cast<const float *>(dAkv), ldg, static_cast<float *>(dAv), ldda, work);
}

}  // extern "C"
