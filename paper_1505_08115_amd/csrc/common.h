// Internal declarations shared by the HIP sources of librqrcp (gfx950 only).
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "rqrcp.h"

namespace rq {

// ---------------------------------------------------------------------------
// Device helpers

// Cross-lane moves on the DPP network (operands of the next VALU op, no LDS
// round trip): lane i reads lane i^1 or i^2 of its quad, lane 7-i of its
// aligned group of 8 (half-row mirror) or lane 15-i of its row of 16 (mirror).
constexpr int kDppXor1 = 0xB1, kDppXor2 = 0x4E, kDppHalfMirror = 0x141, kDppMirror = 0x140;
template <int CTRL>
__device__ __forceinline__ int dpp_mov(int x) {
  return __builtin_amdgcn_mov_dpp(x, CTRL, 0xF, 0xF, false);
}
template <int CTRL>
__device__ __forceinline__ double dpp_mov(double x) {
  return __hiloint2double(dpp_mov<CTRL>(__double2hiint(x)), dpp_mov<CTRL>(__double2loint(x)));
}
// Lanes i and i ^ 16 (the two rows of a 32-lane half), or i and i ^ 32 (the
// two halves of the wave), both get the pair (lo, hi): lo from the lower lane,
// hi from the upper one (v_permlane16_swap / v_permlane32_swap, plain VALU
// register swaps).
template <int SPAN>
__device__ __forceinline__ void lane_pair(int x, int &lo, int &hi) {
  static_assert(SPAN == 16 || SPAN == 32, "span");
  if constexpr (SPAN == 16) {
    const auto r = __builtin_amdgcn_permlane16_swap((unsigned)x, (unsigned)x, false, false);
    lo = (int)r[0];
    hi = (int)r[1];
  } else {
    const auto r = __builtin_amdgcn_permlane32_swap((unsigned)x, (unsigned)x, false, false);
    lo = (int)r[0];
    hi = (int)r[1];
  }
}
template <int SPAN>
__device__ __forceinline__ void lane_pair(double x, double &lo, double &hi) {
  int lh, hh, ll, hl;
  lane_pair<SPAN>(__double2hiint(x), lh, hh);
  lane_pair<SPAN>(__double2loint(x), ll, hl);
  lo = __hiloint2double(lh, ll);
  hi = __hiloint2double(hh, hl);
}

// Sum over each aligned group of 8 lanes; all 8 lanes get the same value
// (pairs are added in the same order on both sides).
__device__ __forceinline__ double group8_sum(double v) {
  v += dpp_mov<kDppXor1>(v);
  v += dpp_mov<kDppXor2>(v);
  v += dpp_mov<kDppHalfMirror>(v);
  return v;
}

// Sum over the wave; every lane gets the same value.  Call with all 64 lanes
// active.
__device__ __forceinline__ double wave_sum(double v) {
  v = group8_sum(v);
  v += dpp_mov<kDppMirror>(v);
  double lo, hi;
  lane_pair<16>(v, lo, hi);
  v = lo + hi;
  lane_pair<32>(v, lo, hi);
  return lo + hi;
}

// Lane 0's value in every lane (wave-uniform).
__device__ __forceinline__ double lane0(double x) {
  return __hiloint2double(__builtin_amdgcn_readfirstlane(__double2hiint(x)),
                          __builtin_amdgcn_readfirstlane(__double2loint(x)));
}
__device__ __forceinline__ int lane0(int x) { return __builtin_amdgcn_readfirstlane(x); }

// Agent-scope relaxed atomic load and store: served at the device's coherence
// point, not by one XCD's L2, so that data exchanged between workgroups needs
// no L2 write-back or invalidation around a barrier (exchange mode below).
__device__ __forceinline__ double ld_agent(const double *p) {
  return __longlong_as_double(
      (long long)__hip_atomic_load((const unsigned long long *)p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
}
__device__ __forceinline__ void st_agent(double *p, double v) {
  __hip_atomic_store((unsigned long long *)p, (unsigned long long)__double_as_longlong(v), __ATOMIC_RELAXED,
                     __HIP_MEMORY_SCOPE_AGENT);
}

// This wave's earlier loads and stores have completed (vmcnt counts both on
// gfx9); the fence keeps the compiler from moving memory operations across.
__device__ __forceinline__ void wave_mem_drain() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
  __builtin_amdgcn_s_waitcnt(0x0F70);   // vmcnt(0)
}

// Grid-wide barrier for cooperatively launched kernels, run by wave 0 of
// each workgroup.  Workgroups arrive on one of 8 group counters (grouped by
// blockIdx % 8, i.e. by the XCD that the round-robin dispatcher puts them
// on, so that arrivals on one counter are few); every waiter polls all 8
// counters at once (lanes 0..7, one load each) until each has reached its
// group's size times the barrier count.  One level: no workgroup relays
// arrivals to another counter (measured 0.5-0.6 us per barrier faster than
// a two-level tree with a published generation).  Counters only grow, so no
// reset is needed between barriers; the host zeroes the state once before
// the launch.  All counters lie in words 64 .. 64 + 32*7 of the state.
//
// Memory ordering, two modes.  Release/acquire (exchange = false): the
// arrival is a release read-modify-write by lane 0, which writes the L2 of
// the workgroup's XCD back, and a waiter that has seen every counter reach
// its target acquires once (each counter's arrivals form one release
// sequence), which invalidates its L2; data may then be written and read
// with plain accesses.  Exchange (exchange = true): every datum that another
// workgroup reads is written with st_agent and read with ld_agent; the
// arrival is a relaxed atomic add issued only after the arriving wave's
// stores have completed, and a waiter issues its later loads only after its
// poll has returned every counter's final value (the loop exit depends on
// them).  No L2 write-back or invalidation happens, so the L2s keep each
// workgroup's own data; in the pivoted QR of the sketch this measured 1.2 us
// less per barrier than release/acquire, with the same pivots.
// In both modes only wave 0's stores are covered (other waves hand their data
// to wave 0 through LDS) unless all_waves is set, in which case every wave
// waits for its own stores to complete before the workgroup barrier.
//
// Every wait is bounded in wall-clock time (limit_ticks of the constant-rate
// device clock): past it the waiter raises the abort word and every later wait
// returns at once, so that a broken launch drains within about one limit.
struct GridBarrier {
  unsigned *state;       // group counter g at [64 + 32 g], g < 8
  int *abort_flag;       // shared abort word (zeroed by the host)
  uint64_t limit_ticks;  // longest wait, in ticks of the constant-rate device clock
};

// Called by all 64 lanes of wave 0 (uniformly); target = number of barriers
// passed so far + 1.
__device__ __forceinline__ bool grid_arrive_wait(const GridBarrier &gb, unsigned target, bool exchange) {
  const unsigned nwg = gridDim.x;
  const unsigned ngroups = nwg < 8 ? nwg : 8;
  const int lane = threadIdx.x & 63;
  unsigned *mine = gb.state + 64 + 32 * (blockIdx.x % ngroups);
  if (exchange) {
    wave_mem_drain();
    if (lane == 0) __hip_atomic_fetch_add(mine, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  } else if (lane == 0) {
    __hip_atomic_fetch_add(mine, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
  }
  const unsigned g = lane < (int)ngroups ? (unsigned)lane : 0u;
  const unsigned want = ((nwg - g + ngroups - 1) / ngroups) * target;   // group g's size times target
  const uint64_t t0 = (uint64_t)wall_clock64();
  // Two polls in flight: the next load is issued before the previous one is
  // tested, so a completed barrier is seen about half a round trip sooner than
  // with one load at a time (measured 0.16 us less per barrier; a four-deep
  // form compiled to a wait for three loads at the loop head).  The abort word
  // and the clock are looked at every 32nd poll only (they matter only when
  // something has already gone wrong).
  const unsigned *pc = gb.state + 64 + 32 * g;
  unsigned va = __hip_atomic_load(pc, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT), vb;
  for (unsigned it = 1;; ++it) {
    // unrolled twice so that each load lands in the register just tested
    // (a register copy would make the loop wait for the younger load)
    vb = __hip_atomic_load(pc, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (__all(lane >= (int)ngroups || va >= want)) break;
    va = __hip_atomic_load(pc, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (__all(lane >= (int)ngroups || vb >= want)) break;
    if ((it & 15) == 0) {
      if (__hip_atomic_load(gb.abort_flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) return false;
      if ((uint64_t)wall_clock64() - t0 > gb.limit_ticks) {
        if (lane == 0) __hip_atomic_store(gb.abort_flag, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        return false;
      }
    }
  }
  if (exchange)
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");   // keeps later loads below the poll
  else
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
  return true;
}

// Workgroup-wide form: call from every thread.
__device__ __forceinline__ bool grid_sync(const GridBarrier &gb, unsigned &gen, bool all_waves = false,
                                          bool exchange = false) {
  __shared__ int s_ok;
  if (all_waves) wave_mem_drain();
  __syncthreads();
  if (threadIdx.x < 64) {
    const bool ok = grid_arrive_wait(gb, gen + 1, exchange);
    if (threadIdx.x == 0) s_ok = ok ? 1 : 0;
  }
  __syncthreads();
  gen += 1;
  return s_ok != 0;
}

// ---------------------------------------------------------------------------
// Host-side launchers (implemented in the .hip files)

// Gaussian sketch: G(r, g - row0) for r < nsample, g in [row0, row0 + nrows).
hipError_t launch_sketch(hipStream_t s, uint64_t seed, int64_t block, int64_t nsample, int64_t row0,
                         int64_t nrows, double *G, int64_t ldg, int max_wg = 0);

// C = alpha op(A) op(B) + beta C on the matrix cores (FP64 or FP32), column-major.  When the
// problem is split along K the partial products go to `partial` (at least
// splits * M * N doubles) and a fixed-order reduction produces C.
template <typename T>
struct Gemm {
  bool ta, tb;
  int64_t M, N, K;
  const T *A; int64_t lda;
  const T *B; int64_t ldb;
  T *C; int64_t ldc;
  T alpha, beta;
  bool trailing = false;   // the factorization's trailing update (a separate kernel name in profiles)
  int max_wg = 0;          // > 0: at most this many workgroups (each loops over tiles), so that a
                           // product on a side stream leaves CUs free for persistent kernels
  bool wprod = false;      // the factorization's W = V^T C (a separate kernel name in profiles)
  // n2 > 0 (W with S = V^T V fused in front): the first n2 columns of op(B)
  // come from B2 (ld ldb2), column n2 + j from column j of B
  const T *B2 = nullptr;
  int64_t ldb2 = 0, n2 = 0;
};
typedef Gemm<double> GemmF64;
typedef Gemm<float> GemmF32;
template <typename T> int gemm_splits(const Gemm<T> &g);   // split count the launcher will use
template <typename T> hipError_t launch_gemm(hipStream_t s, const Gemm<T> &g, T *partial);
inline int gemm_f64_splits(const GemmF64 &g) { return gemm_splits<double>(g); }
inline hipError_t launch_gemm_f64(hipStream_t s, const GemmF64 &g, double *partial) {
  return launch_gemm<double>(s, g, partial);
}

// Zero-fill of n 32-bit words (safe inside graph capture, unlike memset nodes).
hipError_t launch_zero_u32(hipStream_t s, void *p, size_t nwords);

// Launch of a kernel that meets at grid barriers (all its workgroups must be
// resident at once).  A cooperative launch guarantees that but runs on a
// hardware queue of its own, and each change of queue between dependent
// kernels of one stream measured about 12 us (four per block of the
// factorization).  So the kernel is launched as an ordinary kernel on the
// stream's own queue when its grid fits in half the device at the kernel's
// occupancy: the products that run beside it on other streams are capped at
// the other half (their workgroup cap), so every workgroup finds room.
// Larger grids take the cooperative launch.
hipError_t launch_persistent(const void *func, unsigned nwg, unsigned threads, void **args, size_t lds,
                             hipStream_t s);

// Cooperative pivoted QR of a small k x ncols matrix, first nsteps steps
// (classical pivot rule; only the pivot decisions are produced).
struct QrcpSmall {
  double *Y; int64_t ldy; int k; int ncols; int nsteps;
  int32_t *piv;          // [nsteps] swap partner of position j
  int32_t *dest;         // [ncols] final position of each column
  int32_t *moved;        // [2*nsteps] columns whose position changed
  int32_t *moved_cnt;    // [1]
  double *rec;           // exchange records, qrcp_small_rec_doubles()
  double *cand;          // exchange columns, qrcp_small_cand_doubles()
  unsigned *bar;         // barrier state (zeroed), kBarrierWords words
  int *abort_flag;       // zeroed
  int32_t *info;         // may be NULL
  int block_index;
  uint64_t limit_ticks;  // barrier wait limit
};
constexpr int kBarrierWords = 64 + 32 * 8;
int qrcp_small_config(int k, int ncols, int *cpw);   // returns workgroups (0 = unsupported)
size_t qrcp_small_rec_doubles(int nwg);
size_t qrcp_small_cand_doubles(int nwg, int k);
hipError_t launch_qrcp_small(hipStream_t s, const QrcpSmall &q);

// Move the columns listed by a QrcpSmall run: column r0 + c goes to r0 +
// dest[c], for all m rows of A and for jpvt.
template <typename T>
hipError_t launch_apply_moves(hipStream_t s, T *A, int64_t lda, int64_t m, int64_t r0,
                              const int32_t *moved, const int32_t *moved_cnt, const int32_t *dest,
                              int max_moved, T *tmp, int32_t *jpvt, int32_t *jtmp);

// Cooperative unpivoted Householder QR of an mi x nb panel (FP64).
struct PanelQR {
  double *P; int64_t ldp; int64_t mi; int nb;
  double *tau;            // [nb]
  double *V; int64_t ldv; // explicit unit-lower V (mi x nb)
  double *VT; int64_t ldvt;   // NULL, or V^T (nb x mi) written as well
  double *part;           // partial sums, panel_part_doubles()
  double *red;            // reduced sums, nb * kPanelW doubles
  unsigned *bar;
  int *abort_flag;
  int32_t *info;
  int block_index;
  uint64_t limit_ticks;  // barrier wait limit
};
constexpr int kPanelW = 32;
int panel_config(int64_t mi, int nb, int *rpw);   // workgroups (0 = unsupported)
size_t panel_part_doubles(int nwg, int nb);
hipError_t launch_panel_qr(hipStream_t s, const PanelQR &p);

// T of the compact WY form from tau and the Gram matrix S = V^T V (nb x nb,
// ld nb; column j is read for rows <= j).
hipError_t launch_wy_t(hipStream_t s, int nb, const double *tau, const double *S, double *T, int64_t ldt);

// SVD of the nb x nb upper triangle of F (ld ldf, nb <= svd_small_max_block()):
// R22 = U' D V'^T with D decreasing, written as U (nb x nb, ld ldu), V (ld ldv)
// and D on the diagonal of F, whose strict upper triangle is cleared.  Above
// 64 columns a cooperative launch works on the columns in `work`
// (svd_small_work_doubles) with a zeroed barrier slot (its words from
// kBarrierWords on count rotations per sweep).
struct SvdSmall {
  double *F; int64_t ldf; int nb;
  double *U; int64_t ldu;
  double *V; int64_t ldv;
  double *work;          // svd_small_work_doubles(nb) doubles
  unsigned *bar;         // zeroed barrier slot (nb > 64)
  int *abort_flag;
  int32_t *info;         // may be NULL; [2] is set if a grid-wide wait gave up
  uint64_t limit_ticks;
};
int svd_small_max_block();
size_t svd_small_work_doubles(int nb);
hipError_t launch_svd_small(hipStream_t s, const SvdSmall &p);

}  // namespace rq
