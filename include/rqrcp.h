/*
 * rqrcp.h -- blocked randomized QR with column pivoting on one AMD Instinct
 * MI355X (gfx950).
 *
 * The library computes the factorization A P = Q R of an m x n matrix A with
 * m >= n, where Q is orthonormal, R is upper triangular and P is either a
 * permutation or a product of Householder reflectors (P.G. Martinsson,
 * "Blocked rank-revealing QR factorizations: How randomized sampling can be
 * used to avoid single-vector pivoting", 2015: eq. (1.1), Section 4 and the
 * algorithm blockQR of Fig. 3).  Pivots are chosen b at a time: a Gaussian
 * sketch Y = G X of the trailing matrix X is drawn, a pivoted QR of the small
 * Y picks b columns (Section 4.1, eqs. defY and Yrows; oversampling as in
 * Section 4.3), the columns are moved into place, the m' x b panel is
 * factored by unpivoted Householder QR in compact WY form (V, T) and the
 * trailing matrix is updated as C <- (I - V T V^T)^T C (Section 5.1).
 *
 * Conventions for every entry point:
 *   - Matrices are column-major with a leading dimension ld >= rows; indices
 *     are 0-based.  Pointers to matrix data are DEVICE pointers unless a
 *     comment says "host".
 *   - The caller owns every buffer (inputs, outputs and the workspace).  The
 *     library never allocates device memory on these paths and never frees
 *     caller memory.
 *   - Argument, size and workspace errors are reported synchronously, before
 *     anything is launched and without side effects; rqrcp_last_error()
 *     names the offending argument.  RQRCP_OK means the work is ENQUEUED on
 *     the handle's stream; the caller synchronises that stream before reading
 *     results.  Launch failures return RQRCP_ERR_HIP.
 *   - One handle per stream; calls on one handle must not run concurrently
 *     from several host threads.
 *
 * Storage of a factorization (the layout of LAPACK's geqrf/geqp3):
 *   - A is overwritten by R on and above the diagonal and by the Householder
 *     vectors below it (the unit diagonal of each vector is implicit).  The
 *     paper: "The matrix R overwrites A" (captions of Figs. 2 and 3).
 *   - Block i (0-based) covers columns [i*b, i*b + b_i), b_i = min(b, k - i*b),
 *     k = rank (n for a full factorization).  Q = Q_0 Q_1 ... with
 *     Q_i = diag(I_{i*b}, I - V_i T_i V_i^T).
 *   - tau[j], j < k: the scalar of reflector j (H_j = I - tau_j v_j v_j^T).
 *   - T: ceil(k/b) blocks of b*b doubles, block i at T + i*b*b, column-major
 *     with leading dimension b; the leading b_i x b_i part is upper
 *     triangular, the rest is zero.
 *   - jpvt[j] (int32): (A P)(:, j) = A(:, jpvt[j]) for the permutation form;
 *     the identity for the orthonormal form.
 *   - S (orthonormal form only): P = P_0 P_1 ... with
 *     P_i = diag(I_{i*b}, I - VS_i TS_i VS_i^T).  Layout, with nb = ceil(k/b)
 *     and n_i = n - i*b:  VS blocks first (block i is n_i x b, leading
 *     dimension n_i, unit lower trapezoidal, starting at element
 *     b * sum_{t<i} n_t), then tauS (nb*b doubles), then TS (nb*b*b doubles,
 *     like T).  rqrcp_factor_sizes reports the total element count.
 */
#ifndef RQRCP_H
#define RQRCP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct rqrcp_ctx *rqrcp_handle_t;

typedef enum {
  RQRCP_OK = 0,
  RQRCP_ERR_ARG = 1,         /* invalid argument (see rqrcp_last_error)       */
  RQRCP_ERR_WORKSPACE = 2,   /* workspace missing or smaller than required    */
  RQRCP_ERR_HIP = 3,         /* a HIP runtime call or launch failed           */
  RQRCP_ERR_UNSUPPORTED = 4, /* valid but outside what the library supports  */
  RQRCP_ERR_NONFINITE = 5,   /* info[0]: a non-finite norm (rqrcp_check)      */
  RQRCP_ERR_TIMEOUT = 6      /* info[2]: a grid-wide wait gave up; results    */
                             /* invalid (rqrcp_check)                         */
} rqrcp_status_t;

typedef enum { RQRCP_F64 = 0, RQRCP_F32 = 1 } rqrcp_dtype_t;               /* storage type of A   */
typedef enum { RQRCP_PIVOT_PERM = 0, RQRCP_PIVOT_ORTHO = 1 } rqrcp_pivot_t; /* Sec. 4.1 vs 4.2     */
typedef enum { RQRCP_PREC_PLAIN = 0, RQRCP_PREC_MIXED = 1 } rqrcp_prec_t;   /* MIXED: F32 only     */
typedef enum { RQRCP_TAIL_CLASSICAL = 0, RQRCP_TAIL_SAMPLED = 1 } rqrcp_tail_t;

typedef struct {
  int64_t block;        /* b >= 1                                                      */
  int64_t oversample;   /* p >= 0; the sketch has b + p rows (Section 4.3)             */
  int64_t rank;         /* k in [1, n] stops after the block reaching column k; 0 = n  */
  int32_t pivot;        /* rqrcp_pivot_t                                               */
  int32_t precision;    /* rqrcp_prec_t                                                */
  int32_t tail;         /* rqrcp_tail_t: the last block of a full factorization by     */
                        /* classical QRCP (Fig. 3) or by a sketch like the others      */
  int32_t fixed_pivots; /* 1: jpvt is an INPUT (a permutation of 0..n-1); no sketch is */
                        /* drawn, the columns jpvt[0:k] are factored in that order      */
  uint64_t seed;        /* key of the counter-based Gaussian generator                 */
  const double *G;      /* NULL, or device sketches for every sampled block: block i   */
                        /* is (b+p) x (m - i*b), column-major, ld = b+p, blocks stored */
                        /* one after the other                                         */
  int32_t *info;        /* NULL, or device int32[4], zeroed by the library and set:    */
                        /* [0] = 1 if a non-finite norm was met, [1] = first block     */
                        /* where that happened (+1), [2] = 1 if a grid-wide wait gave  */
                        /* up (results invalid), [3] reserved.  With NULL the library  */
                        /* writes the same flags to a word of its own in the handle,   */
                        /* which rqrcp_check reads                                     */
  int32_t power;        /* q in [0, 8]: steps of the power iteration of Section 6.3 on */
                        /* every sketched block, Y_i = G_i X_i (X_i^T X_i)^q; q > 0    */
                        /* moves the trailing update to the caller's stream (the steps */
                        /* read the updated block) and takes (b+p) m more doubles of   */
                        /* workspace; with F32 storage the steps run on                */
                        /* FP32 matrix cores (the sketch scaled by a power of two      */
                        /* before each step); ignored with fixed_pivots                */
  int32_t panel_pivot;  /* 1: Fig. 3's in-block pivot P-hat, a QR with column pivoting */
                        /* of every sketched panel (its order read off a QRCP of the   */
                        /* panel's R', the Remark of Section 2); the columns above the */
                        /* panel and jpvt follow.  The permutation form only (else     */
                        /* RQRCP_ERR_UNSUPPORTED); ignored with fixed_pivots.          */
                        /* 0 (default): P-hat = I                                      */
  int32_t diagonalize;  /* 1: diagonalised blocks of Section 6.2 (with ORTHO pivoting   */
                        /* and power: blockRRQR, Fig. 5): each block's b_i x b_i       */
                        /* triangle R22 = U' D V'^T becomes D (decreasing, >= 0), its  */
                        /* rows right of it get U'^T and its columns above it V'.      */
                        /* Q = prod_i diag(I, (I - V_i T_i V_i^T) diag(U'_i, I)) and   */
                        /* P = prod_i diag(I, S_i) diag(I, V'_i, I); U'_i, V'_i (b x b, */
                        /* ld b) follow the T_S blocks in S (see rqrcp_factor).  ORTHO */
                        /* and b <= 256 only (else RQRCP_ERR_UNSUPPORTED); with F32    */
                        /* storage the SVD and its products run in FP64 on widened     */
                        /* copies of the block's triangle, rows and columns            */
                        /* rqrcp_apply_q (its UV argument), rqrcp_apply_p and          */
                        /* rqrcp_lowrank (their diagonalized flag) apply U' and V';    */
                        /* rqrcp_lowrank_backward covers the permutation form only     */
} rqrcp_opts_t;

/* Default options: b = 128, p = 10, full rank, permutation, plain, classical
 * tail, seed 0, no G hook, no info word.  Host only, cannot fail. */
void rqrcp_default_opts(rqrcp_opts_t *o);

/* Create a handle bound to a HIP stream (hipStream_t passed as void*, NULL =
 * the default stream) on the current device.  Queries the device (it must be
 * gfx950) and prepares the cooperative kernels.  The handle owns two streams
 * of default priority, a few events and 16 bytes of device memory (its info
 * word), all released by rqrcp_destroy; this is the only device memory the
 * library allocates (besides the array of rqrcp_factor_noalloc, which the
 * code object holds on each device).  Errors: RQRCP_ERR_ARG (h == NULL),
 * RQRCP_ERR_UNSUPPORTED (not a gfx950 device), RQRCP_ERR_HIP. */
rqrcp_status_t rqrcp_create(rqrcp_handle_t *h, void *hip_stream);
rqrcp_status_t rqrcp_set_stream(rqrcp_handle_t h, void *hip_stream);
rqrcp_status_t rqrcp_destroy(rqrcp_handle_t h);
const char *rqrcp_status_string(rqrcp_status_t s);
/* Status of the most recent rqrcp_factor call on h that was given no
 * opts.info: synchronises the handle's stream and reads the handle's own info
 * word (layout as opts.info) into info_host (host int32[4], may be NULL).
 * Returns RQRCP_ERR_TIMEOUT if a grid-wide wait gave up (the results of that
 * call are invalid), else RQRCP_ERR_NONFINITE if a non-finite norm was met,
 * else RQRCP_OK; RQRCP_ERR_ARG for a NULL handle, RQRCP_ERR_HIP if the copy
 * fails.  Calls that were given opts.info report only there. */
rqrcp_status_t rqrcp_check(rqrcp_handle_t h, int32_t *info_host);
/* Message of the last failing call on h (or of the last failing call without
 * a handle when h == NULL).  Owned by the library, valid until the next call. */
const char *rqrcp_last_error(rqrcp_handle_t h);

/* Sizes for rqrcp_factor (host only, no GPU needed).  Any output pointer may
 * be NULL.  tau_elems: doubles of tau; T_elems: doubles of T; S_elems:
 * doubles of S (0 for the permutation form); work_bytes: workspace bytes.
 * Errors: RQRCP_ERR_ARG for invalid sizes or options. */
rqrcp_status_t rqrcp_factor_sizes(rqrcp_dtype_t dt, int64_t m, int64_t n, const rqrcp_opts_t *o,
                                  size_t *tau_elems, size_t *T_elems, size_t *S_elems,
                                  size_t *work_bytes);

/* Blocked randomized QR, A P = Q R (Fig. 3, Sections 4.1-4.3, 5.1-5.3).
 *   A    (in/out) m x n, ld lda >= m, of type dt: in A, out R + Householder
 *        vectors (see the header comment).  With rank k < n the rows k:m of
 *        columns k:n hold the updated trailing matrix R_22 of Section 6.1.
 *   jpvt (out, or in with fixed_pivots) int32[n].
 *   tau  (out) double[k];  T (out) double[ceil(k/b) * b * b].
 *   S    (out) ORTHO only, double[S_elems]; must be NULL for PERM.  Layout:
 *        the reflectors V_S of every block ((n - i b) x b, ld n - i b, one
 *        block after the other), then tau_S (nblocks x b), then T_S
 *        (nblocks blocks of b x b, ld b), then with diagonalize U'_i and
 *        V'_i for every block (b x b each, ld b, U'_0 V'_0 U'_1 V'_1 ...).
 *   work, work_bytes: device workspace of at least rqrcp_factor_sizes bytes,
 *        256-byte aligned; its contents on entry do not matter.
 * Precision: dt = F64 computes in FP64 throughout.  dt = F32 stores A in
 * FP32; the panel, tau, T and the pivoted QR of the sketch are FP64; the
 * sketch and trailing-update products use FP32 MFMA (PLAIN) or, for the
 * sketch, BF16 MFMA with FP32 accumulation (MIXED).
 * Errors: RQRCP_ERR_ARG (NULL pointers, m < n, n < 1, lda < m, b < 1, p < 0,
 * k > n, MIXED with F64, S given for PERM or missing for ORTHO),
 * RQRCP_ERR_WORKSPACE, RQRCP_ERR_UNSUPPORTED (sizes beyond the library's
 * limits, e.g. b + p > 512 or fixed_pivots with ORTHO), RQRCP_ERR_HIP. */
rqrcp_status_t rqrcp_factor(rqrcp_handle_t h, rqrcp_dtype_t dt, int64_t m, int64_t n,
                            void *A, int64_t lda, int32_t *jpvt, double *tau, double *T,
                            double *S, const rqrcp_opts_t *o, void *work, size_t work_bytes);

/* rqrcp_factor without a workspace argument, for callers that cannot
 * allocate device memory (code under HIP graph capture, allocation-free
 * serving loops, harnesses that forbid hipMalloc).  Arguments, results and
 * errors are those of rqrcp_factor; the workspace is instead a device array
 * of RQRCP_NOALLOC_WORK_BYTES that the library holds on every device it runs
 * on until the process ends (its address is taken once per device by
 * rqrcp_create).  The call allocates nothing.  Problems whose workspace
 * (rqrcp_factor_sizes) exceeds RQRCP_NOALLOC_WORK_BYTES are refused with
 * RQRCP_ERR_WORKSPACE before any launch; RQRCP_ERR_ARG if the current device
 * is not the handle's.  Every call on a device shares that device's array:
 * calls that overlap on one GPU (other handles or streams) race and give
 * wrong results; calls that follow each other in stream order are safe (the
 * array keeps the last call's contents, and each call writes every part it
 * reads and clears what must start at zero). */
#define RQRCP_NOALLOC_WORK_BYTES (64u << 20)
rqrcp_status_t rqrcp_factor_noalloc(rqrcp_handle_t h, rqrcp_dtype_t dt, int64_t m, int64_t n,
                                    void *A, int64_t lda, int32_t *jpvt, double *tau, double *T,
                                    double *S, const rqrcp_opts_t *o);

/* Apply Q or Q^T from a stored factorization to C (m x ncol, ld ldc >= m):
 * trans = 0: C <- Q C;  trans = 1: C <- Q^T C.  Q = Q_0 Q_1 ... Q_{nb-1} with
 * Q_i = diag(I_{i*b}, I - V_i T_i V_i^T) (Fig. 3's accumulation of Q-tilde,
 * applied in WY form as Section 5.1 asks).  VR, ldvr: the factored A (only
 * the Householder vectors below the diagonal of its first k columns are
 * read); T as written by rqrcp_factor; k, b as used there.  UV: NULL, or for
 * a diagonalised factorization (Section 6.2) its U'/V' blocks in S (at
 * element rqrcp_diag_offset(n, k, b) of S): then every Q_i is followed by
 * diag(I_{i*b}, U'_i, I) and Q = (Q_0 ... Q_{nb-1}) diag(U'_0, U'_1, ...),
 * since U'_i acts on rows that later blocks leave alone.  C has the storage
 * type dt; with dt = F32 the operands are widened to FP64 in the workspace,
 * the products run in FP64 and C is rounded back to FP32.  work: at least
 * rqrcp_apply_q_work_bytes bytes.
 * Errors: RQRCP_ERR_ARG, RQRCP_ERR_WORKSPACE, RQRCP_ERR_HIP. */
size_t rqrcp_apply_q_work_bytes(rqrcp_dtype_t dt, int64_t m, int64_t k, int64_t b, int64_t ncol);
rqrcp_status_t rqrcp_apply_q(rqrcp_handle_t h, rqrcp_dtype_t dt, int trans, int64_t m, int64_t k,
                             int64_t b, const void *VR, int64_t ldvr, const double *T,
                             const double *UV, int64_t ncol, void *C, int64_t ldc, void *work,
                             size_t work_bytes);
/* Offset (in doubles) of the U'_0 V'_0 U'_1 V'_1 ... blocks inside S for a
 * diagonalised factorization of n columns, rank k, block b (host only). */
size_t rqrcp_diag_offset(int64_t n, int64_t k, int64_t b);

/* Apply P or P^T from the right to C (nrow x n, ld ldc >= nrow):
 * trans = 0: C <- C P;  trans = 1: C <- C P^T.  PERM (S == NULL): a column
 * permutation by jpvt ((C P)(:, j) = C(:, jpvt[j])).  ORTHO: the product of
 * the S blocks (k, b as in the factorization); diagonalized = 1 (a
 * diagonalised factorization, Section 6.2): each S_i is followed by
 * diag(I_{i*b}, V'_i, I), so P = (S_0 S_1 ...) diag(V'_0, V'_1, ...) with the
 * V'_i read from S.  C has the storage type dt (F32: computed in FP64 on a
 * widened copy).  work: at least rqrcp_apply_p_work_bytes bytes.
 * Errors: RQRCP_ERR_ARG (also diagonalized without S), RQRCP_ERR_WORKSPACE,
 * RQRCP_ERR_HIP. */
size_t rqrcp_apply_p_work_bytes(rqrcp_dtype_t dt, int64_t nrow, int64_t n, int64_t k, int64_t b);
rqrcp_status_t rqrcp_apply_p(rqrcp_handle_t h, rqrcp_dtype_t dt, int trans, int64_t nrow, int64_t n,
                             int64_t k, int64_t b, const int32_t *jpvt, const double *S,
                             int diagonalized, void *C, int64_t ldc, void *work, size_t work_bytes);

/* Truncated factorization A_k = Q(:, 0:k) R(0:k, :) P^* (Section 7's e_k
 * definition; Section 6.1 for its error ||R_22||).  Inputs as written by
 * rqrcp_factor with rank kf >= k (VR, ldvr, jpvt, T, S); kf fixes how many
 * blocks of T and S exist (P is the product of all kf/b S blocks);
 * diagonalized = 1 reads U' and V' from S as rqrcp_apply_q and
 * rqrcp_apply_p describe.  Ak (out)
 * m x n, ld ldak >= m, type dt (F32: Q_k and R_k P^* are formed in FP64 from
 * widened copies of the reflector columns and of rows 0:k, rounded to FP32,
 * and their m x n x k product runs on FP32 matrix cores).  work: at least
 * rqrcp_lowrank_work_bytes. */
size_t rqrcp_lowrank_work_bytes(rqrcp_dtype_t dt, int64_t m, int64_t n, int64_t k, int64_t b);
rqrcp_status_t rqrcp_lowrank(rqrcp_handle_t h, rqrcp_dtype_t dt, int64_t m, int64_t n, int64_t k,
                             int64_t kf, int64_t b, const void *VR, int64_t ldvr, const int32_t *jpvt,
                             const double *T, const double *S, int diagonalized, void *Ak, int64_t ldak,
                             void *work, size_t work_bytes);

/* Gradient of a loss L(A_k) through the truncated factorization with the
 * pivots held fixed (an addition to the paper).  With Q_k = Q(:, 0:k),
 * Pi = Q_k Q_k^T, R_k = R(0:k, :), R_11 = R(0:k, 0:k) and the upstream
 * gradient dAk = dL/dA_k:
 *   dA = Q_k (Q_k^T dAk) + scatter_{jpvt[0:k]}(Z),
 *   Z  = (I - Pi) [dAk P R_k^T + A dAk^T Q_k] R_11^{-T}.
 * Permutation form only.  A (in) the ORIGINAL input, ld lda.  VR, ldvr, jpvt,
 * T: a factorization of A with rank >= k (e.g. recomputed with fixed_pivots).
 * dAk (in) m x n, ld ldg; dA (out) m x n, ld ldda.  All of type dt (F32:
 * Q_k, R_k and R_11^{-1} in FP64 from widened copies of the reflector columns
 * and rows 0:k, rounded to FP32; the products with A, dAk and dA run on FP32
 * matrix cores on the caller's FP32 data).
 * k <= 8192 (RQRCP_ERR_UNSUPPORTED beyond).
 * work: at least rqrcp_lowrank_backward_work_bytes bytes. */
size_t rqrcp_lowrank_backward_work_bytes(rqrcp_dtype_t dt, int64_t m, int64_t n, int64_t k, int64_t b);
rqrcp_status_t rqrcp_lowrank_backward(rqrcp_handle_t h, rqrcp_dtype_t dt, int64_t m, int64_t n,
                                      int64_t k, int64_t b, const void *A, int64_t lda,
                                      const void *VR, int64_t ldvr, const int32_t *jpvt,
                                      const double *T, const void *dAk, int64_t ldg, void *dA,
                                      int64_t ldda, void *work, size_t work_bytes);

/* Draw the Gaussian sketch G_i of block `block` (Section 4.1's Omega,
 * transposed): G(r, g - row0) for r < nsample and g in [row0, row0 + nrows),
 * from Philox4x64-10 with counter (g, r, block, 0) and key (seed, 1), one
 * uniform per word as ((w >> 12) + 1/2) 2^-52 and Box-Muller on words 0 and 1.
 * G (out, device) nsample x nrows, ld ldg >= nsample, FP64. */
rqrcp_status_t rqrcp_sketch(rqrcp_handle_t h, uint64_t seed, int64_t block, int64_t nsample,
                            int64_t row0, int64_t nrows, double *G, int64_t ldg);

/* Per-kernel-class timing, a measurement aid.  When enabled, every launch of
 * the classes below is bracketed by a pair of HIP events on the handle's
 * stream (no host synchronisation is added).  After the caller has
 * synchronised the stream, rqrcp_timing_read returns, per class, the number
 * of bracketed launches, their summed duration (ms) and the algorithmic flop
 * and HBM byte counts of those launches, and clears the records of that
 * class.  Errors: RQRCP_ERR_ARG for a NULL handle or an unknown class,
 * RQRCP_ERR_HIP if an event query fails (e.g. the stream was not
 * synchronised). */
typedef enum {
  RQRCP_K_SKETCH = 0,      /* drawing G_i                                     */
  RQRCP_K_SAMPLE_GEMM = 1, /* Y_i = G_i X_i                                   */
  RQRCP_K_QRCP = 2,        /* pivoted QR of the sketch / of the last block    */
  RQRCP_K_MOVES = 3,       /* moving the pivot columns (all m rows)           */
  RQRCP_K_PANEL = 4,       /* unpivoted Householder QR of the panel           */
  RQRCP_K_TFACTOR = 5,     /* T of the compact WY form                        */
  RQRCP_K_VT_GEMM = 6,     /* T^T W (FP64), V T^T (FP32 storage)              */
  RQRCP_K_W_GEMM = 7,      /* W = V^T C                                       */
  RQRCP_K_UPDATE_GEMM = 8, /* C -= V (T^T W) (FP64), (V T^T) W (FP32)         */
  RQRCP_K_ORTHO = 9,       /* QR of the sketch and right-application of S_i   */
  RQRCP_K_OTHER = 10,      /* the diagonalised blocks (SVD and rotations)     */
  RQRCP_K_COUNT = 11
} rqrcp_kernel_class_t;
rqrcp_status_t rqrcp_timing_enable(rqrcp_handle_t h, int enable);
rqrcp_status_t rqrcp_timing_read(rqrcp_handle_t h, int kclass, int64_t *launches, double *ms, double *flops,
                                 double *bytes);
/* Restrict the timing to the classes whose bit is set in mask (bit k = class
 * k; the default, and any mask with all bits set, times every class), so that
 * a measurement can bracket one class without the events of the others.
 * Errors: RQRCP_ERR_ARG for a NULL handle. */
rqrcp_status_t rqrcp_timing_classes(rqrcp_handle_t h, uint32_t mask);

#ifdef __cplusplus
}
#endif

#endif /* RQRCP_H */
