"""Plain FP64 CPU oracle for blocked randomized QR with column pivoting.

TEST INFRASTRUCTURE ONLY.  Only tests, the smoke check and the benchmark's
CPU-baseline leg may import this module; the product path never does.

Written from P.G. Martinsson, "Blocked rank-revealing QR factorizations: How
randomized sampling can be used to avoid single-vector pivoting" (2015).
Every function follows the steps of the paper in its order, with numpy
matrix products as the only library primitive.  Nothing here is blocked,
fused or reordered beyond what the paper states.

Conventions (the readings of the paper this oracle takes):

* Householder reflector of a column a (Section 3.1): beta = -sign(a_1)|a|
  with sign(0) = +1; compact form H = I - tau v v^T with v_1 = 1,
  v = (a - beta e_1)/(a_1 - beta) and tau = (beta - a_1)/beta.  a = 0 gives
  H = I (tau = 0).  a_1 != 0 with a(2:) = 0 keeps the paper's formula
  (tau = 2, R_jj = -a_1).  A column of length 1 gets no reflector (tau = 0):
  the paper's loop runs n - 1 reflectors for a square matrix (Sections 3.2,
  3.3).
* Pivot rule (Section 3.3, Fig. 2): the largest 2-norm of the remaining
  columns over the remaining rows, recomputed exactly at every step; ties go
  to the lowest current position.  Pivoting swaps positions j and j'
  (sequential swaps), applied to every row of the matrix and to jpvt.
* Blocked loop (Section 4.1 eq. defY and eq. Yrows; Section 4.3; Fig. 3):
  block i (0-based) starts at r0 = i*b.  The sketch is Y_i = G_i X_i with
  X_i = A(r0:m, r0:n) and G_i = Omega_i^T of size (b+p) x (m-r0); only the
  first b_i = min(b, columns left) steps of the QR process on Y_i run.  The
  pivot matrix is applied to columns r0:n of all m rows.  The panel
  A(r0:m, r0:r0+b_i) is factored by unpivoted Householder QR (the in-block
  pivot P-hat of Fig. 3 is the identity; with panel_pivot it is the pivot
  of a classical QRCP of the panel), and the trailing matrix is updated
  with the compact WY form of the panel's reflectors (Section 5.1).
* n need not be a multiple of b: the last block takes what is left.  With a
  full factorization the last block is the "tail" of Fig. 3 and gets a
  classical QRCP; with a target rank k < n the loop stops after the block
  that reaches column k (no tail).
* Orthonormal pivoting (Section 4.2, eq. Ycols, first Remark of 4.2): an
  unpivoted QR of Y_i^T, first b_i steps, gives S_i = H_1...H_b; it is
  applied from the right to columns r0:n of all m rows.  The tail block of
  this variant is treated like every other block (sampled).
"""
import numpy as np

from . import philox

# ---------------------------------------------------------------------------
# Section 3.1: the Householder reflector


def householder(a):
    """Reflector H(a) = I - tau v v^T with v[0] = 1 and H a = beta e_1.

    Returns (v, tau, beta).  See the module header for the degenerate cases.
    """
    a = np.asarray(a, dtype=np.float64)
    v = np.zeros_like(a)
    v[0] = 1.0
    if a.shape[0] <= 1:
        return v, 0.0, float(a[0]) if a.shape[0] else 0.0
    norm = float(np.sqrt(np.dot(a, a)))
    if norm == 0.0:
        return v, 0.0, 0.0
    a1 = float(a[0])
    sign = 1.0 if a1 >= 0.0 else -1.0
    beta = -sign * norm
    v[1:] = a[1:] / (a1 - beta)
    tau = (beta - a1) / beta
    return v, tau, beta


def apply_reflector_left(v, tau, C):
    """C <- (I - tau v v^T) C, in place on a 2-D view."""
    if tau == 0.0:
        return
    w = v @ C
    C -= tau * np.outer(v, w)


# ---------------------------------------------------------------------------
# Section 3.2: QR without pivoting (each A_j overwrites A_{j-1})


def householder_qr(A, steps=None):
    """Unpivoted Householder QR of A (m x n) in place, `steps` reflectors.

    On return the upper triangle of A holds R and the strict lower part of
    column j holds v_j(1:) (v_j(0) = 1 is implicit).  Returns tau.
    """
    m, n = A.shape
    if steps is None:
        steps = min(m, n)
    tau = np.zeros(steps)
    for j in range(steps):
        v, t, beta = householder(A[j:, j])
        tau[j] = t
        apply_reflector_left(v, t, A[j:, j + 1:])
        A[j, j] = beta
        A[j + 1:, j] = v[1:]
    return tau


# ---------------------------------------------------------------------------
# Section 3.3, Fig. 2: classical Householder QR with column pivoting


def _column_norms(A, j):
    return np.sqrt(np.einsum("ij,ij->j", A[j:, j:], A[j:, j:]))


def qrcp(A, steps=None, record_margins=False, tops=None):
    """Classical QRCP (Fig. 2) of A in place, running `steps` pivot steps.

    Returns (piv, jpvt, tau, margins):
      piv[j]  : the position swapped with position j at step j (swap list),
      jpvt    : (A P)(:, j) = A_in(:, jpvt[j]),
      tau     : reflector scalars,
      margins : per step, (nu_1^2 - nu_2^2) / nu_1^2 for the top two
                remaining norms (inf when one candidate, 0 when nu_1 = 0).
    If `tops` is a list, the largest remaining norm nu_1 of every step is
    appended to it.
    """
    m, n = A.shape
    if steps is None:
        steps = min(m, n)
    piv = np.zeros(steps, dtype=np.int64)
    jpvt = np.arange(n)
    tau = np.zeros(steps)
    margins = np.zeros(steps)
    for j in range(steps):
        nu = _column_norms(A, j)
        jj = int(np.argmax(nu))          # first maximum = lowest position
        if tops is not None:
            tops.append(float(nu[jj]))
        if record_margins:
            top = nu[jj]
            rest = np.delete(nu, jj)
            if rest.size == 0:
                margins[j] = np.inf
            elif top == 0.0:
                margins[j] = 0.0
            else:
                margins[j] = (top * top - rest.max() ** 2) / (top * top)
        jp = j + jj
        piv[j] = jp
        if jp != j:
            A[:, [j, jp]] = A[:, [jp, j]]
            jpvt[[j, jp]] = jpvt[[jp, j]]
        v, t, beta = householder(A[j:, j])
        tau[j] = t
        apply_reflector_left(v, t, A[j:, j + 1:])
        A[j, j] = beta
        A[j + 1:, j] = v[1:]
    return piv, jpvt, tau, margins


# ---------------------------------------------------------------------------
# Section 5.1: the compact WY form of a product of reflectors


def wy_T(V, tau):
    """Upper-triangular T with H_1 H_2 ... H_k = I - V T V^T.

    V is m x k with unit diagonal and zeros above it.  Forward recurrence:
    T(j, j) = tau_j and T(0:j, j) = -tau_j T(0:j, 0:j) V(:, 0:j)^T v_j.
    """
    k = V.shape[1]
    T = np.zeros((k, k))
    for j in range(k):
        T[j, j] = tau[j]
        if j > 0:
            T[:j, j] = -tau[j] * (T[:j, :j] @ (V[:, :j].T @ V[:, j]))
    return T


def unit_lower(F, rows, cols):
    """Householder vectors of a factored block as an explicit matrix."""
    V = np.tril(F[:rows, :cols], -1)
    k = min(rows, cols)
    V[np.arange(k), np.arange(k)] = 1.0
    return V


# ---------------------------------------------------------------------------
# Sections 4 and 5: blocked randomized QR (Fig. 3)


def sketch(seed, block, nsample, row0, nrows):
    """G_i = Omega_i^T (Section 4.1), from the counter-based generator."""
    return philox.sketch_block(seed, block, nsample, row0, nrows)


def rqrcp(A, b, p, seed, pivot="perm", rank=0, tail="classical", G=None,
          sampler="gaussian", trace=False, power=0, panel_pivot=False, diagonalize=False):
    """Blocked randomized QR (Fig. 3) of a copy of A; returns a dict.

    pivot   : "perm" (Section 4.1) or "ortho" (Section 4.2)
    rank    : 0 for a full factorization, else stop after the block reaching k
    tail    : "classical" (Fig. 3, last block by QRCP) or "sampled" (perm)
    G       : optional list of per-block sketches G_i ((b+p) x (m-r0));
              None draws them from the counter-based generator
    sampler : "gaussian", or "identity" (Y_i := X_i; test reduction only)
    power   : q >= 0 steps of the power iteration of Section 6.3 on each
              sketched block: Y_i := G_i X_i (X_i^T X_i)^q
    panel_pivot : Fig. 3's in-block pivot P-hat (permutation form): the
              panel of every sketched block is factored by classical QRCP
              (Fig. 2) instead of unpivoted Householder QR, and its swaps
              reorder the columns above the panel and jpvt as well
    diagonalize : Section 6.2 (with pivot="ortho": blockRRQR, Fig. 5): the
              b_i x b_i triangle R22 of every panel is replaced by its
              singular values, R22 = U' D V'^T; U'^T rotates the block's
              rows to the right of it, V' its columns above it and P

    Output keys: F (R on and above the diagonal, Householder vectors below),
    tau, T (list of per-block T), jpvt, S (list of (V_S, tau_S, T_S) per block
    for ortho), piv (list of per-block swap lists), margins (list), xnorm
    (Frobenius norm of each block's trailing matrix X_i), ynorm (Frobenius
    norm of the matrix each pivoted QR ran on), tops (per block, the largest
    remaining norm at every pivot step), and, with trace=True, Y (list of
    per-block samples before factoring).
    """
    A = np.array(A, dtype=np.float64, copy=True)
    m, n = A.shape
    if m < n:
        raise ValueError("the method assumes m >= n")
    if diagonalize and pivot != "ortho":
        raise ValueError("the diagonalised blocks (Section 6.2) go with orthonormal pivoting")
    k = n if rank in (0, None) else int(rank)
    if not 1 <= k <= n:
        raise ValueError("rank out of range")
    jpvt = np.arange(n)
    tau = np.zeros(k)
    out = {"T": [], "S": [], "piv": [], "margins": [], "Y": [], "blocks": [], "xnorm": [], "ynorm": [],
           "tops": [], "pmargins": [], "ptops": [], "pnorm": [], "D": []}
    nblocks = -(-k // b)
    for i in range(nblocks):
        r0 = i * b
        bi = min(b, k - r0)
        mi, ni = m - r0, n - r0
        X = A[r0:, r0:]
        is_tail = (k == n) and (r0 + b >= n)
        out["blocks"].append((r0, bi))
        out["xnorm"].append(float(np.linalg.norm(X)))
        if is_tail and tail == "classical" and pivot == "perm":
            # last block of Fig. 3: classical QRCP of the remaining block
            Xc = X.copy()
            out["ynorm"].append(float(np.linalg.norm(Xc)))
            tp = []
            piv, jp, t, mg = qrcp(Xc, steps=bi, record_margins=True, tops=tp)
            out["tops"].append(np.array(tp))
            A[:r0, r0:] = A[:r0, r0:][:, jp]
            A[r0:, r0:] = Xc
            jpvt[r0:] = jpvt[r0:][jp]
            tau[r0:r0 + bi] = t
            out["piv"].append(piv)
            out["margins"].append(mg)
            out["T"].append(wy_T(unit_lower(A[r0:, r0:], mi, bi), t))
            continue
        # draw the sketch (Section 4.1; oversampled per Section 4.3)
        if sampler == "identity":
            Y = X.copy()
        else:
            Gi = G[i] if G is not None else sketch(seed, i, b + p, r0, mi)
            Y = Gi @ X
            # Section 6.3, in the row form of the sample: each step multiplies
            # by X_i^T X_i, as (Y X_i^T) X_i, with no re-orthonormalisation
            for _ in range(int(power)):
                Y = (Y @ X.T) @ X
        if trace:
            out["Y"].append(Y.copy())
        if pivot == "perm":
            # eq. Yrows: classical QRCP of Y, first b_i steps only
            out["ynorm"].append(float(np.linalg.norm(Y)))
            tp = []
            piv, jp, _, mg = qrcp(Y, steps=bi, record_margins=True, tops=tp)
            out["tops"].append(np.array(tp))
            for j in range(bi):                    # P-tilde on all m rows
                jj = int(piv[j])
                if jj != j:
                    A[:, [r0 + j, r0 + jj]] = A[:, [r0 + jj, r0 + j]]
                    jpvt[[r0 + j, r0 + jj]] = jpvt[[r0 + jj, r0 + j]]
            out["piv"].append(piv)
            out["margins"].append(mg)
        else:
            # eq. Ycols without pivoting (Remark), first b_i steps only
            Yt = Y.T.copy()
            ts = householder_qr(Yt, steps=bi)
            VS = unit_lower(Yt, ni, bi)
            TS = wy_T(VS, ts)
            # columns r0:n of all rows <- (...) S_i, S_i = I - V_S T_S V_S^T
            C = A[:, r0:]
            C -= ((C @ VS) @ TS) @ VS.T
            out["S"].append((VS, ts, TS))
        panel = A[r0:, r0:r0 + bi]
        if panel_pivot and pivot == "perm":
            # Fig. 3 with P-hat: QR with column pivoting of the panel; qrcp
            # swaps the panel's own rows in place, the rows above follow
            out["pnorm"].append(float(np.linalg.norm(panel)))
            tp = []
            ppiv, _, t, pmg = qrcp(panel, steps=bi, record_margins=True, tops=tp)
            for j in range(bi):
                jj = int(ppiv[j])
                if jj != j:
                    A[:r0, [r0 + j, r0 + jj]] = A[:r0, [r0 + jj, r0 + j]]
                    jpvt[[r0 + j, r0 + jj]] = jpvt[[r0 + jj, r0 + j]]
            out["pmargins"].append(pmg)
            out["ptops"].append(np.array(tp))
        else:
            # unpivoted Householder QR of the panel (P-hat = I)
            t = householder_qr(panel, steps=bi)
        tau[r0:r0 + bi] = t
        V = unit_lower(A[r0:, r0:r0 + bi], mi, bi)
        T = wy_T(V, t)
        out["T"].append(T)
        # trailing update: C <- (I - V T V^T)^T C = C - V (T^T (V^T C))
        C = A[r0:, r0 + bi:]
        if C.shape[1]:
            C -= V @ (T.T @ (V.T @ C))
        if diagonalize:
            # Section 6.2: R22 = U' D V'^T (full SVD of the b_i x b_i triangle);
            # U-tilde = Q-tilde diag(U', I) puts U'^T on the block's rows right
            # of it, V-tilde = V' multiplies the block's columns above it (and
            # P); the triangle becomes D, the reflectors below it stay
            R22 = np.triu(A[r0:r0 + bi, r0:r0 + bi])
            U1, d, V1t = np.linalg.svd(R22)
            V1 = V1t.T
            A[r0:r0 + bi, r0 + bi:] = U1.T @ A[r0:r0 + bi, r0 + bi:]
            A[:r0, r0:r0 + bi] = A[:r0, r0:r0 + bi] @ V1
            blk = A[r0:r0 + bi, r0:r0 + bi]
            blk[np.triu_indices(bi)] = 0.0
            blk[np.arange(bi), np.arange(bi)] = d
            out["D"].append((U1, V1))
    out.update(F=A, tau=tau, jpvt=jpvt, rank=k, b=b, p=p, pivot=pivot)
    return out


# ---------------------------------------------------------------------------
# Q and P from the stored factors; truncation (Section 6.1)


def block_reflectors(res):
    """Per block: (r0, V_i, T_i) with V_i of size (m - r0) x b_i."""
    F = res["F"]
    m = F.shape[0]
    outl = []
    for (r0, bi), T in zip(res["blocks"], res["T"]):
        outl.append((r0, unit_lower(F[r0:, r0:r0 + bi], m - r0, bi), T))
    return outl


def apply_q(res, C, trans):
    """Q C (trans=False) or Q^T C (trans=True), Q = prod_i diag(I, Q_i) with
    Q_i = I - V_i T_i V_i^T, times diag(U'_i, I) for diagonalised blocks."""
    C = np.array(C, dtype=np.float64, copy=True)
    blocks = block_reflectors(res)
    Us = [u for u, _ in res.get("D", [])] or [None] * len(blocks)
    seq = list(zip(blocks, Us))
    for (r0, V, T), U1 in (seq if trans else seq[::-1]):
        bi = V.shape[1]
        if U1 is not None and not trans:
            C[r0:r0 + bi] = U1 @ C[r0:r0 + bi]
        Tt = T.T if trans else T
        Cs = C[r0:]
        Cs -= V @ (Tt @ (V.T @ Cs))
        if U1 is not None and trans:
            C[r0:r0 + bi] = U1.T @ C[r0:r0 + bi]
    return C


def form_q(res, ncols):
    m = res["F"].shape[0]
    E = np.zeros((m, ncols))
    E[np.arange(ncols), np.arange(ncols)] = 1.0
    return apply_q(res, E, trans=False)


def form_p(res):
    """P as an explicit n x n matrix, so that A P = Q R."""
    n = res["F"].shape[1]
    if res["pivot"] == "perm":
        P = np.zeros((n, n))
        P[res["jpvt"], np.arange(n)] = 1.0
        return P
    P = np.eye(n)
    Vs = [v for _, v in res.get("D", [])] or [None] * len(res["S"])
    for (r0, bi), (VS, _, TS), V1 in zip(res["blocks"], res["S"], Vs):
        Pc = P[:, r0:]
        Pc -= ((Pc @ VS) @ TS) @ VS.T
        if V1 is not None:
            P[:, r0:r0 + bi] = P[:, r0:r0 + bi] @ V1
    return P


def r_factor(res):
    return np.triu(res["F"])


def lowrank(res, k):
    """A_k = Q(:, 0:k) R(0:k, :) P^* (Section 7's truncation of eq. AP=QR)."""
    Qk = form_q(res, k)
    Rk = np.triu(res["F"])[:k, :]
    return (Qk @ Rk) @ form_p(res).T


# ---------------------------------------------------------------------------
# Gradient of L(A) = ||A_k - B||_F^2 with the pivots held fixed


def lowrank_grad(A, jpvt, k, Gbar):
    """dL/dA for A_k = Pi A, Pi = Q_k Q_k^T, Q_k spanning A(:, jpvt[:k]).

    With A_1 = A P_k, A_1 = Q_k R_11 and R_k = Q_k^T A P:
      dA = Q_k (Q_k^T Gbar) + scatter_{jpvt[:k]}(Z),
      Z  = (I - Pi) [Gbar P R_k^T + A Gbar^T Q_k] R_11^{-T}.
    Q_k, R_11 come from this oracle's own unpivoted Householder QR of A_1.
    """
    A = np.asarray(A, dtype=np.float64)
    m, n = A.shape
    jpvt = np.asarray(jpvt)
    A1 = A[:, jpvt[:k]].copy()
    F = A1.copy()
    t = householder_qr(F, steps=k)
    V = unit_lower(F, m, k)
    T = wy_T(V, t)
    E = np.zeros((m, k))
    E[np.arange(k), np.arange(k)] = 1.0
    Qk = E - V @ (T @ (V.T @ E))
    R11 = np.triu(F[:k, :k])
    Rk = Qk.T @ A[:, jpvt]
    GP = Gbar[:, jpvt]
    M = GP @ Rk.T + A @ (Gbar.T @ Qk)
    M = M - Qk @ (Qk.T @ M)
    Z = np.linalg.solve(R11, M.T).T           # M R_11^{-T}
    dA = Qk @ (Qk.T @ Gbar)
    dA[:, jpvt[:k]] += Z
    return dA


# ---------------------------------------------------------------------------
# One-sided (Hestenes) Jacobi SVD, for singular values (Section 6.1)


def jacobi_singular_values(A, max_sweeps=60):
    """Singular values of A (m >= n) by one-sided Jacobi rotations.

    Columns are orthogonalised pairwise until every pair satisfies
    |a_p^T a_q| <= eps * |a_p| |a_q|; the singular values are the final
    column norms, sorted in decreasing order.  Pairs are visited in
    round-robin order, n/2 disjoint pairs at a time.
    """
    U = np.array(A, dtype=np.float64, copy=True)
    m, n = U.shape
    eps = np.finfo(np.float64).eps
    nn = n + (n % 2)
    idx = list(range(nn))
    for _ in range(max_sweeps):
        rotated = False
        for _ in range(nn - 1):
            ps = np.array([idx[t] for t in range(nn // 2)])
            qs = np.array([idx[nn - 1 - t] for t in range(nn // 2)])
            keep = (ps < n) & (qs < n)
            ps, qs = ps[keep], qs[keep]
            if ps.size:
                a = np.einsum("ij,ij->j", U[:, ps], U[:, ps])
                bb = np.einsum("ij,ij->j", U[:, qs], U[:, qs])
                c = np.einsum("ij,ij->j", U[:, ps], U[:, qs])
                act = np.abs(c) > eps * np.sqrt(a * bb)
                if np.any(act):
                    rotated = True
                    a, bb, c = a[act], bb[act], c[act]
                    pa, qa = ps[act], qs[act]
                    zeta = (bb - a) / (2.0 * c)
                    tt = np.sign(zeta) / (np.abs(zeta) + np.sqrt(1.0 + zeta * zeta))
                    tt[zeta == 0] = 1.0
                    cs = 1.0 / np.sqrt(1.0 + tt * tt)
                    sn = cs * tt
                    up = U[:, pa].copy()
                    uq = U[:, qa].copy()
                    U[:, pa] = cs * up - sn * uq
                    U[:, qa] = sn * up + cs * uq
            idx = [idx[0]] + [idx[-1]] + idx[1:-1]
        if not rotated:
            break
    return np.sort(np.sqrt(np.einsum("ij,ij->j", U, U)))[::-1]
