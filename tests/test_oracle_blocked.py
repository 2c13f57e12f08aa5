"""Pins of the oracle's blocked randomized QR (Sections 4-6, Fig. 3) against
invariants, reductions to textbook routines and library factorizations."""
import numpy as np
import pytest
import scipy.linalg as sla

import workloads as W
from oracle import rqrcp as O

U = np.finfo(np.float64).eps / 2


def _factors(res, n):
    Q = O.form_q(res, n)
    R = np.triu(res["F"])[:n]
    P = O.form_p(res)
    return Q, R, P


def _sign_normalise(R):
    d = np.sign(np.diag(R))
    d[d == 0] = 1
    return d[:, None] * R


CASES = [
    # m, n, b, p, pivot
    (64, 64, 8, 4, "perm"),
    (90, 70, 16, 5, "perm"),       # n not a multiple of b, m > n
    (50, 50, 64, 3, "perm"),       # b >= n: one block, the tail
    (77, 77, 10, 0, "perm"),       # no oversampling
    (64, 64, 8, 4, "ortho"),
    (90, 70, 16, 5, "ortho"),
]


@pytest.mark.parametrize("m,n,b,p,pivot", CASES)
def test_factorisation_invariants(m, n, b, p, pivot):
    A = W.make_matrix(m, n, W.sigma_geometric(n, 8.0), seed=m + n).numpy()
    res = O.rqrcp(A, b, p, seed=7, pivot=pivot)
    Q, R, P = _factors(res, n)
    nA = np.linalg.norm(A)
    assert np.linalg.norm(A @ P - Q @ R) / nA <= 10 * n * U
    assert np.linalg.norm(Q.T @ Q - np.eye(n)) <= 10 * n * U
    assert np.linalg.norm(P.T @ P - np.eye(n)) <= 10 * n * U
    assert np.all(np.tril(R, -1) == 0)
    if pivot == "perm":
        assert sorted(res["jpvt"]) == list(range(n))
    else:
        assert list(res["jpvt"]) == list(range(n))


def test_blocks_zero_below_diagonal_after_each_block():
    # Fig. 4: after block i the first r0 + b columns are upper triangular
    m, n, b = 40, 40, 8
    A = W.make_matrix(m, n, W.sigma_geometric(n, 4.0), seed=3).numpy()
    for k in (8, 16, 24):
        res = O.rqrcp(A, b, 3, seed=1, rank=k)
        Q = O.form_q(res, m)
        Rk = Q.T @ A[:, res["jpvt"]]
        assert np.abs(Rk[k:, :k]).max() <= 64 * U * np.linalg.norm(A)


@pytest.mark.parametrize("m,n,b,pivot", [(60, 48, 8, "perm"), (60, 48, 8, "ortho"), (41, 41, 7, "perm")])
def test_r_is_the_qr_factor_of_a_times_p(m, n, b, pivot):
    """Given P, R is unique up to row signs: the blocked loop's R equals
    LAPACK's unpivoted QR of A P (pins the panel, WY and trailing update)."""
    A = W.make_matrix(m, n, W.sigma_geometric(n, 3.0), seed=11).numpy()
    res = O.rqrcp(A, b, 4, seed=5, pivot=pivot)
    _, R, P = _factors(res, n)
    Rl = sla.qr(A @ P, mode="r")[0][:n]
    np.testing.assert_allclose(_sign_normalise(R), _sign_normalise(Rl), atol=1e-12 * np.linalg.norm(A))


def test_exact_sample_reduces_to_classical_qrcp():
    """With Y_i := X_i every block repeats classical QRCP's choices: the
    blocked loop must give the pivots and R of Fig. 2's algorithm."""
    m, n = 48, 40
    A = W.make_matrix(m, n, W.sigma_geometric(n, 6.0), seed=9).numpy()
    res = O.rqrcp(A, 8, 0, seed=0, sampler="identity")
    F = A.copy()
    _, jpvt, _, margins = O.qrcp(F, record_margins=True)
    assert margins[:-1].min() > 1e-8
    assert list(res["jpvt"]) == list(jpvt)
    np.testing.assert_allclose(_sign_normalise(np.triu(res["F"])[:n]),
                               _sign_normalise(np.triu(F)[:n]), atol=1e-13)


def test_block_pivots_equal_geqp3_on_the_sketch():
    """Eq. Yrows, first b steps: each block's chosen columns are LAPACK's
    pivoted QR of Y_i (leading b_i entries of its permutation)."""
    m, n, b, p = 80, 64, 16, 6
    A = W.make_matrix(m, n, W.sigma_geometric(n, 5.0), seed=21).numpy()
    res = O.rqrcp(A, b, p, seed=4, trace=True, tail="sampled")
    for (r0, bi), Y, piv, mg in zip(res["blocks"], res["Y"], res["piv"], res["margins"]):
        if mg[:bi].min() < 1e-8:
            continue
        _, _, Pl = sla.qr(Y, pivoting=True)
        order = np.arange(Y.shape[1])
        for j in range(bi):
            order[[j, piv[j]]] = order[[piv[j], j]]
        assert list(order[:bi]) == list(Pl[:bi])


def test_sketch_uses_counter_generator_and_explicit_g_hook():
    m, n, b, p = 30, 24, 8, 2
    A = W.make_matrix(m, n, W.sigma_geometric(n, 3.0), seed=2).numpy()
    r1 = O.rqrcp(A, b, p, seed=13, tail="sampled")
    Gs = [O.sketch(13, i, b + p, i * b, m - i * b) for i in range(3)]
    r2 = O.rqrcp(A, b, p, seed=0, G=Gs, tail="sampled")
    np.testing.assert_array_equal(r1["F"], r2["F"])
    np.testing.assert_array_equal(r1["jpvt"], r2["jpvt"])


def test_truncated_run_repeats_the_leading_rows_of_the_full_run():
    m, n, b = 64, 64, 8
    A = W.make_matrix(m, n, W.sigma_geometric(n, 8.0), seed=5).numpy()
    full = O.rqrcp(A, b, 4, seed=3)
    for k in (5, 16, 20):
        tr = O.rqrcp(A, b, 4, seed=3, rank=k)
        # same sketches and pivot choices for the first k columns
        np.testing.assert_array_equal(tr["jpvt"][:k], full["jpvt"][:k])
        if k % b == 0:      # whole blocks: the very same arithmetic
            np.testing.assert_array_equal(tr["F"][:, :k], full["F"][:, :k])
        # R(0:k, :) P^T does not depend on where the unchosen columns went
        Rt = np.zeros((k, n))
        Rf = np.zeros((k, n))
        Rt[:, tr["jpvt"]] = np.triu(tr["F"])[:k]
        Rf[:, full["jpvt"]] = np.triu(full["F"])[:k]
        np.testing.assert_allclose(Rt, Rf, atol=1e-13 * np.linalg.norm(A))


def test_exact_rank_input_leaves_a_zero_trailing_block():
    m, n, k = 60, 60, 13
    A = W.integer_rank_k(m, n, k, seed=1)
    res = O.rqrcp(A, 8, 4, seed=2)
    R = np.triu(res["F"])
    assert np.linalg.norm(R[k:, k:]) <= 100 * U * np.sqrt(n) * np.linalg.norm(A)
    assert np.abs(np.diag(R)[:k]).min() > 1e-6 * np.linalg.norm(A)


@pytest.mark.parametrize("pivot", ["perm", "ortho"])
def test_singular_value_identities(pivot):
    """|R_11| <= s_1; sum_{i<=k} log|R_ii| <= sum_{i<=k} log s_i, with
    equality at k = n for a square matrix (|det A| = |det R|)."""
    n = 48
    s = W.sigma_geometric(n, 4.0)
    A = W.make_matrix(n, n, s, seed=8).numpy()
    sv = np.linalg.svd(A, compute_uv=False)
    res = O.rqrcp(A, 8, 4, seed=1, pivot=pivot)
    d = np.abs(np.diag(res["F"]))
    assert d[0] <= sv[0] * (1 + 1e-13)
    cl = np.cumsum(np.log(d))
    cs = np.cumsum(np.log(sv))
    assert np.all(cl <= cs + 1e-10)
    assert abs(cl[-1] - cs[-1]) <= 1e-9
    assert d[-1] >= sv[-1] * (1 - 1e-10)


@pytest.mark.parametrize("pivot", ["perm", "ortho"])
def test_truncation_error_identity_and_eckart_young(pivot):
    """Section 6.1: |A P - Q_1 [R_11 R_12]| = |R_22|, and no rank-k
    approximation beats the truncated SVD."""
    m, n, k = 70, 50, 17
    s = W.sigma_geometric(n, 6.0)
    A = W.make_matrix(m, n, s, seed=4).numpy()
    sv = np.linalg.svd(A, compute_uv=False)
    res = O.rqrcp(A, 8, 4, seed=9, pivot=pivot)
    Ak = O.lowrank(res, k)
    R22 = np.triu(res["F"])[k:n, k:]
    err_f = np.linalg.norm(A - Ak)
    assert err_f == pytest.approx(np.linalg.norm(R22), rel=1e-8)
    assert err_f >= np.sqrt(np.sum(sv[k:] ** 2)) * (1 - 1e-12)
    assert np.linalg.norm(A - Ak, 2) >= sv[k] * (1 - 1e-12)


def test_graded_orthogonal_randomized_pivots_are_the_closed_form_order():
    A, order = W.graded_orthogonal(64, 48, seed=6, decades=12.0)
    res = O.rqrcp(A, 8, 8, seed=3)
    assert list(res["jpvt"]) == list(order)


def test_margin_log_marks_exact_ties_as_unseparated():
    A = np.zeros((20, 10))
    A[:3, :3] = np.eye(3)
    res = O.rqrcp(A, 4, 2, seed=1)
    assert min(mg.min() for mg in res["margins"]) == 0.0


def test_rejects_wide_matrices_and_bad_rank():
    with pytest.raises(ValueError):
        O.rqrcp(np.zeros((3, 5)), 2, 1, seed=0)
    with pytest.raises(ValueError):
        O.rqrcp(np.zeros((5, 5)), 2, 1, seed=0, rank=9)


@pytest.mark.parametrize("m,n,b,p", [(200, 160, 32, 8), (150, 150, 40, 0), (300, 250, 64, 20)])
def test_ortho_S_equals_lapack_qr_of_the_sketch_transpose(m, n, b, p):
    """Section 4.2 (eq. Ycols and its Remark): S_i = H_1 ... H_{b_i} of the
    unpivoted Householder QR of Y_i^T.  LAPACK's dgeqrf of Y_i^T (all b+p
    columns; the first b_i reflectors depend only on the first b_i columns)
    must give the same reflectors and scalars (dlarfg takes beta =
    -sign(alpha) |x|, the paper's sign), and its explicit Q the same first
    b_i columns as I - V_S T_S V_S^T.  A transposed sketch, a pivoted QR or a
    wrong block of rows would fail here."""
    A = W.make_matrix(m, n, W.sigma_geometric(n, 3.0), seed=m + b).numpy()
    ref = O.rqrcp(A, b, p, seed=4, pivot="ortho", trace=True)
    for (r0, bi), Y, (VS, ts, TS) in zip(ref["blocks"], ref["Y"], ref["S"]):
        ni = n - r0
        qr, tau, _, info = sla.lapack.dgeqrf(Y.T.copy())
        assert info == 0
        VL = np.tril(qr[:, :bi], -1)
        VL[np.arange(bi), np.arange(bi)] = 1.0
        scale = np.linalg.cond(Y[:bi]) * 1e-14
        np.testing.assert_allclose(ts, tau[:bi], rtol=0, atol=scale)
        np.testing.assert_allclose(VS, VL, rtol=0, atol=scale * max(1.0, np.abs(VL).max()))
        QL, _, info = sla.lapack.dorgqr(qr[:, :bi].copy(), tau[:bi].copy())
        assert info == 0
        S = np.eye(ni) - VS @ TS @ VS.T
        np.testing.assert_allclose(S[:, :bi], QL, rtol=0, atol=scale)
