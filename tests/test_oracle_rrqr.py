"""Pins of the oracle's diagonalised blocks (Section 6.2) and blockRRQR
(Method 3: orthonormal pivoting, power iteration, diagonalised blocks;
Fig. 5).  Checked against the SVD (a single block is a full SVD of A),
the factorization invariants with the U' and V' factors folded into Q and
P, the structure of R, and Section 7's observation that Method 3 with q = 2
puts the singular values on the diagonal of R."""
import numpy as np
import pytest

import workloads as W
from oracle import rqrcp as O
from tests import section7 as S7

U = np.finfo(np.float64).eps / 2


def test_one_block_is_a_full_svd():
    m, n = 60, 40
    A = W.make_matrix(m, n, W.sigma_geometric(n, 6.0), seed=3).numpy()
    res = O.rqrcp(A, 64, 8, seed=1, pivot="ortho", diagonalize=True)
    s = np.linalg.svd(A, compute_uv=False)
    R = np.triu(res["F"])[:n]
    assert np.allclose(R, np.diag(np.diag(R)), atol=0.0)
    assert np.max(np.abs(np.diag(R) - s)) <= 50 * U * s[0]


@pytest.mark.parametrize("m,n,b,p,q,rank", [(90, 70, 16, 8, 1, 0), (64, 64, 8, 4, 2, 0), (100, 80, 24, 12, 0, 40)])
def test_invariants_and_diagonal_blocks(m, n, b, p, q, rank):
    A = W.make_matrix(m, n, W.sigma_geometric(n, 8.0), seed=m + q).numpy()
    res = O.rqrcp(A, b, p, seed=2, pivot="ortho", diagonalize=True, power=q, rank=rank)
    k = res["rank"]
    Q, P = O.form_q(res, m), O.form_p(res)
    R = np.triu(res["F"])
    nA = np.linalg.norm(A)
    QAP = Q.T @ A @ P
    assert np.linalg.norm(QAP[:k] - R[:k]) / nA <= 20 * n * U
    if rank == 0:
        assert np.linalg.norm(QAP - R) / nA <= 20 * n * U
    assert np.linalg.norm(Q.T @ Q - np.eye(m)) <= 20 * n * U
    assert np.linalg.norm(P.T @ P - np.eye(n)) <= 20 * n * U
    for r0, bi in res["blocks"]:
        blk = R[r0:r0 + bi, r0:r0 + bi]
        d = np.diag(blk)
        assert np.all(blk - np.diag(d) == 0.0)
        assert np.all(d >= 0) and np.all(d[:-1] >= d[1:])


def test_diagonalisation_needs_orthonormal_pivoting():
    with pytest.raises(ValueError):
        O.rqrcp(np.eye(8), 4, 0, seed=1, pivot="perm", diagonalize=True)


@pytest.mark.parametrize("name,make", [("fast", S7.a_fast), ("gauss", S7.a_gauss)])
def test_section_7_method_3_diagonal_tracks_the_singular_values(name, make):
    A = make(1)
    s = np.linalg.svd(A, compute_uv=False)
    dev, gm = [], []
    for q in (0, 1, 2):
        res = O.rqrcp(A, S7.B, S7.B // 2, seed=1, pivot="ortho", diagonalize=True, power=q)
        d = np.abs(np.diag(res["F"]))
        dev.append(np.median(np.abs(np.log(d / s))))
        gm.append(S7.summary(S7.errors_from_r(res["F"]), A)["to_svd_geomean"])
    # q = 2: |R_kk| within a few per cent of sigma_k in the median, e_k within 2 %
    # of the optimum on average; more power steps help
    assert dev[2] <= 0.05 and gm[2] <= 1.02
    assert dev[2] <= dev[1] <= dev[0] and gm[2] <= gm[1] <= gm[0]
    # and Method 3 beats Method 2 at the same q
    m2 = O.rqrcp(A, S7.B, S7.B // 2, seed=1, pivot="ortho", power=2)
    assert gm[2] <= S7.summary(S7.errors_from_r(m2["F"]), A)["to_svd_geomean"]
