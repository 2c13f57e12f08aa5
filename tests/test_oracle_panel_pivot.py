"""Pins of the oracle's in-block pivot P-hat (Fig. 3: the panel of every
sketched block factored by QR with column pivoting).  Checked against
LAPACK's column-pivoted QR (geqp3 through scipy) of each block's columns
projected off the span of the earlier blocks' columns, against the ordering
property of column pivoting, and against the factorization invariants."""
import numpy as np
import pytest
import scipy.linalg as sla

import workloads as W
from oracle import rqrcp as O

U = np.finfo(np.float64).eps / 2


@pytest.mark.parametrize("m,n,b,p,tail", [(90, 70, 16, 5, "classical"), (64, 64, 8, 4, "sampled"),
                                          (120, 100, 24, 0, "classical")])
def test_in_block_order_is_lapack_pivoted_qr_of_the_projected_block(m, n, b, p, tail):
    A = W.make_matrix(m, n, W.sigma_geometric(n, 6.0), seed=m + b).numpy()
    res = O.rqrcp(A, b, p, seed=3, tail=tail, panel_pivot=True)
    jp = res["jpvt"]
    for i, (r0, bi) in enumerate(res["blocks"]):
        if i >= len(res["pmargins"]):
            break                                 # the classical tail has no P-hat step
        cols = np.sort(jp[r0:r0 + bi])            # the block's column set, in input order
        if r0:
            Q1 = np.linalg.qr(A[:, jp[:r0]])[0]
            M = A[:, cols] - Q1 @ (Q1.T @ A[:, cols])
        else:
            M = A[:, cols]
        _, _, perm = sla.qr(M, pivoting=True, mode="economic")
        assert list(cols[perm]) == list(jp[r0:r0 + bi]), f"block {i}"


def test_diagonal_of_r_decreases_inside_every_pivoted_block():
    m, n, b = 100, 80, 16
    A = W.make_matrix(m, n, W.sigma_geometric(n, 5.0), seed=4).numpy()
    res = O.rqrcp(A, b, 6, seed=1, panel_pivot=True)
    d = np.abs(np.diag(res["F"]))
    for r0, bi in res["blocks"]:
        blk = d[r0:r0 + bi]
        assert np.all(blk[:-1] >= blk[1:] * (1 - 1e-12))


def test_factorisation_invariants_and_default_off():
    m, n, b = 90, 70, 16
    A = W.make_matrix(m, n, W.sigma_geometric(n, 8.0), seed=9).numpy()
    res = O.rqrcp(A, b, 5, seed=2, panel_pivot=True)
    Q, R, P = O.form_q(res, n), np.triu(res["F"])[:n], O.form_p(res)
    assert np.linalg.norm(A @ P - Q @ R) / np.linalg.norm(A) <= 10 * n * U
    assert np.linalg.norm(Q.T @ Q - np.eye(n)) <= 10 * n * U
    assert sorted(res["jpvt"]) == list(range(n))
    # the first block takes the same columns as without P-hat, in another
    # order (later blocks sample a trailing matrix whose rows are expressed
    # in another orthonormal basis, hence see other sketches)
    ref = O.rqrcp(A, b, 5, seed=2)
    assert set(ref["jpvt"][:b]) == set(res["jpvt"][:b])
    assert list(ref["jpvt"][:b]) != list(res["jpvt"][:b])
    assert not ref["pmargins"]
