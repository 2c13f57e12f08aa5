"""GPU parity of the diagonalised blocks (Section 6.2) and of blockRRQR
(Method 3, Fig. 5: orthonormal pivoting, power iteration, diagonal blocks)
through the C ABI, against the oracle on the same sketches.

Compared: the diagonal D of R within max(1e-10, u kappa) |A| (kappa as in
the orthonormal-form parity of the power iteration: the conditioning of the
sketch rows that fix S_i), the truncation errors e_k, the structure of R
(exactly diagonal blocks, D >= 0 decreasing inside a block) and the
invariants Q^T A P = R, Q and P orthogonal, with Q and P assembled from the
library's outputs (reflectors, T, S blocks, U' and V') by the oracle's
routines."""
import numpy as np
import pytest
import torch

import paper_1505_08115_amd as R
import workloads as W
from oracle import rqrcp as O
from tests import section7 as S7
from tests.parity import progress

pytestmark = pytest.mark.gpu
DEV = "cuda"
U = np.finfo(np.float64).eps / 2


def _as_result(Fz, m, n, b):
    """The library's outputs in the oracle's result layout."""
    k = Fz.rank
    F = Fz.F.cpu().numpy()
    T = Fz.T.cpu().numpy()
    S = Fz.S.cpu().numpy()
    nb = -(-k // b)
    blocks = [(i * b, min(b, k - i * b)) for i in range(nb)]
    vs, off = [], 0
    for i in range(nb):
        vs.append(S[off:off + (n - i * b) * b].reshape((n - i * b, b), order="F"))
        off += (n - i * b) * b
    off += nb * b                                   # tau_S
    ts = [S[off + i * b * b: off + (i + 1) * b * b].reshape((b, b), order="F") for i in range(nb)]
    off += nb * b * b
    uv = []
    for i in range(nb):
        u = S[off + 2 * i * b * b: off + (2 * i + 1) * b * b].reshape((b, b), order="F")
        v = S[off + (2 * i + 1) * b * b: off + (2 * i + 2) * b * b].reshape((b, b), order="F")
        uv.append((u, v))
    res = {"F": F, "blocks": blocks, "pivot": "ortho", "rank": k, "T": [], "S": [], "D": []}
    for i, (r0, bi) in enumerate(blocks):
        res["T"].append(T[i * b * b:(i + 1) * b * b].reshape((b, b), order="F")[:bi, :bi])
        res["S"].append((vs[i][:, :bi], None, ts[i][:bi, :bi]))
        res["D"].append((uv[i][0][:bi, :bi], uv[i][1][:bi, :bi]))
    return res


def _kappa(ref):
    return max(np.linalg.cond(Y[:bi]) * ref["xnorm"][0] / xn
               for (_, bi), Y, xn in zip(ref["blocks"], ref["Y"], ref["xnorm"]))


CASES = [
    # m, n, b, p, q, rank
    (96, 96, 16, 8, 1, 0),
    (300, 250, 32, 16, 2, 0),       # ragged last block
    (256, 200, 64, 32, 1, 100),     # truncated rank, b at the kernel's limit
    (200, 150, 25, 12, 0, 0),       # odd block: the Jacobi schedule's padding column
]


@pytest.mark.parametrize("m,n,b,p,q,rank", CASES)
def test_diagonalised_blocks_match_oracle(m, n, b, p, q, rank):
    progress(f"blockRRQR m={m} n={n} b={b} p={p} q={q} rank={rank}")
    A = W.make_matrix(m, n, W.sigma_geometric(n, 6.0), seed=m + b).numpy()
    ref = O.rqrcp(A, b, p, seed=21, pivot="ortho", power=q, rank=rank, diagonalize=True, trace=True)
    Fz = R.factor(torch.tensor(A, device=DEV), block=b, oversample=p, seed=21, pivot="ortho", power=q, rank=rank,
                  diagonalize=True)
    torch.cuda.synchronize()
    k = ref["rank"]
    nA = np.linalg.norm(A)
    tol = max(1e-10, U * _kappa(ref))
    d_gpu, d_ref = np.diag(Fz.F.cpu().numpy())[:k], np.diag(ref["F"])[:k]
    assert np.max(np.abs(d_gpu - d_ref)) <= tol * nA
    res = _as_result(Fz, m, n, b)
    Rg = np.triu(res["F"])
    for r0, bi in res["blocks"]:
        blk = Rg[r0:r0 + bi, r0:r0 + bi]
        d = np.diag(blk)
        assert np.all(blk - np.diag(d) == 0.0)
        assert np.all(d >= 0) and np.all(d[:-1] >= d[1:])
    Q, P = O.form_q(res, m), O.form_p(res)
    QAP = Q.T @ A @ P
    assert np.linalg.norm(QAP[:k] - Rg[:k]) / nA <= 1e-13
    assert np.linalg.norm(Q.T @ Q - np.eye(m)) <= 1e-12
    assert np.linalg.norm(P.T @ P - np.eye(n)) <= 1e-12
    with pytest.raises(R.RqrcpError):
        R.lowrank(Fz)


@pytest.mark.parametrize("name,make", [("fast", S7.a_fast), ("gauss", S7.a_gauss)])
def test_gpu_method_3_diagonal_tracks_the_singular_values(name, make):
    """Section 7's Method 3 (b = 50, p = 25) with q = 2 power steps."""
    A = make(1)
    Fz = R.factor(torch.tensor(A, device=DEV), block=S7.B, oversample=S7.B // 2, seed=1, pivot="ortho", power=2,
                  diagonalize=True)
    torch.cuda.synchronize()
    ref = O.rqrcp(A, S7.B, S7.B // 2, seed=1, pivot="ortho", power=2, diagonalize=True)
    e_gpu = S7.errors_from_r(Fz.F.cpu().numpy())
    np.testing.assert_allclose(e_gpu, S7.errors_from_r(ref["F"]), rtol=1e-6, atol=0)
    s = np.linalg.svd(A, compute_uv=False)
    d = np.diag(Fz.F.cpu().numpy())
    assert np.median(np.abs(np.log(d / s))) <= 0.05
    assert S7.summary(e_gpu, A)["to_svd_geomean"] <= 1.02


@pytest.mark.parametrize("rank_a", [0, 20])
def test_diagonalised_blocks_of_rank_deficient_inputs(rank_a):
    """Exact rank 20 (the rank falls inside the second block) and the zero
    matrix: the triangles past the rank have singular values at rounding
    level, whose U' columns the kernel completes to an orthonormal basis."""
    m, n, b = 120, 96, 16
    progress(f"blockRRQR rank-deficient rank={rank_a}")
    if rank_a:
        A = W.make_matrix(m, n, W.sigma_rank(n, rank_a), seed=7).numpy()
    else:
        A = np.zeros((m, n))
    Fz = R.factor(torch.tensor(A, device=DEV), block=b, oversample=8, seed=3, pivot="ortho", power=1,
                  diagonalize=True)
    torch.cuda.synchronize()
    ref = O.rqrcp(A, b, 8, seed=3, pivot="ortho", power=1, diagonalize=True)
    nA = max(np.linalg.norm(A), 1.0)
    d = np.diag(Fz.F.cpu().numpy())
    assert np.max(np.abs(d - np.diag(ref["F"]))) <= 1e-9 * nA
    assert np.all(d[max(rank_a, 0):] <= 1e-12 * nA)
    res = _as_result(Fz, m, n, b)
    Q, P = O.form_q(res, m), O.form_p(res)
    Rg = np.triu(res["F"])
    assert np.linalg.norm(Q.T @ A @ P - Rg) / nA <= 1e-13
    assert np.linalg.norm(Q.T @ Q - np.eye(m)) <= 1e-12
    assert np.linalg.norm(P.T @ P - np.eye(n)) <= 1e-12


def test_orthonormal_completion_with_noise_across_the_threshold():
    """Rank 20 plus trailing singular values spread from 1e-11 to 1e-18: the
    triangles past the rank hold rounding-level entries on both sides of the
    Jacobi kernel's acceptance threshold (b eps times the triangle's largest
    singular value), so some columns of U' come from the rotations and the
    rest from the orthonormal completion; U' must stay orthogonal."""
    m, n, b = 120, 96, 16
    s = np.concatenate([np.ones(20), np.geomspace(1e-11, 1e-18, n - 20)])
    A = W.make_matrix(m, n, s, seed=17).numpy()
    Fz = R.factor(torch.tensor(A, device=DEV), block=b, oversample=8, seed=5, pivot="ortho", power=1,
                  diagonalize=True)
    assert Fz.check() == [0, 0, 0, 0]
    res = _as_result(Fz, m, n, b)
    worst = 0.0
    for u, v in res["D"]:
        bi = u.shape[0]
        worst = max(worst, np.linalg.norm(u.T @ u - np.eye(bi)), np.linalg.norm(v.T @ v - np.eye(bi)))
    progress(f"completion across the threshold: worst |U'^T U' - I|, |V'^T V' - I| = {worst:.2e}")
    assert worst <= 1e-12
    Q, P = O.form_q(res, m), O.form_p(res)
    nA = np.linalg.norm(A)
    assert np.linalg.norm(Q.T @ A @ P - np.triu(res["F"])) / nA <= 1e-13
    assert np.linalg.norm(Q.T @ Q - np.eye(m)) <= 1e-12
    assert np.linalg.norm(P.T @ P - np.eye(n)) <= 1e-12
