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


def _bar(*dims):
    """The invariant bound of any output, |A P - Q R| / |A| and |Q^T Q - I|
    within 10 n u (n the larger dimension), never below the 1e-13 that the
    small cases meet."""
    return max(1e-13, 10 * max(dims) * U)


def _orth_bar(n, b):
    """|Q^T Q - I| and |P^T P - I|: 10 n u for the reflectors (at least 1e-12),
    plus what V' (and U') gather from the Jacobi rotations: a column of the
    b x b block meets at most 40 (b - 1) of them, each adding a rounding of
    about u, so a pair of columns drifts by about u sqrt(40 b) and the b x b
    block by b u sqrt(40 b) in norm (twice that here; 1.5e-12 measured at
    b = 256 in an FP64 numpy run of the same iteration)."""
    return max(1e-12, 10 * n * U) + 2 * b * np.sqrt(40 * b) * U


def _errors(F):
    """e_k = |R(k:, k:)|_F for every k (Section 6.1's truncation error)."""
    rows = (np.triu(F) ** 2).sum(axis=1)
    return np.sqrt(np.cumsum(rows[::-1])[::-1])


def _kappa(ref):
    return max(np.linalg.cond(Y[:bi]) * ref["xnorm"][0] / xn
               for (_, bi), Y, xn in zip(ref["blocks"], ref["Y"], ref["xnorm"]))


CASES = [
    # m, n, b, p, q, rank
    (96, 96, 16, 8, 1, 0),
    (300, 250, 32, 16, 2, 0),       # ragged last block
    (256, 200, 64, 32, 1, 100),     # truncated rank, b at the kernel's limit
    (200, 150, 25, 12, 0, 0),       # odd block: the Jacobi schedule's padding column
    (300, 256, 128, 16, 1, 0),      # blocks above 64 columns: the cooperative Jacobi kernel
    (500, 400, 100, 16, 1, 0),      # 100 columns: a partial block of 16 and a padding block
    (600, 520, 256, 10, 2, 0),      # b = 256 with a last block of 8 (one-workgroup kernel)
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
    assert np.linalg.norm(QAP[:k] - Rg[:k]) / nA <= _bar(m, n)
    assert np.linalg.norm(Q.T @ Q - np.eye(m)) <= _orth_bar(m, b)
    assert np.linalg.norm(P.T @ P - np.eye(n)) <= _orth_bar(n, b)
    _check_apply_and_lowrank(Fz, res, A, Q, P)


def _check_apply_and_lowrank(Fz, res, A, Q, P):
    """Q and P applied by the library (with U' and V') against Q and P
    assembled from the same outputs by the oracle's routines, and the
    truncation A_k of every block boundary and of a column inside a block
    against the oracle's Section 6.1 formula on the same factors."""
    m, n = A.shape
    rng = np.random.default_rng(m + n)
    C = rng.standard_normal((m, 7))
    for trans in (False, True):
        Cg = R.colmajor(torch.tensor(C, device=DEV))
        R.apply_q(Fz, Cg, trans=trans)
        want = (Q.T if trans else Q) @ C
        assert np.linalg.norm(Cg.cpu().numpy() - want) <= _bar(m, n) * np.linalg.norm(C)
    D = rng.standard_normal((5, n))
    for trans in (False, True):
        Dg = R.colmajor(torch.tensor(D, device=DEV))
        R.apply_p(Fz, Dg, trans=trans)
        want = D @ (P.T if trans else P)
        assert np.linalg.norm(Dg.cpu().numpy() - want) <= _bar(m, n) * np.linalg.norm(D)
    nA = np.linalg.norm(A)
    b = Fz.block
    for k in sorted({min(b, Fz.rank), Fz.rank, max(1, min(Fz.rank, b + b // 2 + 1))}):
        Ak = R.lowrank(Fz, k).cpu().numpy()
        want = O.lowrank(res, k)
        progress(f"  lowrank k={k}: |A_k - oracle formula| / |A| = {np.linalg.norm(Ak - want) / nA:.2e}")
        assert np.linalg.norm(Ak - want) <= 1e-12 * nA


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


@pytest.mark.parametrize("rank_a,m,n,b", [(0, 120, 96, 16), (20, 120, 96, 16), (0, 300, 256, 128),
                                           (150, 300, 256, 128)])
def test_diagonalised_blocks_of_rank_deficient_inputs(rank_a, m, n, b):
    """Exact rank (falling inside the second block) and the zero matrix: the
    triangles past the rank have singular values at rounding level, whose U'
    columns the kernel completes to an orthonormal basis (b = 128: in the
    single-workgroup pass after the cooperative sweeps)."""
    progress(f"blockRRQR rank-deficient rank={rank_a} m={m} n={n} b={b}")
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
    assert np.linalg.norm(Q.T @ A @ P - Rg) / nA <= _bar(m, n)
    assert np.linalg.norm(Q.T @ Q - np.eye(m)) <= _orth_bar(m, b)
    assert np.linalg.norm(P.T @ P - np.eye(n)) <= _orth_bar(n, b)


@pytest.mark.parametrize("m,n,b,r", [(120, 96, 16, 20), (300, 256, 128, 150)])
def test_orthonormal_completion_with_noise_across_the_threshold(m, n, b, r):
    """Rank r plus trailing singular values spread from 1e-11 to 1e-18: the
    triangles past the rank hold rounding-level entries on both sides of the
    Jacobi kernel's acceptance threshold (b eps times the triangle's largest
    singular value), so some columns of U' come from the rotations and the
    rest from the orthonormal completion; U' must stay orthogonal."""
    s = np.concatenate([np.ones(r), np.geomspace(1e-11, 1e-18, n - r)])
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
    assert worst <= _orth_bar(0, b)
    Q, P = O.form_q(res, m), O.form_p(res)
    nA = np.linalg.norm(A)
    assert np.linalg.norm(Q.T @ A @ P - np.triu(res["F"])) / nA <= _bar(m, n)
    assert np.linalg.norm(Q.T @ Q - np.eye(m)) <= _orth_bar(m, b)
    assert np.linalg.norm(P.T @ P - np.eye(n)) <= _orth_bar(n, b)


@pytest.mark.parametrize("q", [1, 2])
def test_method_3_on_C3s_at_block_256(q):
    """blockRRQR at block size 256 on C3's 1024^2 subcase (singular
    values 1/j, a 1e-6 gap after 256): four blocks of 256, each triangle
    diagonalised by the cooperative Jacobi kernel.  D holds the singular
    values of A restricted to the span that a block's sketch picks, so it does
    not depend on the rotation inside that span (whose entries the u kappa
    bar of the other cases covers, above 1e-5 here); the span itself is as
    sensitive as the power-iterated sketch rows make it: at q = 2 the weak
    directions of the first block carry (sigma_256/sigma_1)^5 = 1e-12 of the
    rows' weight, and an input perturbation of u |A| moves the oracle's own D
    there by 1e-8 |A|.  So D and e_k are held to the oracle's within ten times
    what two such seeded perturbations change in the oracle's own result, and
    never looser than needed below 1e-10 |A|; then the invariants, and D on
    the singular values."""
    w = W.WORKLOADS["C3s"]
    A = W.workload_matrix(w).numpy()
    n = A.shape[1]
    progress(f"blockRRQR C3s b=256 q={q}")
    Fz = R.factor(torch.tensor(A, device=DEV), block=256, oversample=w.p, seed=w.seed, pivot="ortho", power=q,
                  diagonalize=True)
    assert Fz.check() == [0, 0, 0, 0]
    nA = np.linalg.norm(A)

    def oracle(M):
        r = O.rqrcp(M, 256, w.p, seed=w.seed, pivot="ortho", power=q, diagonalize=True)
        return r, np.diag(r["F"]), _errors(r["F"])

    ref, d_ref, e_ref = oracle(A)
    rng = np.random.default_rng(31)
    spread_d = spread_e = 0.0
    for _ in range(2):
        E = rng.standard_normal(A.shape)
        _, d2, e2 = oracle(A + E * (U * nA / np.linalg.norm(E)))
        spread_d = max(spread_d, np.max(np.abs(d2 - d_ref)))
        spread_e = max(spread_e, np.max(np.abs(e2 - e_ref)))
    tol_d, tol_e = max(1e-10 * nA, 10 * spread_d), max(1e-10 * nA, 10 * spread_e)
    d_gpu, e_gpu = np.diag(Fz.F.cpu().numpy()), _errors(Fz.F.cpu().numpy())
    progress(f"  max |D_gpu - D_oracle| / |A| = {np.max(np.abs(d_gpu - d_ref)) / nA:.2e} "
             f"(oracle under u|A| perturbations: {spread_d / nA:.2e}); e_k: "
             f"{np.max(np.abs(e_gpu - e_ref)) / nA:.2e} ({spread_e / nA:.2e})")
    assert np.max(np.abs(d_gpu - d_ref)) <= tol_d
    np.testing.assert_allclose(e_gpu, e_ref, rtol=1e-6, atol=tol_e)
    res = _as_result(Fz, n, n, 256)
    Rg = np.triu(res["F"])
    for r0, bi in res["blocks"]:
        blk = Rg[r0:r0 + bi, r0:r0 + bi]
        d = np.diag(blk)
        assert np.all(blk - np.diag(d) == 0.0)
        assert np.all(d >= 0) and np.all(d[:-1] >= d[1:])
    Q, P = O.form_q(res, n), O.form_p(res)
    assert np.linalg.norm(Q.T @ A @ P - Rg) / nA <= _bar(n)
    assert np.linalg.norm(Q.T @ Q - np.eye(n)) <= _orth_bar(n, 256)
    assert np.linalg.norm(P.T @ P - np.eye(n)) <= _orth_bar(n, 256)
    _check_apply_and_lowrank(Fz, res, A, Q, P)
    ratio = np.abs(np.log(d_gpu / w.sigma()))
    progress(f"  median |log(D/sigma)| = {np.median(ratio):.2e}, max {ratio.max():.2e}")
    assert np.median(ratio) <= (0.05 if q == 2 else 0.1)


@pytest.mark.parametrize("b", [32, 128])
def test_diagonalised_blocks_with_a_non_finite_input(b):
    """A NaN in the input reaches the SVD of the blocks' triangles: the
    factorization reports it in the info word (non-finite norm met, no
    grid-wide wait given up), and the finishing kernel's sort of the singular
    values still forms a permutation (a non-finite value sorts last)."""
    m, n = 300, 256
    A = W.make_matrix(m, n, W.sigma_geometric(n, 3.0), seed=3).numpy()
    A[5, 7] = np.nan
    progress(f"blockRRQR non-finite input b={b}")
    Fz = R.factor(torch.tensor(A, device=DEV), block=b, oversample=8, seed=2, pivot="ortho", power=1,
                  diagonalize=True)
    iv = Fz.check()
    assert iv[0] == 1 and iv[1] >= 1 and iv[2] == 0


@pytest.mark.parametrize("m,n,b,q,precision", [(300, 256, 64, 1, "plain"), (600, 520, 128, 1, "mixed"),
                                                (600, 520, 256, 2, "plain")])
def test_diagonalised_blocks_with_fp32_storage(m, n, b, q, precision):
    """FP32 storage (plain, or mixed with the BF16 sketch): the triangles'
    SVD and U'^T, V' products run in FP64 on widened copies.  Against the
    FP64 oracle on the FP32-rounded input (plain, q = 1): D within 1e-5 |A|
    (the FP32 rounding of the stored trailing matrices); every case: D on the
    singular values (median |log(D/sigma)|), exactly diagonal blocks with
    D >= 0 decreasing, Q^T A P = R within 1e-5, Q (reflectors stored in FP32)
    orthogonal to 1e-4 and P (FP64 S blocks and V') to the FP64 bar."""
    A32 = W.make_matrix(m, n, W.sigma_geometric(n, 4.0), seed=m + b).numpy().astype(np.float32)
    A = A32.astype(np.float64)
    progress(f"blockRRQR FP32 {precision} m={m} n={n} b={b} q={q}")
    Fz = R.factor(torch.tensor(A32, device=DEV), block=b, oversample=10, seed=9, pivot="ortho", power=q,
                  precision=precision, diagonalize=True)
    assert Fz.check() == [0, 0, 0, 0]
    nA = np.linalg.norm(A)
    d = np.diag(Fz.F.double().cpu().numpy())
    if precision == "plain" and q == 1:
        # (with q = 2 the FP32 power steps keep a block's weak directions only
        # to about u_32 (sigma_1 / sigma_b)^5 of the rows' weight, 1e-6 at b = 256
        # here, so the span a block picks, and its D, legitimately move away
        # from the FP64 oracle's; there D is held to the singular values below)
        ref = O.rqrcp(A, b, 10, seed=9, pivot="ortho", power=q, diagonalize=True)
        progress(f"  max |D - D_oracle| / |A| = {np.max(np.abs(d - np.diag(ref['F']))) / nA:.2e}")
        assert np.max(np.abs(d - np.diag(ref["F"]))) <= 1e-5 * nA
    res = _as_result(Fz, m, n, b)
    res["F"] = Fz.F.double().cpu().numpy()
    Rg = np.triu(res["F"])
    for r0, bi in res["blocks"]:
        blk = Rg[r0:r0 + bi, r0:r0 + bi]
        dd = np.diag(blk)
        assert np.all(blk - np.diag(dd) == 0.0)
        assert np.all(dd >= 0) and np.all(dd[:-1] >= dd[1:])
    Q, P = O.form_q(res, m), O.form_p(res)
    resid = np.linalg.norm(Q.T @ A @ P - Rg) / nA
    progress(f"  |Q^T A P - R| / |A| = {resid:.2e}")
    assert resid <= 1e-5
    # Q from reflectors stored in FP32 (with T and U' in FP64): the FP32-storage
    # bar of every other test; P from the FP64 S blocks and V': the FP64 bar
    assert np.linalg.norm(Q.T @ Q - np.eye(m)) <= 1e-4
    assert np.linalg.norm(P.T @ P - np.eye(n)) <= _orth_bar(n, b)
    s_ = np.linalg.svd(A, compute_uv=False)
    ratio = np.abs(np.log(d / s_))
    progress(f"  median |log(D/sigma)| = {np.median(ratio):.2e}")
    # 0.003-0.009 at q = 1; 0.09 at q = 2, where the FP32 power steps blur the
    # blocks' weak directions (see above)
    assert np.median(ratio) <= (0.1 if q == 1 else 0.15)
