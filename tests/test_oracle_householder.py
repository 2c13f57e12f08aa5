"""Pins of the oracle's Householder reflector (Section 3.1), QR (3.2), QRCP (3.3) and WY form (5.1)."""
import os

import numpy as np
import pytest
import scipy.linalg as sla

from oracle import rqrcp as O

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
U = np.finfo(np.float64).eps / 2


def _vec(s):
    return np.array([float(x) for x in s.split(",")])


def _golden_householder():
    rows = []
    for line in open(os.path.join(GOLDEN, "householder_examples.txt")):
        if line.startswith("#") or not line.strip():
            continue
        a, beta, v, tau = (x.strip() for x in line.split("|"))
        rows.append((_vec(a), float(beta), _vec(v), float(tau)))
    return rows


@pytest.mark.parametrize("a,beta,v,tau", _golden_householder())
def test_householder_hand_worked_examples(a, beta, v, tau):
    gv, gt, gb = O.householder(a)
    assert gb == pytest.approx(beta, abs=1e-15)
    np.testing.assert_allclose(gv, v, atol=1e-15)
    assert gt == pytest.approx(tau, abs=1e-15)


@pytest.mark.parametrize("seed", range(6))
def test_reflector_maps_a_to_beta_e1(seed):
    rng = np.random.default_rng(seed)
    a = rng.standard_normal(7 + seed) * 10.0 ** rng.integers(-5, 5)
    v, tau, beta = O.householder(a)
    H = np.eye(a.size) - tau * np.outer(v, v)
    Ha = H @ a
    na = np.linalg.norm(a)
    assert abs(Ha[0] - beta) <= 8 * U * na
    assert np.all(np.abs(Ha[1:]) <= 8 * U * na)
    assert abs(abs(beta) - na) <= 4 * U * na
    np.testing.assert_allclose(H @ H.T, np.eye(a.size), atol=16 * U)
    np.testing.assert_allclose(H, H.T, atol=0)
    # the paper's normalised form H = I - 2 w w^T, w = (beta e1 - a)/|beta e1 - a|
    w = -a.copy()
    w[0] += beta
    w /= np.linalg.norm(w)
    np.testing.assert_allclose(H, np.eye(a.size) - 2 * np.outer(w, w), atol=16 * U)


def _sign_normalise(R):
    d = np.sign(np.diag(R))
    d[d == 0] = 1
    return d[:, None] * R


@pytest.mark.parametrize("m,n", [(9, 5), (40, 40), (64, 17)])
def test_unpivoted_qr_matches_lapack_geqrf(m, n):
    rng = np.random.default_rng(m * n)
    A = rng.standard_normal((m, n))
    F = A.copy()
    tau = O.householder_qr(F)
    R = np.triu(F[: min(m, n)])
    Rl = sla.qr(A, mode="r")[0][: min(m, n)]
    np.testing.assert_allclose(_sign_normalise(R), _sign_normalise(Rl), atol=64 * U * np.linalg.norm(A))
    V = O.unit_lower(F, m, min(m, n))
    T = O.wy_T(V, tau)
    Q = (np.eye(m) - V @ T @ V.T)[:, : min(m, n)]
    np.testing.assert_allclose(Q.T @ Q, np.eye(min(m, n)), atol=64 * U * n)
    np.testing.assert_allclose(Q @ R, A, atol=64 * U * np.linalg.norm(A))


def test_unpivoted_r_is_cholesky_factor_of_gram():
    rng = np.random.default_rng(5)
    A = rng.standard_normal((50, 12))
    F = A.copy()
    O.householder_qr(F)
    L = np.linalg.cholesky(A.T @ A)
    np.testing.assert_allclose(np.abs(np.diag(F)), np.diag(L), rtol=1e-12)
    np.testing.assert_allclose(_sign_normalise(np.triu(F[:12])), L.T, atol=1e-12)


def test_wy_form_equals_product_of_reflectors():
    rng = np.random.default_rng(1)
    m, k = 13, 6
    F = rng.standard_normal((m, k))
    tau = O.householder_qr(F)
    V = O.unit_lower(F, m, k)
    T = O.wy_T(V, tau)
    P = np.eye(m)
    for j in range(k):
        P = P @ (np.eye(m) - tau[j] * np.outer(V[:, j], V[:, j]))
    np.testing.assert_allclose(np.eye(m) - V @ T @ V.T, P, atol=32 * U)
    assert np.all(np.tril(T, -1) == 0)


def test_qrcp_hand_worked_orthogonal_columns():
    spec = {}
    for line in open(os.path.join(GOLDEN, "qrcp_orthogonal_columns.txt")):
        if line.startswith("#") or "=" not in line:
            continue
        key, val = (x.strip() for x in line.split("=", 1))
        spec[key] = val
    A = np.array([[float(x) for x in row.split(",")] for row in spec["A"].split(";")])
    F = A.copy()
    piv, jpvt, tau, _ = O.qrcp(F)
    assert list(piv) == [int(x) for x in spec["piv"].split(",")]
    assert list(jpvt) == [int(x) for x in spec["jpvt"].split(",")]
    np.testing.assert_allclose(np.abs(np.diag(F)), [float(x) for x in spec["absdiagR"].split(",")], rtol=1e-15)
    R = np.triu(F[:3])
    np.testing.assert_allclose(R - np.diag(np.diag(R)), 0, atol=1e-15)


@pytest.mark.parametrize("seed", range(5))
def test_qrcp_pivots_match_lapack_geqp3(seed):
    rng = np.random.default_rng(100 + seed)
    m, n = 30 + seed, 20
    A = rng.standard_normal((m, n)) * np.logspace(0, -3, n)[None, rng.permutation(n)]
    F = A.copy()
    _, jpvt, _, margins = O.qrcp(F, record_margins=True)
    _, _, P = sla.qr(A, pivoting=True)
    # every decision is well separated for these inputs, so the orders agree
    assert margins[: n - 1].min() > 1e-6
    assert list(jpvt) == list(P)


def _brute_force_greedy(A, steps):
    chosen = []
    n = A.shape[1]
    for _ in range(steps):
        best, bestc = -1.0, None
        for c in range(n):
            if c in chosen:
                continue
            if chosen:
                B = A[:, chosen]
                coef = np.linalg.lstsq(B, A[:, c], rcond=None)[0]
                d = np.linalg.norm(A[:, c] - B @ coef)
            else:
                d = np.linalg.norm(A[:, c])
            if d > best:
                best, bestc = d, c
        chosen.append(bestc)
    return chosen


@pytest.mark.parametrize("seed", range(4))
def test_qrcp_equals_brute_force_greedy_volume(seed):
    rng = np.random.default_rng(200 + seed)
    A = rng.standard_normal((10, 9))
    F = A.copy()
    _, jpvt, _, _ = O.qrcp(F, steps=7)
    assert list(jpvt[:7]) == _brute_force_greedy(A, 7)


def test_qrcp_graded_orthogonal_closed_form():
    from workloads import graded_orthogonal
    A, order = graded_orthogonal(40, 24, seed=3)
    F = A.copy()
    _, jpvt, _, _ = O.qrcp(F)
    assert list(jpvt) == list(order)


def test_qrcp_ties_go_to_lowest_position_and_zero_columns():
    A = np.zeros((6, 5))
    A[:, 3] = [0, 0, 1, 0, 0, 0]
    F = A.copy()
    piv, jpvt, tau, margins = O.qrcp(F, record_margins=True)
    assert jpvt[0] == 3
    assert list(piv[1:]) == [1, 2, 3, 4]      # all remaining norms zero -> lowest position
    assert np.all(tau[1:] == 0) and margins[1] == 0
