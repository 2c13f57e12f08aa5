"""Pins of the oracle's power iteration (Section 6.3): the sample of block i
is G_i X_i (X_i^T X_i)^q.  Checked against the closed form through the SVD
of X_i (G_i U diag(s^(2q+1)) V^T), against the factorization invariants, and
against the experiments' findings of Section 7 (hardly any gain for the
permutation form, a fast gain for the Householder form)."""
import numpy as np
import pytest

import workloads as W
from oracle import rqrcp as O
from tests import section7 as S7

U = np.finfo(np.float64).eps / 2


def _svd_sample(G, X, q):
    u, s, vt = np.linalg.svd(X, full_matrices=False)
    return (G @ u) * s ** (2 * q + 1) @ vt


@pytest.mark.parametrize("pivot", ["perm", "ortho"])
@pytest.mark.parametrize("q", [1, 2])
def test_sample_is_the_svd_closed_form_in_every_block(pivot, q):
    m, n, b, p, seed = 60, 44, 8, 4, 3
    A = W.make_matrix(m, n, W.sigma_geometric(n, 2.0), seed=5).numpy()
    res = O.rqrcp(A, b, p, seed=seed, pivot=pivot, power=q, trace=True)
    # block 0 samples A itself; block 1 samples the trailing matrix left by
    # block 0, which a run stopped after block 0 leaves in F(b:, b:)
    X1 = O.rqrcp(A, b, p, seed=seed, pivot=pivot, power=q, rank=b)["F"][b:, b:]
    for i, X in ((0, A), (1, X1)):
        G = O.sketch(seed, i, b + p, i * b, m - i * b)
        want = _svd_sample(G, X, q)
        got = res["Y"][i]
        assert got.shape == want.shape
        assert np.linalg.norm(got - want) <= 1e-12 * np.linalg.norm(want)


def test_power_zero_is_the_plain_sketch():
    A = W.make_matrix(50, 40, W.sigma_geometric(40, 3.0), seed=2).numpy()
    r0 = O.rqrcp(A, 8, 3, seed=4)
    r1 = O.rqrcp(A, 8, 3, seed=4, power=0)
    assert np.array_equal(r0["F"], r1["F"]) and np.array_equal(r0["jpvt"], r1["jpvt"])


@pytest.mark.parametrize("pivot", ["perm", "ortho"])
def test_factorisation_invariants_hold_with_the_power_iteration(pivot):
    m, n, b = 90, 70, 16
    A = W.make_matrix(m, n, W.sigma_geometric(n, 8.0), seed=9).numpy()
    res = O.rqrcp(A, b, b, seed=2, pivot=pivot, power=2)
    Q, R, P = O.form_q(res, n), np.triu(res["F"])[:n], O.form_p(res)
    assert np.linalg.norm(A @ P - Q @ R) / np.linalg.norm(A) <= 10 * n * U
    assert np.linalg.norm(Q.T @ Q - np.eye(n)) <= 10 * n * U
    assert np.linalg.norm(P.T @ P - np.eye(n)) <= 10 * n * U


@pytest.mark.parametrize("name,make", [("fast", S7.a_fast), ("gauss", S7.a_gauss)])
def test_section_7_power_method_findings(name, make):
    A = make(1)

    def gm(pivot, q):
        e = S7.errors_from_r(O.rqrcp(A, S7.B, 0, seed=1, pivot=pivot, power=q)["F"])
        s = S7.summary(e, A)
        assert s["to_svd_min"] >= 1.0 - 1e-12   # nothing beats Eckart-Young
        return s["to_svd_geomean"]

    m1 = [gm("perm", q) for q in (0, 1, 2)]
    m2 = [gm("ortho", q) for q in (0, 1, 2)]
    # permutation form: almost no improvement, still far above the optimum
    assert min(m1[1:]) >= 0.9 * m1[0] and min(m1) >= 1.4
    # Householder form: rapid improvement towards the optimum
    assert m2[1] <= 0.9 * m2[0] and m2[2] <= m2[1] and m2[2] <= 1.1
