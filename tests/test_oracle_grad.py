"""Pins of the oracle's gradient of L = |A_k - B|_F^2 with fixed pivots, and of its Jacobi SVD."""
import numpy as np
import pytest
import torch

import workloads as W
from oracle import rqrcp as O


def _ak_fixed(A, jpvt, k):
    Q, _ = np.linalg.qr(A[:, jpvt[:k]])
    return Q @ (Q.T @ A)


def test_full_rank_gradient_is_the_upstream_gradient():
    n = 20
    A = W.make_matrix(n, n, W.sigma_geometric(n, 2.0), seed=1).numpy()
    B = W.gaussian_matrix(n, n, seed=2).numpy()
    res = O.rqrcp(A, 4, 2, seed=3)
    Gbar = 2 * (O.lowrank(res, n) - B)
    dA = O.lowrank_grad(A, res["jpvt"], n, Gbar)
    np.testing.assert_allclose(dA, Gbar, atol=1e-10)


@pytest.mark.parametrize("m,n,k", [(12, 9, 3), (15, 15, 5), (20, 11, 8)])
def test_gradient_matches_torch_autograd(m, n, k):
    A = W.make_matrix(m, n, W.sigma_geometric(n, 2.0), seed=m).numpy()
    B = W.gaussian_matrix(m, n, seed=n).numpy()
    res = O.rqrcp(A, 4, 2, seed=1, rank=k)
    jpvt = res["jpvt"]
    Gbar = 2 * (O.lowrank(res, k) - B)
    dA = O.lowrank_grad(A, jpvt, k, Gbar)
    At = torch.tensor(A, requires_grad=True)
    Q, _ = torch.linalg.qr(At[:, torch.as_tensor(jpvt[:k])])
    L = ((Q @ (Q.T @ At)) - torch.tensor(B)).pow(2).sum()
    L.backward()
    np.testing.assert_allclose(dA, At.grad.numpy(), atol=1e-9 * np.abs(dA).max())


def test_gradient_matches_central_differences():
    m, n, k = 10, 8, 3
    A = W.make_matrix(m, n, W.sigma_geometric(n, 1.0), seed=4).numpy()
    B = W.gaussian_matrix(m, n, seed=5).numpy()
    res = O.rqrcp(A, 4, 2, seed=2, rank=k)
    jpvt = res["jpvt"]
    dA = O.lowrank_grad(A, jpvt, k, 2 * (_ak_fixed(A, jpvt, k) - B))
    h = 1e-6
    rng = np.random.default_rng(0)
    for _ in range(6):
        E = rng.standard_normal((m, n))
        E /= np.linalg.norm(E)
        fp, fm = _ak_fixed(A + h * E, jpvt, k), _ak_fixed(A - h * E, jpvt, k)
        fd = np.sum((fp - fm) * (fp + fm - 2 * B)) / (2 * h)
        assert fd == pytest.approx(np.sum(dA * E), rel=1e-6, abs=1e-8)


@pytest.mark.parametrize("m,n", [(30, 30), (45, 20), (64, 64)])
def test_jacobi_singular_values_match_lapack(m, n):
    A = W.make_matrix(m, n, W.sigma_geometric(n, 10.0), seed=m + n).numpy()
    sv = O.jacobi_singular_values(A)
    ref = np.linalg.svd(A, compute_uv=False)
    np.testing.assert_allclose(sv, ref, rtol=0, atol=64 * np.finfo(float).eps * ref[0])


def test_jacobi_recovers_prescribed_spectrum():
    n = 40
    s = W.sigma_geometric(n, 3.0)
    A = W.make_matrix(n, n, s, seed=3).numpy()
    np.testing.assert_allclose(O.jacobi_singular_values(A), s, atol=1e-13)
