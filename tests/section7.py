"""Truncation errors of Section 7's experiments (shared by the oracle and GPU
tests): e_k = |A - A_k|_F = |R(k:, k:)|_F for a full factorization A P =
Q R (the identity of Section 5's truncation), next to the optimum of the
truncated SVD (Eckart-Young) and to classical column-pivoted QR (LAPACK
geqp3 through scipy)."""
import numpy as np
import scipy.linalg as sla

import workloads as W

N, B = 300, 50   # the experiments' size and block size


def a_fast(seed):
    """U diag(s) V^T, U and V Haar, s_j = (1e-5)^((j-1)/(n-1))."""
    return W.make_matrix(N, N, W.sigma_geometric(N, 5.0), seed=seed).numpy()


def a_gauss(seed):
    """i.i.d. N(0, 1/n) entries."""
    return np.random.default_rng(seed).standard_normal((N, N)) / np.sqrt(N)


def errors_from_r(R):
    """e_k for k = 0 .. n-1 from the upper triangle of R (n x n)."""
    R = np.triu(np.asarray(R, dtype=np.float64)[:N, :N])
    sq = R ** 2
    # |R(k:, k:)|_F^2 = sum over rows i >= k of sum_{j >= i} R_ij^2
    rows = sq.sum(axis=1)
    return np.sqrt(np.cumsum(rows[::-1])[::-1])


def errors_svd(A):
    s = np.linalg.svd(A, compute_uv=False)
    return np.sqrt(np.cumsum((s ** 2)[::-1])[::-1])


def errors_cpqr(A):
    _, R, _ = sla.qr(A, pivoting=True, mode="economic")
    return errors_from_r(R)


def summary(e_method, A):
    """Ratios over k = 1 .. n-2 (e_0 = |A|_F for every method)."""
    ks = np.arange(1, N - 1)
    es, ec = errors_svd(A)[ks], errors_cpqr(A)[ks]
    em = e_method[ks]
    return {"to_cpqr_median": float(np.median(em / ec)), "to_cpqr_max": float(np.max(em / ec)),
            "to_svd_geomean": float(np.exp(np.mean(np.log(em / es)))), "to_svd_min": float(np.min(em / es)),
            "cpqr_to_svd_geomean": float(np.exp(np.mean(np.log(ec / es))))}
