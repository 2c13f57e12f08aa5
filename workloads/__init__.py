"""Seeded synthetic input matrices shared by the tests and the benchmark.

This module holds none of the factorization's arithmetic: it only builds
inputs A = U diag(s) V^T with prescribed singular values, the structure of
the paper's test matrices (Section 7: A^fast has Haar U, V and a geometric
decay of the singular values), scaled to the workload sizes below.

U and V are Haar-distributed: the Q factor of a QR factorisation of an i.i.d.
N(0,1) matrix, with its columns multiplied by sign(diag R).  The Gaussians
come from a seeded torch CPU generator, so every machine draws the same
numbers; the QR and the product may run on a GPU for the large sizes, which
changes only the rounding of A.
"""
from dataclasses import dataclass, field

import numpy as np
import torch


def sigma_geometric(n, decades):
    """s_j = 10^(-decades (j-1)/(n-1)), j = 1..n."""
    if n == 1:
        return np.ones(1)
    j = np.arange(n, dtype=np.float64)
    return 10.0 ** (-decades * j / (n - 1))


def sigma_rank(n, k):
    """s_j = 1 for j <= k, 0 after: an exactly rank-k spectrum."""
    s = np.zeros(n)
    s[:k] = 1.0
    return s


def sigma_gap(n, gap_at, gap=1e-6):
    """Slow decay 1/j with a drop by `gap` after index gap_at (1-based)."""
    j = np.arange(1, n + 1, dtype=np.float64)
    s = 1.0 / j
    s[j > gap_at] *= gap
    return s


@dataclass(frozen=True)
class Workload:
    name: str
    m: int
    n: int
    b: int
    p: int
    pivot: str          # "perm" | "ortho"
    precision: str      # "f64" | "mixed" (FP32 storage, BF16 sketch)
    profile: tuple      # ("geom", decades) | ("rank", k) | ("gap", j, gap)
    seed: int
    rank: int = 0       # 0 = full factorization
    extra: dict = field(default_factory=dict, hash=False, compare=False)

    def sigma(self):
        kind = self.profile[0]
        if kind == "geom":
            return sigma_geometric(self.n, self.profile[1])
        if kind == "rank":
            return sigma_rank(self.n, self.profile[1])
        if kind == "gap":
            return sigma_gap(self.n, self.profile[1], self.profile[2])
        raise ValueError(kind)


WORKLOADS = {
    "C1": Workload("C1", 512, 512, 32, 8, "perm", "f64", ("geom", 8.0), 1),
    "C2": Workload("C2", 4096, 4096, 128, 10, "perm", "f64", ("geom", 12.0), 2),
    "C2r": Workload("C2r", 4096, 4096, 128, 10, "perm", "f64", ("rank", 1000), 21),
    "C3": Workload("C3", 8192, 8192, 256, 10, "ortho", "f64", ("gap", 2048, 1e-6), 3),
    "C3s": Workload("C3s", 1024, 1024, 256, 10, "ortho", "f64", ("gap", 256, 1e-6), 31),
    "H1": Workload("H1", 8192, 8192, 256, 10, "perm", "f64", ("geom", 6.0), 6),
    "H2": Workload("H2", 8192, 8192, 256, 16, "perm", "mixed", ("geom", 6.0), 6),
    "C4": Workload("C4", 16384, 8192, 256, 16, "perm", "mixed", ("geom", 6.0), 4),
    "C5": Workload("C5", 4096, 4096, 128, 10, "perm", "f64", ("geom", 4.0), 5, rank=256),
}


def _gaussian(rows, cols, seed, stream):
    g = torch.Generator(device="cpu")
    g.manual_seed(int(seed) * 1000003 + int(stream))
    return torch.randn(rows, cols, generator=g, dtype=torch.float64)


def haar(rows, cols, seed, stream, device="cpu"):
    """rows x cols matrix with Haar-distributed orthonormal columns."""
    X = _gaussian(rows, cols, seed, stream).to(device)
    Q, R = torch.linalg.qr(X, mode="reduced")
    d = torch.sign(torch.diagonal(R))
    d[d == 0] = 1.0
    return Q * d[None, :]


def make_matrix(m, n, s, seed, device="cpu"):
    """A = U diag(s) V^T (m x n, FP64), U m x n and V n x n Haar."""
    s = torch.as_tensor(np.asarray(s, dtype=np.float64), device=device)
    U = haar(m, n, seed, 1, device)
    V = haar(n, n, seed, 2, device)
    return (U * s[None, :]) @ V.T


def workload_matrix(w, device="cpu", m=None, n=None):
    """Input of a named workload (optionally resized, keeping its recipe)."""
    m = w.m if m is None else m
    n = w.n if n is None else n
    if (m, n) != (w.m, w.n):
        w = Workload(w.name, m, n, w.b, w.p, w.pivot, w.precision, w.profile, w.seed, w.rank)
    return make_matrix(m, n, w.sigma(), w.seed, device)


def gaussian_matrix(m, n, seed, stream=7, device="cpu"):
    """i.i.d. N(0,1) m x n (for B in the loss, and for A^gauss-like inputs)."""
    return _gaussian(m, n, seed, stream).to(device)


def integer_rank_k(m, n, k, seed, lo=-3, hi=3):
    """A = X1 X2^T with small-integer X1 (m x k), X2 (n x k): exact rank k,
    exactly representable in FP64."""
    rng = np.random.default_rng(seed)
    X1 = rng.integers(lo, hi + 1, size=(m, k)).astype(np.float64)
    X2 = rng.integers(lo, hi + 1, size=(n, k)).astype(np.float64)
    return X1 @ X2.T


def graded_orthogonal(m, n, seed, decades=10.0):
    """A = W diag(d) Pi_0: orthonormal W (m x n), geometric d, random
    column permutation Pi_0.  Returns (A, order) where order lists the
    columns of A by decreasing norm."""
    rng = np.random.default_rng(seed)
    W = haar(m, n, seed, 3).numpy()
    d = sigma_geometric(n, decades)
    perm = rng.permutation(n)
    A = np.empty((m, n))
    A[:, perm] = W * d[None, :]
    order = perm.copy()          # column perm[t] has norm d[t], d decreasing
    return A, order


def flops_normalised(m, n):
    """2 m n^2 - 2 n^3 / 3 (= 4/3 n^3 for m = n): Householder QR flops."""
    return 2.0 * m * n * n - 2.0 * n ** 3 / 3.0


def flops_normalised_prefix(m, n, c):
    """Householder-QR flop count of processing the first c columns:
    sum over t < c of 4 (m - t)(n - t), the leading-order count whose
    total over all n columns is flops_normalised(m, n)."""
    t = np.arange(c, dtype=np.float64)
    return float(np.sum(4.0 * (m - t) * (n - t)))

