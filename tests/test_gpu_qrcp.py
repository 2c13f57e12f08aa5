"""GPU pivoted QR (Section 3.3, Fig. 2) at exact ties spread over workgroups.

The kernel takes most pivot decisions inside a pool of published candidates
and goes back to a grid-wide exchange only when a column outside the pool
could be as large, so ties between columns owned by different workgroups are
the delicate case.  A scaled permutation matrix (A(:, c) = d_c e_{pi(c)} with
small integer d_c) keeps every residual norm exactly |d_c| through every
reflector of the classical process (each reflector only swaps and negates
rows), so every decision is an exact tie or exactly separated and the whole
pivot sequence is fixed: ties go to the lowest current position (Section
3.3's rule with the oracle's tie convention).  One block with b = n makes the
factorization the classical QRCP of the whole matrix (the last block of
Fig. 3), run by the same kernel as the pivoted QR of a sketch.
"""
import numpy as np
import pytest
import torch

import paper_1505_08115_amd as R
from oracle import rqrcp as O
from tests.parity import progress

pytestmark = pytest.mark.gpu
DEV = "cuda"


def scaled_permutation(m, n, seed, levels=5):
    rng = np.random.default_rng(seed)
    d = 1.0 + (np.arange(n) * 7) % levels          # each value repeated across the column range
    rows = rng.permutation(m)[:n]
    A = np.zeros((m, n))
    A[rows, np.arange(n)] = d * rng.choice([-1.0, 1.0], n)
    return A


@pytest.mark.parametrize("m,n,levels", [(300, 280, 5), (320, 320, 3), (150, 130, 40), (200, 190, 1)])
def test_exact_ties_across_workgroups(m, n, levels):
    A = scaled_permutation(m, n, seed=m + n, levels=levels)
    progress(f"scaled permutation {m} x {n}, {levels} distinct norms")
    Fz = R.factor(torch.tensor(A, device=DEV), block=n, oversample=0, seed=1)
    assert Fz.check() == [0, 0, 0, 0]
    _, jpvt, _, _ = O.qrcp(A.copy())
    jg = Fz.jpvt.cpu().numpy()
    bad = np.nonzero(jg != jpvt)[0]
    assert bad.size == 0, f"pivots differ first at position {bad[0]}: GPU {jg[bad[0]]}, oracle {jpvt[bad[0]]}"
    # the diagonal of R is the sorted norms, exactly
    d = np.abs(np.diag(Fz.F.cpu().numpy()))
    assert np.array_equal(d, np.sort(np.abs(A).max(axis=0))[::-1])
