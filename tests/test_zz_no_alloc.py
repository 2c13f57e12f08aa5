"""The allocation-free entry point rqrcp_factor_noalloc (through the C ABI)
against rqrcp_factor on the same inputs: two calls in a row, the second on a
smaller problem (the library's device array keeps the first call's contents),
both identical to the workspace entry point bit for bit (the same kernels on
the same data, every reduction in a fixed order); a problem whose workspace
exceeds the array is refused before any launch."""
import numpy as np
import pytest
import torch

import paper_1505_08115_amd as R
import workloads as W

pytestmark = pytest.mark.gpu
DEV = "cuda"
ERR_WORKSPACE = 2


def _same(Fa, Fb):
    assert torch.equal(Fa.jpvt, Fb.jpvt)
    assert torch.equal(Fa.F, Fb.F)
    assert torch.equal(Fa.tau, Fb.tau)
    assert torch.equal(Fa.T, Fb.T)
    if Fa.S is not None:
        assert torch.equal(Fa.S, Fb.S)


@pytest.mark.parametrize("dtype,precision", [(torch.float64, "plain"), (torch.float32, "mixed")])
def test_noalloc_matches_the_workspace_entry_point(dtype, precision):
    cases = [(1024, 1000, 64, 8, "perm", 3), (600, 500, 32, 8, "perm", 4)]   # the second one smaller
    if dtype == torch.float64:
        cases.append((300, 260, 32, 6, "ortho", 5))
    for m, n, b, p, pivot, seed in cases:
        sizes = R.factor_sizes(m, n, dtype, block=b, oversample=p, pivot=pivot, precision=precision, seed=seed)
        assert sizes[3] <= R.NOALLOC_WORK_BYTES
        A = W.make_matrix(m, n, W.sigma_geometric(n, 6.0), seed=seed).to(DEV).to(dtype)
        Fa = R.factor(A, block=b, oversample=p, seed=seed, pivot=pivot, precision=precision)
        Fb = R.factor_noalloc(A, block=b, oversample=p, seed=seed, pivot=pivot, precision=precision)
        assert Fa.check() == [0, 0, 0, 0] and Fb.check() == [0, 0, 0, 0]
        _same(Fa, Fb)


def test_noalloc_refuses_a_workspace_beyond_its_array():
    m = n = 2048
    sizes = R.factor_sizes(m, n, torch.float64, block=128, oversample=10)
    assert sizes[3] > R.NOALLOC_WORK_BYTES
    A = torch.zeros(m, n, dtype=torch.float64, device=DEV)
    with pytest.raises(R.RqrcpError) as ei:
        R.factor_noalloc(A, block=128, oversample=10)
    assert ei.value.status == ERR_WORKSPACE
    assert "rqrcp_factor_noalloc has" in str(ei.value)
