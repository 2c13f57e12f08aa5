"""Section 7 (f3) on the GPU path: Methods 1 and 2 (permutation and
Householder pivoting, no oversampling, b = 50) on the experiments' two
synthetic 300 x 300 matrices, through the C ABI.  The same bounds as the
oracle's test, and the truncation errors e_k = |R(k:, k:)|_F next to the
oracle's (same seed, hence the same sketches)."""
import numpy as np
import pytest
import torch

import paper_1505_08115_amd as R
from oracle import rqrcp as O
from tests import section7 as S7

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("name,make", [("fast", S7.a_fast), ("gauss", S7.a_gauss)])
def test_gpu_methods_1_and_2_reproduce_the_section_7_findings(name, make):
    A = make(1)
    A_dev = torch.tensor(A, device="cuda")
    out = {}
    for pivot in ("perm", "ortho"):
        Fz = R.factor(A_dev, block=S7.B, oversample=0, seed=1, pivot=pivot)
        torch.cuda.synchronize()
        e_gpu = S7.errors_from_r(Fz.F.cpu().numpy())
        e_ref = S7.errors_from_r(O.rqrcp(A, S7.B, 0, seed=1, pivot=pivot)["F"])
        np.testing.assert_allclose(e_gpu, e_ref, rtol=1e-6, atol=0)
        out[pivot] = S7.summary(e_gpu, A)
    m1, m2 = out["perm"], out["ortho"]
    assert m1["to_cpqr_median"] <= 1.15 and m1["to_cpqr_max"] <= 1.4
    assert m1["to_svd_geomean"] >= 1.4
    assert m2["to_svd_geomean"] <= 1.5 and m2["to_svd_geomean"] <= 0.8 * m1["to_svd_geomean"]
    assert m1["to_svd_min"] >= 1.0 - 1e-12 and m2["to_svd_min"] >= 1.0 - 1e-12


@pytest.mark.parametrize("name,make", [("fast", S7.a_fast), ("gauss", S7.a_gauss)])
def test_gpu_power_method_brings_method_2_to_the_optimum(name, make):
    """Section 6.3 on Method 2: q = 2 steps of the power iteration."""
    A = make(1)
    Fz = R.factor(torch.tensor(A, device="cuda"), block=S7.B, oversample=0, seed=1, pivot="ortho", power=2)
    torch.cuda.synchronize()
    e_gpu = S7.errors_from_r(Fz.F.cpu().numpy())
    e_ref = S7.errors_from_r(O.rqrcp(A, S7.B, 0, seed=1, pivot="ortho", power=2)["F"])
    np.testing.assert_allclose(e_gpu, e_ref, rtol=1e-6, atol=0)
    s = S7.summary(e_gpu, A)
    assert s["to_svd_geomean"] <= 1.1 and s["to_svd_min"] >= 1.0 - 1e-12
