"""Section 7 (f3): the oracle's Methods 1 and 2 (Fig. 3 with permutation and
with Householder pivoting, no oversampling) on the two synthetic test
matrices of the experiments, against the truncated SVD and classical
column-pivoted QR.  The experiments' findings as bounds: Method 1 tracks
column-pivoted QR; both permutation methods stay well above the SVD optimum;
Method 2 comes much closer to it; no method beats the optimum."""
import pytest

from oracle import rqrcp as O
from tests import section7 as S7


@pytest.mark.parametrize("name,make", [("fast", S7.a_fast), ("gauss", S7.a_gauss)])
def test_methods_1_and_2_reproduce_the_section_7_findings(name, make):
    A = make(1)
    m1 = S7.summary(S7.errors_from_r(O.rqrcp(A, S7.B, 0, seed=1, pivot="perm")["F"]), A)
    m2 = S7.summary(S7.errors_from_r(O.rqrcp(A, S7.B, 0, seed=1, pivot="ortho")["F"]), A)
    assert m1["to_cpqr_median"] <= 1.15 and m1["to_cpqr_max"] <= 1.4
    assert m1["to_svd_geomean"] >= 1.4 and m1["cpqr_to_svd_geomean"] >= 1.4
    assert m2["to_svd_geomean"] <= 1.5 and m2["to_svd_geomean"] <= 0.8 * m1["to_svd_geomean"]
    assert m1["to_svd_min"] >= 1.0 - 1e-12 and m2["to_svd_min"] >= 1.0 - 1e-12
