"""Helpers shared by the GPU parity tests (not collected by pytest)."""
import numpy as np

U = np.finfo(np.float64).eps / 2

# A pivot decision of the oracle is "separated" when its top-two margin
# (nu_1^2 - nu_2^2)/nu_1^2 exceeds the relative perturbation that rounding
# differences between two FP64 implementations can cause in that block's
# sketch.  That perturbation is taken as NOISE * u * |A|_F / |X_i|_F: errors
# of earlier blocks are absolute (a few u |A|) while X_i shrinks.
NOISE = 1.0e4


def separated_prefix(res, noise=NOISE):
    """Number of leading pivot positions fixed by separated decisions."""
    if not res["margins"]:
        return 0
    nA = res["xnorm"][0]
    for (r0, bi), mg, xn in zip(res["blocks"], res["margins"], res["xnorm"]):
        delta = noise * U * nA / max(xn, 1e-300)
        for j in range(bi):
            if not (mg[j] > delta):
                return r0 + j
    return res["F"].shape[1]


def min_margin(res):
    return float(min(np.min(m) for m in res["margins"])) if res["margins"] else float("inf")


def r_times_pt(F, jpvt, rows):
    """Row-sign-normalised R(0:rows, :) P^T: independent of where later
    pivots put the remaining columns."""
    n = F.shape[1]
    R = sign_rows(np.triu(F[:rows]))
    out = np.zeros((rows, n))
    out[:, jpvt] = R
    return out


def sign_rows(R):
    d = np.sign(np.diag(R[:, : R.shape[0]])) if R.shape[0] <= R.shape[1] else np.sign(np.diag(R))
    d = np.where(d == 0, 1.0, d)
    return d[:, None] * R
