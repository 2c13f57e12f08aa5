"""Helpers shared by the GPU parity tests (not collected by pytest)."""
import os
import sys
import time

import numpy as np

U = np.finfo(np.float64).eps / 2

# A pivot decision of the oracle is "separated" when its top-two margin
# (nu_1^2 - nu_2^2)/nu_1^2 exceeds what rounding differences between two FP64
# implementations can cause.  Those differences are absolute: a few u |A| in
# the trailing matrix X_i, hence about u (|A|/|X_i|) |Y_i| in the sketch Y_i
# and in every residual norm nu computed from it.  Relative to the leading
# residual norm nu_1 of the step, that is u (|A|/|X_i|) (|Y_i|/nu_1); the
# threshold is NOISE times that.  Late steps whose residuals are at roundoff
# level (e.g. past the rank of an exactly rank-deficient input) are therefore
# never counted as separated.
NOISE = 1.0e4


def separated_prefix(res, noise=NOISE):
    """Number of leading pivot positions fixed by separated decisions."""
    if not res["margins"]:
        return 0
    nA = res["xnorm"][0]
    pm, pt = res.get("pmargins", []), res.get("ptops", [])
    for i, ((r0, bi), mg, xn, yn, tops) in enumerate(zip(res["blocks"], res["margins"], res["xnorm"], res["ynorm"],
                                                          res["tops"])):
        for j in range(bi):
            delta = noise * U * (nA / max(xn, 1e-300)) * (yn / max(tops[j], 1e-300))
            if not (mg[j] > delta):
                # with the in-block pivot P-hat a column chosen differently
                # may land anywhere in the block
                return r0 + j if i >= len(pm) else r0
        if i < len(pm):
            # P-hat: QRCP of the panel, whose residual norms carry absolute
            # differences of a few u |A|
            for j in range(bi):
                if not (pm[i][j] > noise * U * nA / max(pt[i][j], 1e-300)):
                    return r0 + j
    return res["rank"]


def first_mismatch(a, b):
    """Index of the first differing entry of two equal-length sequences, or -1."""
    a, b = np.asarray(a), np.asarray(b)
    d = np.nonzero(a != b)[0]
    return int(d[0]) if d.size else -1


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


_T0 = time.time()


def progress(msg):
    """Flush a timestamped step line to stderr and to gpurun_out/progress.log."""
    line = f"[{time.time() - _T0:8.1f}s] {msg}"
    print(line, file=sys.stderr, flush=True)
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    out = os.path.join(root, "gpurun_out")
    if os.path.isdir(out):
        with open(os.path.join(out, "progress.log"), "a") as f:
            f.write(line + "\n")
