"""Writes box_muller_examples.txt: known-answer normals of the sketch generator.

For a few (seed, counter) pairs, the two Philox4x64-10 output words come from
numpy.random.Philox (an implementation independent of the oracle), the two
uniforms u = ((w >> 12) + 1/2) 2^-52 are exact, and z = sqrt(-2 ln u1)
cos(2 pi u2) (Box-Muller) is evaluated with Python's decimal module at 50
significant digits (its own ln and sqrt; cos by its Taylor series, pi by
Machin's formula), then rounded to 20 digits.  Run from the repository root:
python tests/golden/make_box_muller.py
"""
import os
from decimal import Decimal, getcontext

import numpy as np

getcontext().prec = 50
CASES = [  # (seed, tag, counter c0..c3): c0 = global row, c1 = sample row, c2 = block
    (0, 1, (0, 0, 0, 0)),
    (6, 1, (12345, 266, 31, 0)),
    (11, 1, (7, 3, 2, 0)),
    (2**63 + 5, 1, (5, 2, 7, 0)),
    (1, 1, (511, 39, 0, 0)),
]


def philox_words(seed, tag, ctr):
    # numpy's Philox adds 1 to its 256-bit counter (word 0 lowest) before
    # producing each block of 4 words: start it one below
    v = (sum(c << (64 * i) for i, c in enumerate(ctr)) - 1) % 2**256
    pre = [(v >> (64 * i)) & (2**64 - 1) for i in range(4)]
    bg = np.random.Philox(counter=np.array(pre, dtype=np.uint64),
                         key=np.array([seed, tag], dtype=np.uint64))
    return [int(x) for x in bg.random_raw(2)]


def atan_inv(x):
    """arctan(1/x) for an integer x > 1 by its series."""
    x = Decimal(x)
    term = 1 / x
    total, k, sign = term, 1, -1
    while True:
        term = term / (x * x)
        add = sign * term / (2 * k + 1)
        if add == 0 or abs(add) < Decimal(10) ** -60:
            break
        total += add
        k += 1
        sign = -sign
    return total


def cos(x):
    total, term, k = Decimal(1), Decimal(1), 0
    while True:
        k += 2
        term = -term * x * x / (k * (k - 1))
        if abs(term) < Decimal(10) ** -60:
            break
        total += term
    return total


def main():
    pi = 4 * (4 * atan_inv(5) - atan_inv(239))
    lines = ["# Known-answer normals of the sketch generator (Philox4x64-10 + Box-Muller); written by",
             "# tests/golden/make_box_muller.py from numpy.random.Philox words and a 50-digit decimal evaluation.",
             "# Columns: seed | tag | counter c0,c1,c2,c3 | word0 | word1 | z"]
    for seed, tag, ctr in CASES:
        w0, w1 = philox_words(seed, tag, ctr)
        u1 = (Decimal(w0 >> 12) + Decimal("0.5")) * Decimal(2) ** -52
        u2 = (Decimal(w1 >> 12) + Decimal("0.5")) * Decimal(2) ** -52
        z = (-2 * u1.ln()).sqrt() * cos(2 * pi * u2)
        lines.append(f"{seed} | {tag} | {','.join(str(c) for c in ctr)} | {w0} | {w1} | {z:.20e}")
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "box_muller_examples.txt")
    with open(path, "w") as f:
        f.write("\n".join(lines) + "\n")


if __name__ == "__main__":
    main()
