"""Counter-based Gaussian generator for the sketch matrices Omega / G.

TEST INFRASTRUCTURE ONLY: this module is part of the CPU oracle. Only tests,
the smoke check and the benchmark's CPU-baseline leg may import it.

The paper draws a Gaussian test matrix Omega (m x b, or m x (b+r) with
oversampling) for every pivot-block selection (Section 4.1, eq. defY;
Section 4.3).  It does not say how the random numbers are produced.  So that
the GPU path and this oracle can be driven by the *same* G without sharing
code, both sides implement one published, counter-based generator from its
definition:

* Philox4x64-10 (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as
  easy as 1, 2, 3", SC'11): a 4 x 64-bit counter, a 2 x 64-bit key, ten
  rounds of two 64x64->128-bit multiplies, with a Weyl key schedule.
* One uniform per 64-bit word: u = (floor(w / 2^12) + 1/2) * 2^-52, in (0,1);
  every step of this map is exact in FP64.
* Box-Muller: z = sqrt(-2 ln u1) * cos(2 pi u2) from words 0 and 1 of one
  counter, so every entry depends only on its own counter.

Entry (r, g) of the block-i sketch G_i (sample row r, global row g of A) uses
counter (g, r, i, 0) and key (seed, tag).  Tag 1 is the sketch.
"""
import numpy as np

M0 = np.uint64(0xD2E7470EE14C6C93)
M1 = np.uint64(0xCA5A826395121157)
W0 = np.uint64(0x9E3779B97F4A7C15)
W1 = np.uint64(0xBB67AE8584CAA73B)
_LO32 = np.uint64(0xFFFFFFFF)
_S32 = np.uint64(32)

TAG_SKETCH = 1


def _mulhilo(a, b):
    """Full 128-bit product of uint64 arrays: returns (high word, low word)."""
    a = np.asarray(a, dtype=np.uint64)
    b = np.asarray(b, dtype=np.uint64)
    al, ah = a & _LO32, a >> _S32
    bl, bh = b & _LO32, b >> _S32
    p0 = al * bl
    p1 = al * bh
    p2 = ah * bl
    p3 = ah * bh
    mid = (p0 >> _S32) + (p1 & _LO32) + (p2 & _LO32)
    hi = p3 + (p1 >> _S32) + (p2 >> _S32) + (mid >> _S32)
    lo = a * b
    return hi, lo


def philox4x64_10(c0, c1, c2, c3, k0, k1):
    """Philox4x64 with 10 rounds on broadcastable uint64 arrays.

    Returns the four output words.  Round: (hi0, lo0) = M0*c0, (hi1, lo1) =
    M1*c2, new counter = (hi1^c1^k0, lo1, hi0^c3^k1, lo0); the key is bumped
    by the Weyl constants between rounds.
    """
    with np.errstate(over="ignore"):
        c0, c1, c2, c3 = (np.asarray(x, dtype=np.uint64) for x in (c0, c1, c2, c3))
        k0 = np.asarray(k0, dtype=np.uint64)
        k1 = np.asarray(k1, dtype=np.uint64)
        for rnd in range(10):
            if rnd > 0:
                k0 = k0 + W0
                k1 = k1 + W1
            hi0, lo0 = _mulhilo(M0, c0)
            hi1, lo1 = _mulhilo(M1, c2)
            c0, c1, c2, c3 = hi1 ^ c1 ^ k0, lo1, hi0 ^ c3 ^ k1, lo0
    return c0, c1, c2, c3


def uniform_open01(w):
    """Map a uint64 word to a double in (0, 1): (w >> 12) + 1/2, times 2^-52."""
    w = np.asarray(w, dtype=np.uint64)
    return ((w >> np.uint64(12)).astype(np.float64) + 0.5) * (2.0 ** -52)


def normal_from_counter(c0, c1, c2, c3, seed, tag):
    """One standard normal per counter by Box-Muller on output words 0 and 1."""
    w0, w1, _, _ = philox4x64_10(c0, c1, c2, c3, np.uint64(seed), np.uint64(tag))
    u1 = uniform_open01(w0)
    u2 = uniform_open01(w1)
    return np.sqrt(-2.0 * np.log(u1)) * np.cos(2.0 * np.pi * u2)


def sketch_block(seed, block, nsample, row0, nrows):
    """G_i of size nsample x nrows: entry (r, g - row0) for g in [row0, row0+nrows).

    This is the Gaussian test matrix of block `block` (0-based), transposed
    to the orientation G = Omega^T used by Y = G X (Section 4.1, eq. defY).
    """
    r = np.arange(nsample, dtype=np.uint64)[:, None]
    g = np.arange(row0, row0 + nrows, dtype=np.uint64)[None, :]
    return normal_from_counter(g, r, np.uint64(block), np.uint64(0), seed, TAG_SKETCH)
