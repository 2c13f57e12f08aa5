"""Pins of the oracle's counter-based Gaussian generator (sketch matrices, Section 4.1)."""
import numpy as np
import pytest
from scipy import stats

from oracle import philox


@pytest.mark.parametrize("ctr,key", [
    ((1, 0, 0, 0), (0, 0)),
    ((5, 7, 9, 11), (123, 456)),
    ((2**64 - 1, 3, 2**63, 17), (2**64 - 5, 99)),
    ((12345, 266, 31, 0), (6, 1)),
])
def test_philox_words_match_numpy_philox(ctr, key):
    # numpy's Philox (Philox4x64-10) increments its counter before each block of 4 words
    c0 = (ctr[0] - 1) % 2**64
    bg = np.random.Philox(counter=np.array([c0, ctr[1], ctr[2], ctr[3]], dtype=np.uint64),
                         key=np.array(key, dtype=np.uint64))
    want = [int(x) for x in bg.random_raw(4)]
    got = [int(x) for x in philox.philox4x64_10(*[np.uint64(c) for c in ctr], np.uint64(key[0]), np.uint64(key[1]))]
    assert got == want


def test_philox_vectorised_equals_scalar():
    g = np.arange(100, 140, dtype=np.uint64)
    words = philox.philox4x64_10(g, np.uint64(3), np.uint64(2), np.uint64(0), np.uint64(9), np.uint64(1))
    for t in range(0, 40, 7):
        one = philox.philox4x64_10(g[t], np.uint64(3), np.uint64(2), np.uint64(0), np.uint64(9), np.uint64(1))
        assert [int(w[t]) for w in words] == [int(x) for x in one]


def test_uniform_open_interval_endpoints():
    u = philox.uniform_open01(np.array([0, 2**64 - 1], dtype=np.uint64))
    assert u[0] == 2.0 ** -53
    assert u[1] == 1.0 - 2.0 ** -53
    assert np.all((u > 0) & (u < 1))


def test_sketch_is_standard_normal():
    G = philox.sketch_block(seed=11, block=3, nsample=200, row0=0, nrows=2000)
    z = G.ravel()
    n = z.size
    assert abs(z.mean()) < 5.0 / np.sqrt(n)
    assert abs(z.var() - 1.0) < 5.0 * np.sqrt(2.0 / n)
    assert stats.kstest(z, "norm").pvalue > 1e-4


def test_sketch_entries_depend_only_on_their_counter():
    G = philox.sketch_block(seed=2, block=1, nsample=12, row0=100, nrows=50)
    Gsub = philox.sketch_block(seed=2, block=1, nsample=5, row0=120, nrows=10)
    np.testing.assert_array_equal(G[:5, 20:30], Gsub)
    Gother = philox.sketch_block(seed=2, block=2, nsample=12, row0=100, nrows=50)
    assert np.all(G != Gother)


def _box_muller_cases():
    import os
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "box_muller_examples.txt")
    out = []
    for line in open(path):
        if line.startswith("#") or not line.strip():
            continue
        seed, tag, ctr, w0, w1, z = [f.strip() for f in line.split("|")]
        out.append((int(seed), int(tag), tuple(int(c) for c in ctr.split(",")), int(w0), int(w1), float(z)))
    return out


@pytest.mark.parametrize("seed,tag,ctr,w0,w1,z", _box_muller_cases())
def test_sketch_entries_match_known_answers(seed, tag, ctr, w0, w1, z):
    # words from numpy's Philox, normals from a 50-digit decimal evaluation of
    # Box-Muller (tests/golden/make_box_muller.py): pins the uniform map and
    # the transform (a wrong shift, constant, or cos/sin swap fails here)
    got_w = philox.philox4x64_10(*[np.uint64(c) for c in ctr], np.uint64(seed), np.uint64(tag))
    assert [int(got_w[0]), int(got_w[1])] == [w0, w1]
    got = float(philox.normal_from_counter(*[np.uint64(c) for c in ctr], seed, tag))
    assert abs(got - z) <= 4 * np.spacing(abs(z)), (got, z)
    if tag == philox.TAG_SKETCH and ctr[3] == 0:
        # the same entry of the block sketch: counter (g, r, i, 0)
        g, r, i = ctr[0], ctr[1], ctr[2]
        G = philox.sketch_block(seed, i, r + 1, g, 1)
        assert abs(G[r, 0] - z) <= 4 * np.spacing(abs(z))
