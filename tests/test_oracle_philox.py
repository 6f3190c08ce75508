"""Pins of the oracle's counter-based noise (CPU only).

The generator is pinned to numpy's own Philox bit generator (an independent
implementation of the same published definition) and to the published
known-answer vectors; the normal transform to the Box-Muller identities and the
N(0, 1) law; the coupled coarse noise to the restriction of eq. ml-linsys.
"""
import math
import os

import numpy as np
import pytest
from scipy import stats as st

from oracle import noise as N
from oracle import philox as P

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "philox4x64_10_kat.txt")


def kat_vectors():
    out = []
    for line in open(GOLDEN):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        w = [int(x, 16) for x in line.split()]
        out.append((tuple(w[:4]), tuple(w[4:6]), tuple(w[6:])))
    return out


@pytest.mark.parametrize("ctr,key,want", kat_vectors())
def test_known_answer_vectors(ctr, key, want):
    assert P.philox4x64(ctr, key) == want


@pytest.mark.parametrize("key,ctr", [((0, 0), (0, 0, 0, 0)),
                                     ((12345, 678), (5, 0, 0, 0)),
                                     ((2 ** 64 - 1, 3), (2 ** 64 - 1, 7, 0, 0)),
                                     ((0xDEADBEEF, 2 ** 63 + 11), (1 << 40, 128, 3, 9))])
def test_matches_numpy_bit_generator(key, ctr):
    """numpy's Philox bit generator emits the block of counter + 1 first (the
    counter is a 256-bit integer whose lowest word comes first)."""
    c = sum(int(v) << (64 * i) for i, v in enumerate(ctr))
    prev = c - 1 if c > 0 else (1 << 256) - 1
    words = np.array([(prev >> (64 * i)) & P.MASK64 for i in range(4)], dtype=np.uint64)
    bg = np.random.Philox(key=np.array(key, dtype=np.uint64), counter=words)
    raw = [int(v) for v in bg.random_raw(8)]
    assert tuple(raw[:4]) == P.philox4x64(ctr, key)
    nxt = c + 1
    ctr2 = tuple((nxt >> (64 * i)) & P.MASK64 for i in range(4))
    assert tuple(raw[4:]) == P.philox4x64(ctr2, key)


def test_vectorised_matches_scalar_definition():
    rng = np.random.default_rng(5)
    c0 = rng.integers(0, 2 ** 63, size=64, dtype=np.uint64) * np.uint64(2) + np.uint64(1)
    key = (0x0123456789ABCDEF, 0xFEDCBA9876543210)
    x = P.philox4x64_batch(c0, 77, key)
    for i in range(c0.size):
        assert tuple(int(a[i]) for a in x) == P.philox4x64((int(c0[i]), 77, 0, 0), key)


def test_box_muller_identities():
    """z_a^2 + z_b^2 = -2 ln u and atan2(z_b, z_a) = 2 pi t (mod 2 pi)."""
    rng = np.random.default_rng(6)
    xa = rng.integers(0, 2 ** 64, size=4000, dtype=np.uint64, endpoint=False)
    xb = rng.integers(0, 2 ** 64, size=4000, dtype=np.uint64, endpoint=False)
    za, zb = P.box_muller(xa, xb)
    u = ((xa >> np.uint64(11)).astype(np.float64) + 1.0) / 2.0 ** 53
    t = (xb >> np.uint64(11)).astype(np.float64) / 2.0 ** 53
    np.testing.assert_allclose(za ** 2 + zb ** 2, -2.0 * np.log(u), rtol=1e-13, atol=1e-15)
    ang = np.mod(np.arctan2(zb, za), 2 * np.pi)
    d = np.abs(ang - 2 * np.pi * t)
    d = np.minimum(d, 2 * np.pi - d)
    r = np.sqrt(za ** 2 + zb ** 2)
    assert np.all(d[r > 1e-3] < 1e-12)


def test_extreme_words():
    """u = 1 (all-ones word) gives r = 0; u = 2^-53 (zero word) stays finite."""
    za, zb = P.box_muller(np.array([2 ** 64 - 1, 0], dtype=np.uint64), np.array([0, 0], dtype=np.uint64))
    assert za[0] == 0.0 and zb[0] == 0.0
    assert za[1] == pytest.approx(math.sqrt(2 * 53 * math.log(2)), rel=1e-14) and zb[1] == 0.0


def test_noise_is_standard_normal():
    xi = P.noise(32, seed=2024, event=3)
    assert xi.shape == (32 ** 3,)
    n = xi.size
    assert abs(xi.mean()) < 4.0 / math.sqrt(n)
    assert abs(xi.var() - 1.0) < 4.0 * math.sqrt(2.0 / n)
    assert st.kstest(xi, "norm").pvalue > 1e-3
    # the four lanes of one call and neighbouring cells are uncorrelated
    for lag in (1, 2, 3, 4, 32, 32 * 32):
        r = np.corrcoef(xi[:-lag], xi[lag:])[0, 1]
        assert abs(r) < 4.0 / math.sqrt(n)


def test_events_seeds_and_grids_are_independent():
    a = P.noise(16, 7, 0)
    for b in (P.noise(16, 7, 1), P.noise(16, 8, 0), P.noise(32, 7, 0)[: 16 ** 3]):
        assert abs(np.corrcoef(a, b)[0, 1]) < 4.0 / math.sqrt(a.size)
    np.testing.assert_array_equal(a, P.noise(16, 7, 0))     # a pure function of its key


def test_cell_spot_check_matches_field():
    xi = P.noise(8, 99, 5)
    for c in (0, 1, 2, 3, 4, 77, 511):
        assert P.noise_cell(8, 99, 5, c) == xi[c]


def test_coupled_noise_is_restriction_and_normal():
    xc = P.noise_coupled(16, 11, 4)
    np.testing.assert_array_equal(xc, N.restrict(32, P.noise(32, 11, 4)))
    assert st.kstest(xc, "norm").pvalue > 1e-3
    assert abs(xc.var() - 1.0) < 4.0 * math.sqrt(2.0 / xc.size)


def test_batch_is_consecutive_events():
    xb = P.noise_batch(8, 3, 10, 3)
    for b in range(3):
        np.testing.assert_array_equal(xb[b], P.noise(8, 3, 10 + b))
