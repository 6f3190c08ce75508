"""Counter-based white noise (oracle; test infrastructure).

The sampler's load is g W^{1/2} xi with xi ~ N(0, I) on the cells (eq. linsys).
The paper draws the coefficient vector with a parallel pseudo-random library on
the host (Sec. "Implementation details").  The device path can instead generate
xi where it is consumed, from a counter-based generator: a pure function of
(key, counter) that any thread can evaluate for any cell, so no noise is stored
or copied.

Generator: Philox4x64-10 (Salmon, Moraes, Dror, Shaw, "Parallel random numbers:
as easy as 1, 2, 3", SC 2011).  One call maps a 256-bit counter and a 128-bit
key to four 64-bit words through 10 rounds of

    (hi0, lo0) = M0 * c0,  (hi1, lo1) = M1 * c2        (full 128-bit products)
    c <- (hi1 ^ c1 ^ k0, lo1, hi0 ^ c3 ^ k1, lo0)

with the key advanced by the Weyl constants (W0, W1) before every round after
the first.

Normals: the four words of one call give two Box-Muller pairs,
    u = ((x_a >> 11) + 1) 2^-53  in (0, 1],   t = (x_b >> 11) 2^-53  in [0, 1),
    (z_a, z_b) = sqrt(-2 ln u) (cos 2 pi t, sin 2 pi t),
for (a, b) = (0, 1) and (2, 3).

Noise of one field: key = (seed, event), counter = (c >> 2, n, 0, 0) for the
cell c = i + n (j + n k) of the n^3 box, and xi[c] is normal (c & 3) of that
call.  The grid size in the counter keeps the fields of different grids
independent.  The coupled coarse field of an event (eq. ml-linsys) is the
restriction of the event's fine field (oracle.noise.restrict), not a field of
its own.

Pins (tests/test_oracle_philox.py): numpy's own Philox bit generator, the
generator's published known-answer vectors, the Box-Muller identities and the
normal law.
"""
from __future__ import annotations

import numpy as np

from . import noise as _noise

M0 = 0xD2E7470EE14C6C93
M1 = 0xCA5A826395121157
W0 = 0x9E3779B97F4A7C15
W1 = 0xBB67AE8584CAA73B
MASK64 = (1 << 64) - 1


def philox4x64(ctr, key, rounds: int = 10):
    """One Philox4x64 call with Python integers: 4 counter words, 2 key words."""
    x0, x1, x2, x3 = (int(v) & MASK64 for v in ctr)
    k0, k1 = (int(v) & MASK64 for v in key)
    for r in range(rounds):
        if r:
            k0 = (k0 + W0) & MASK64
            k1 = (k1 + W1) & MASK64
        p0 = M0 * x0
        p1 = M1 * x2
        x0, x1, x2, x3 = (p1 >> 64) ^ x1 ^ k0, p1 & MASK64, (p0 >> 64) ^ x3 ^ k1, p0 & MASK64
    return x0, x1, x2, x3


def _mulhilo(a: int, b: np.ndarray):
    """128-bit product of the constant a with every entry of b (uint64):
    schoolbook over 32-bit halves, all partial products exact in uint64."""
    m32 = np.uint64(0xFFFFFFFF)
    s32 = np.uint64(32)
    a0, a1 = np.uint64(a & 0xFFFFFFFF), np.uint64(a >> 32)
    b0, b1 = b & m32, b >> s32
    ll = a0 * b0
    lh = a0 * b1
    hl = a1 * b0
    hh = a1 * b1
    mid = (ll >> s32) + (lh & m32) + (hl & m32)          # < 3 * 2^32
    lo = (ll & m32) | ((mid & m32) << s32)
    hi = hh + (lh >> s32) + (hl >> s32) + (mid >> s32)
    return hi, lo


def philox4x64_batch(c0: np.ndarray, c1: int, key, rounds: int = 10):
    """Philox4x64 for the counters (c0[i], c1, 0, 0): four uint64 arrays."""
    with np.errstate(over="ignore"):
        x0 = np.asarray(c0, dtype=np.uint64).copy()
        x1 = np.full_like(x0, np.uint64(int(c1) & MASK64))
        x2 = np.zeros_like(x0)
        x3 = np.zeros_like(x0)
        k0, k1 = (int(v) & MASK64 for v in key)
        for r in range(rounds):
            if r:
                k0 = (k0 + W0) & MASK64
                k1 = (k1 + W1) & MASK64
            hi0, lo0 = _mulhilo(M0, x0)
            hi1, lo1 = _mulhilo(M1, x2)
            x0, x1, x2, x3 = hi1 ^ x1 ^ np.uint64(k0), lo1, hi0 ^ x3 ^ np.uint64(k1), lo0
    return x0, x1, x2, x3


def box_muller(xa: np.ndarray, xb: np.ndarray):
    """Two standard normals from two 64-bit words (see the module docstring)."""
    u = ((np.asarray(xa, dtype=np.uint64) >> np.uint64(11)).astype(np.float64) + 1.0) * 2.0 ** -53
    t = (np.asarray(xb, dtype=np.uint64) >> np.uint64(11)).astype(np.float64) * 2.0 ** -53
    r = np.sqrt(-2.0 * np.log(u))
    th = 2.0 * np.pi * t
    return r * np.cos(th), r * np.sin(th)


def noise(n: int, seed: int, event: int) -> np.ndarray:
    """xi of the n^3 box for one event (length n^3, cell order i + n (j + n k))."""
    if n < 4 or n % 4:
        raise ValueError("n must be a multiple of 4")
    nb = n ** 3 // 4
    x0, x1, x2, x3 = philox4x64_batch(np.arange(nb, dtype=np.uint64), n, (seed, event))
    za, zb = box_muller(x0, x1)
    zc, zd = box_muller(x2, x3)
    return np.stack([za, zb, zc, zd], axis=1).reshape(-1)


def noise_batch(n: int, seed: int, event0: int, batch: int) -> np.ndarray:
    """[batch][n^3]: events event0, event0 + 1, ..."""
    return np.stack([noise(n, seed, event0 + b) for b in range(batch)])


def noise_coupled(n: int, seed: int, event: int) -> np.ndarray:
    """Noise of the coarse n^3 sample coupled to the event's (2n)^3 field."""
    return _noise.restrict(2 * n, noise(2 * n, seed, event))


def noise_cell(n: int, seed: int, event: int, c: int) -> float:
    """xi[c] alone, through the scalar definition (spot checks at any size)."""
    x = philox4x64((c >> 2, n, 0, 0), (seed, event))
    pair, lane = divmod(c & 3, 2)
    za, zb = box_muller(np.array([x[2 * pair]], dtype=np.uint64), np.array([x[2 * pair + 1]], dtype=np.uint64))
    return float((za, zb)[lane][0])
