"""Philox4x32-10 counter-based random numbers (oracle side).

Definition: Salmon, Moraes, Dror & Shaw, "Parallel Random Numbers: As Easy as
1, 2, 3", SC'11, Sec. 3 (the Philox-4x32 bijection, 10 rounds).  The paper being
reproduced names no generator (its stochastic model only needs independent
Poisson draws per pixel and isochrone point, Sec. 2.1); a counter-based
generator makes every draw a pure function of (seed, pixel, entry, purpose), so
any implementation and any launch shape produce the same stars.

Pinned by the published known-answer vectors of the Random123 distribution
(tests/golden/philox4x32_10_kat.txt) and by uniformity tests.
"""
from __future__ import annotations

import numpy as np

M0 = 0xD2511F53
M1 = 0xCD9E8D57
W0 = 0x9E3779B9
W1 = 0xBB67AE85
MASK32 = 0xFFFFFFFF

# Purpose tags: counter word c2 tells the streams apart.
TAG_MAIN = 0      # (pixel, entry // 4, 0, 0): one 32-bit word per entry for inversion
TAG_SPLIT = 1     # (pixel, entry // 4, 1, 0): dust split, first word of entry i
TAG_SPLIT_X = 2   # (pixel, entry, 2, j): dust split, further words
TAG_PTRS = 3      # (pixel, entry, 3, j): transformed rejection, attempts 2j and 2j+1
TAG_DUST = 4      # (pixel, 0, 4, 0): per-pixel log-normal dust draw
TAG_NOISE = 5     # (pixel, band, 5, 0): per-pixel, per-band photometric noise
# block-skip sampler (a separate stream; Sec. 2.1 footnote on Poisson superposition)
TAG_BLOCK = 6       # (pixel, block, 6, 0): word 0 draws the block's star total by inversion
TAG_BLOCK_PTRS = 7  # (pixel, block, 7, j): the total by transformed rejection, attempts 2j, 2j+1
TAG_STAR = 8        # (pixel, block, 8, s // 4): word s % 4 places star s on a point
TAG_STAR_SPLIT = 9  # (pixel, block, 9, s // 4): word s % 4 decides whether star s is reddened
TAG_RED = 10        # (pixel, entry // 4, 10, 0): word entry % 4 draws a thinned entry's reddened count
TAG_PTRS_RED = 11   # (pixel, entry, 11, j): that count by transformed rejection, attempts 2j, 2j+1


def philox4x32_10(c0, c1, c2, c3, seed: int):
    """Apply the 10-round Philox-4x32 bijection to counters (c0, c1, c2, c3)
    (array-likes of uint32, broadcast together) under the 64-bit key `seed`
    (k0 = low 32 bits, k1 = high 32 bits).  Returns four uint32 arrays."""
    x0, x1, x2, x3 = (np.asarray(c, dtype=np.uint64) & np.uint64(MASK32) for c in (c0, c1, c2, c3))
    x0, x1, x2, x3 = np.broadcast_arrays(x0, x1, x2, x3)
    k0 = int(seed) & MASK32
    k1 = (int(seed) >> 32) & MASK32
    m0 = np.uint64(M0)
    m1 = np.uint64(M1)
    s32 = np.uint64(32)
    lo_mask = np.uint64(MASK32)
    for r in range(10):
        p0 = m0 * x0                     # exact: 32 x 32 -> 64 bits
        p1 = m1 * x2
        hi0, lo0 = p0 >> s32, p0 & lo_mask
        hi1, lo1 = p1 >> s32, p1 & lo_mask
        x0, x1, x2, x3 = (hi1 ^ x1 ^ np.uint64(k0), lo1, hi0 ^ x3 ^ np.uint64(k1), lo0)
        k0 = (k0 + W0) & MASK32
        k1 = (k1 + W1) & MASK32
    return tuple(v.astype(np.uint32) for v in (x0, x1, x2, x3))


def u01_open_f64(w):
    """32-bit word -> uniform in (0, 1): (w + 1/2) * 2^-32, exact in FP64."""
    return (np.asarray(w, dtype=np.float64) + 0.5) * (2.0 ** -32)


def u01_open_f32(w):
    """32-bit word -> uniform in (0, 1) with 24 significant bits:
    ((w >> 9) + 1/2) * 2^-23, exact in FP32."""
    w = np.asarray(w, dtype=np.uint32)
    return ((w >> np.uint32(9)).astype(np.float32) + np.float32(0.5)) * np.float32(2.0 ** -23)


def box_muller_f64(w0, w1):
    """Standard normal from two words: sqrt(-2 ln u1) cos(2 pi u2), FP64."""
    u1 = u01_open_f64(w0)
    u2 = u01_open_f64(w1)
    return np.sqrt(-2.0 * np.log(u1)) * np.cos(2.0 * np.pi * u2)
