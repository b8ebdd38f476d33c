"""Gaussian random projection P (the paper's random projection matrix).

TEST INFRASTRUCTURE ONLY (see the package header).

The paper draws a random projection matrix P of size N x l once per
decomposition (section "Randomized matrix decompositions") and does not name
its distribution. Reading taken here: i.i.d. standard normal entries, drawn
from a counter-based generator so that an independent implementation can
reproduce every entry from (seed, channel, row, column) alone.

Generator: Philox4x64 with 10 rounds (Salmon, Moraes, Dror, Shaw, "Parallel
random numbers: as easy as 1, 2, 3", SC'11). One call maps a 4-word counter
and a 2-word key to four 64-bit words. Each round multiplies counter words 0
and 2 by two fixed odd constants into 128-bit products and recombines the
high and low halves with the other two words and the key; the key is bumped
by two Weyl constants between rounds.

Entry Omega[i, j] (0 <= i < n, 0 <= j < l) takes the Philox block with
counter (i, j // 4, 0, 0) and key (seed, channel), giving words r0..r3, and
applies the Box-Muller transform to the pairs (r0, r1) and (r2, r3):
    u1 = ((r >> 11) + 1) * 2^-53  in (0, 1]
    u2 = (r' >> 11) * 2^-53       in [0, 1)
    z  = sqrt(-2 ln u1) * cos(2 pi u2),   z' = sqrt(-2 ln u1) * sin(2 pi u2)
Omega[i, j] is z0, z1, z2, z3 for j mod 4 = 0, 1, 2, 3. A column never
depends on l, so growing l only appends columns.

Pins: the raw blocks equal numpy's own Philox4x64-10 (numpy advances its
counter before each block, so its block c+1 is ours at counter c); the normal
deviates are checked by moments and a Kolmogorov-Smirnov test.
"""

import numpy as np

# Philox4x64 constants (Salmon et al. 2011): round multipliers and the key
# schedule's Weyl increments (golden ratio and sqrt(3) - 1, as 64-bit fractions).
PHILOX_M0 = np.uint64(0xD2E7470EE14C6C93)
PHILOX_M1 = np.uint64(0xCA5A826395121157)
PHILOX_W0 = np.uint64(0x9E3779B97F4A7C15)
PHILOX_W1 = np.uint64(0xBB67AE8584CAA73B)
PHILOX_ROUNDS = 10

_LO32 = np.uint64(0xFFFFFFFF)
_SH32 = np.uint64(32)


def _mulhilo64(a, b):
    """Return (high, low) 64-bit halves of the 128-bit product a * b."""
    a = np.asarray(a, dtype=np.uint64)
    b = np.asarray(b, dtype=np.uint64)
    a_lo, a_hi = a & _LO32, a >> _SH32
    b_lo, b_hi = b & _LO32, b >> _SH32
    ll = a_lo * b_lo
    lh = a_lo * b_hi
    hl = a_hi * b_lo
    hh = a_hi * b_hi
    mid = (ll >> _SH32) + (lh & _LO32) + (hl & _LO32)
    hi = hh + (lh >> _SH32) + (hl >> _SH32) + (mid >> _SH32)
    return hi, a * b


def philox4x64_10(ctr, key):
    """Philox4x64-10 block function.

    ctr: sequence of 4 uint64 arrays (broadcastable), key: 2 uint64 arrays.
    Returns a list of 4 uint64 arrays.
    """
    c0, c1, c2, c3 = (np.asarray(x, dtype=np.uint64) for x in ctr)
    k0, k1 = (np.asarray(x, dtype=np.uint64) for x in key)
    with np.errstate(over="ignore"):
        for r in range(PHILOX_ROUNDS):
            if r > 0:
                k0 = k0 + PHILOX_W0
                k1 = k1 + PHILOX_W1
            hi0, lo0 = _mulhilo64(PHILOX_M0, c0)
            hi1, lo1 = _mulhilo64(PHILOX_M1, c2)
            c0, c1, c2, c3 = hi1 ^ c1 ^ k0, lo1, hi0 ^ c3 ^ k1, lo0
    return [c0, c1, c2, c3]


def box_muller(r_a, r_b):
    """Two 64-bit words -> two independent N(0,1) deviates (FP64)."""
    u1 = ((np.asarray(r_a, np.uint64) >> np.uint64(11)).astype(np.float64) + 1.0) * 2.0 ** -53
    u2 = (np.asarray(r_b, np.uint64) >> np.uint64(11)).astype(np.float64) * 2.0 ** -53
    rad = np.sqrt(-2.0 * np.log(u1))
    ang = (2.0 * np.pi) * u2
    return rad * np.cos(ang), rad * np.sin(ang)


def gaussian_omega(n, l, seed, channel=0, col0=0):
    """Omega (n x l, row-major FP64), columns col0 .. col0+l-1 of the stream."""
    n = int(n)
    l = int(l)
    out = np.empty((n, l), dtype=np.float64)
    if n == 0 or l == 0:
        return out
    cols = np.arange(col0, col0 + l, dtype=np.int64)
    blocks = np.unique(cols // 4)
    rows = np.arange(n, dtype=np.uint64)[:, None]
    r = philox4x64_10(
        (rows, blocks.astype(np.uint64)[None, :], np.uint64(0), np.uint64(0)),
        (np.uint64(seed), np.uint64(channel)),
    )
    z0, z1 = box_muller(r[0], r[1])
    z2, z3 = box_muller(r[2], r[3])
    z = np.stack([z0, z1, z2, z3], axis=-1).reshape(n, -1)  # columns 4*b0 ..
    base = int(blocks[0]) * 4
    out[:, :] = z[:, cols - base]
    return out
