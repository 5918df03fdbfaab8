"""Philox4x64-10 and the Box-Muller normal transform, in plain numpy.

Test infrastructure (see the package docstring).  The paper draws its test
matrix with randn() (Section II-A, notation; the sketch of Section III-A) and does
not fix a generator.  Reading used here: a counter-based generator so that
every entry of the n x d sketch matrix is a function of (seed, index) alone.

Philox4x64-10 is the block function published by Salmon, Moraes, Dror and
Shaw, "Parallel random numbers: as easy as 1, 2, 3" (SC'11): a 4-word
counter and a 2-word key go through ten rounds; each round multiplies two
counter words by fixed odd constants, keeps the high and low halves of the
128-bit products, mixes them with the other two words and the key, and the
key is advanced by two Weyl increments between rounds.

Pinned by: tests/test_oracle_philox.py checks the block function against
numpy's independent Philox bit generator (same published algorithm) on many
keys and counters, and the normal transform against moments, a KS test and
closed-form special cases.
"""

import numpy as np

_M32 = np.uint64(0xFFFFFFFF)
_S32 = np.uint64(32)

# Round multipliers and Weyl key increments of Philox4x64 (Salmon et al.).
PHILOX_M0 = np.uint64(0xD2E7470EE14C6C93)
PHILOX_M1 = np.uint64(0xCA5A826395121157)
PHILOX_W0 = np.uint64(0x9E3779B97F4A7C15)
PHILOX_W1 = np.uint64(0xBB67AE8584CAA73B)

# Second key word of the sketch stream: ASCII "RQLP".
SKETCH_KEY1 = 0x52514C50


def _mulhilo(a, b):
    """(high, low) 64-bit halves of the 128-bit product a*b, elementwise."""
    a = np.asarray(a, dtype=np.uint64)
    b = np.uint64(b)
    a_lo, a_hi = a & _M32, a >> _S32
    b_lo, b_hi = b & _M32, b >> _S32
    p_ll = a_lo * b_lo
    p_lh = a_lo * b_hi
    p_hl = a_hi * b_lo
    p_hh = a_hi * b_hi
    mid = (p_ll >> _S32) + (p_lh & _M32) + (p_hl & _M32)
    hi = p_hh + (p_lh >> _S32) + (p_hl >> _S32) + (mid >> _S32)
    with np.errstate(over="ignore"):
        lo = a * b
    return hi, lo


def philox4x64_10(ctr, key):
    """Apply the ten-round Philox4x64 block function.

    ctr: uint64 array of shape (..., 4); key: pair of ints.
    Returns a uint64 array of shape (..., 4).
    """
    ctr = np.asarray(ctr, dtype=np.uint64)
    x0, x1, x2, x3 = (ctr[..., i].copy() for i in range(4))
    k0 = np.uint64(key[0] & 0xFFFFFFFFFFFFFFFF)
    k1 = np.uint64(key[1] & 0xFFFFFFFFFFFFFFFF)
    with np.errstate(over="ignore"):
        for r in range(10):
            if r > 0:
                k0 = np.uint64((int(k0) + int(PHILOX_W0)) & 0xFFFFFFFFFFFFFFFF)
                k1 = np.uint64((int(k1) + int(PHILOX_W1)) & 0xFFFFFFFFFFFFFFFF)
            hi0, lo0 = _mulhilo(x0, PHILOX_M0)
            hi1, lo1 = _mulhilo(x2, PHILOX_M1)
            x0, x1, x2, x3 = hi1 ^ x1 ^ k0, lo1, hi0 ^ x3 ^ k1, lo0
    return np.stack([x0, x1, x2, x3], axis=-1)


def uniform_pair(w0, w1):
    """Map two 64-bit words to (u1, u2) with u1 in (0, 1] and u2 in [0, 1).

    Each uses the top 53 bits, so both are exact doubles.
    """
    scale = 2.0 ** -53
    u1 = ((np.asarray(w0, np.uint64) >> np.uint64(11)).astype(np.float64) + 1.0) * scale
    u2 = (np.asarray(w1, np.uint64) >> np.uint64(11)).astype(np.float64) * scale
    return u1, u2


def box_muller(u1, u2):
    """Box-Muller: two independent N(0,1) values from two uniforms."""
    r = np.sqrt(-2.0 * np.log(u1))
    t = (2.0 * np.pi) * u2
    return r * np.cos(t), r * np.sin(t)


def gaussian_matrix(seed, n, d, stream=0):
    """The n x d standard Gaussian sketch matrix, in float64.

    Entry (i, j) has logical index l = j*n + i.  Block c = l // 4 is the
    Philox output for counter (c, 0, 0, 0) under key (seed, 0x52514C50 +
    stream); its words (w0, w1) give the normals for l = 4c, 4c+1 and
    (w2, w3) those for l = 4c+2, 4c+3.
    """
    total = n * d
    nblocks = (total + 3) // 4
    ctr = np.zeros((nblocks, 4), dtype=np.uint64)
    ctr[:, 0] = np.arange(nblocks, dtype=np.uint64)
    words = philox4x64_10(ctr, (int(seed), SKETCH_KEY1 + int(stream)))
    u1a, u2a = uniform_pair(words[:, 0], words[:, 1])
    u1b, u2b = uniform_pair(words[:, 2], words[:, 3])
    z0, z1 = box_muller(u1a, u2a)
    z2, z3 = box_muller(u1b, u2b)
    flat = np.stack([z0, z1, z2, z3], axis=1).reshape(-1)[:total]
    # flat[l] with l = j*n + i  ->  column-major n x d
    return flat.reshape(d, n).T.copy()
