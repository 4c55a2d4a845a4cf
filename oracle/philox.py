"""Philox4x32-10 counter-based generator, written from its published definition.

Reference: J. K. Salmon, M. A. Moraes, R. O. Dror, D. E. Shaw, "Parallel random
numbers: as easy as 1, 2, 3", SC'11 (the Philox-4x32 bijection with 10 rounds).

The paper draws exactly one random object, the Gaussian starting block of the
subspace iteration (Section 2.2.1, Algorithm "subspace iteration"; Section 2.5
states it is the only randomness).  The stochastic inner solver that the paper
invokes (Section 2.3, Theorem "svrgSolve") also samples columns of X.  Both
draws are keyed by a 64-bit seed and addressed by an explicit 128-bit counter so
that any element of any stream can be produced independently of the others.

Counter layout (four 32-bit words c0..c3):
  c0  element or draw index inside a step (row index for the Gaussian block)
  c1  step index t (column index for the Gaussian block)
  c2  epoch index e (0 for the Gaussian block)
  c3  (stream tag << 28) | solve index

Stream tags: 1 = estimate-phase starting block, 2 = shift-and-invert starting
block, 3 = inner-solver column samples.

Everything here is plain NumPy on uint64 arrays so that a 32x32 -> 64 bit
product is exact.
"""
import numpy as np

M0 = np.uint64(0xD2511F53)
M1 = np.uint64(0xCD9E8D57)
W0 = 0x9E3779B9
W1 = 0xBB67AE85
MASK32 = np.uint64(0xFFFFFFFF)

TAG_EST_INIT = 1
TAG_SI_INIT = 2
TAG_SAMPLES = 3


def philox4x32_10(c0, c1, c2, c3, k0, k1):
    """Apply the ten-round Philox-4x32 bijection to counters (c0, c1, c2, c3)
    under key (k0, k1).  Counter words may be arrays (broadcast together); the
    key words are Python ints.  Returns four uint64 arrays holding 32-bit words.
    """
    c0 = np.asarray(c0, dtype=np.uint64) & MASK32
    c1 = np.asarray(c1, dtype=np.uint64) & MASK32
    c2 = np.asarray(c2, dtype=np.uint64) & MASK32
    c3 = np.asarray(c3, dtype=np.uint64) & MASK32
    c0, c1, c2, c3 = np.broadcast_arrays(c0, c1, c2, c3)
    k0 = int(k0) & 0xFFFFFFFF
    k1 = int(k1) & 0xFFFFFFFF
    for r in range(10):
        if r > 0:
            k0 = (k0 + W0) & 0xFFFFFFFF
            k1 = (k1 + W1) & 0xFFFFFFFF
        p0 = M0 * c0
        p1 = M1 * c2
        hi0, lo0 = p0 >> np.uint64(32), p0 & MASK32
        hi1, lo1 = p1 >> np.uint64(32), p1 & MASK32
        c0, c1, c2, c3 = (hi1 ^ c1 ^ np.uint64(k0), lo1,
                          hi0 ^ c3 ^ np.uint64(k1), lo0)
    return c0, c1, c2, c3


def key_of(seed):
    """Split a 64-bit seed into the two 32-bit Philox key words (low, high)."""
    seed = int(seed) & 0xFFFFFFFFFFFFFFFF
    return seed & 0xFFFFFFFF, seed >> 32


def stream_word(tag, solve):
    """Fourth counter word: stream tag in the top four bits, solve index below."""
    if not (0 <= solve < (1 << 28)):
        raise ValueError("solve index out of range")
    return (int(tag) << 28) | int(solve)


def unit53(a, b):
    """Map two 32-bit words to a double in (0, 1): 53 bits (a:32, b>>11:21),
    offset by one half so that neither 0 nor 1 is produced."""
    a = np.asarray(a, dtype=np.uint64)
    b = np.asarray(b, dtype=np.uint64)
    v = (a << np.uint64(21)) | (b >> np.uint64(11))
    return (v.astype(np.float64) + 0.5) * (2.0 ** -53)


def gaussian_block(seed, tag, solve, d, p):
    """d x p block with N(0,1) entries: element (i, j) uses counter
    (i, j, 0, stream_word(tag, solve)) and the Box-Muller transform
    z = sqrt(-2 ln u1) cos(2 pi u2) with u1 from words (0,1) and u2 from (2,3).
    This is the random start S^(0) of the subspace iteration."""
    k0, k1 = key_of(seed)
    i = np.arange(d, dtype=np.uint64)[:, None]
    j = np.arange(p, dtype=np.uint64)[None, :]
    o0, o1, o2, o3 = philox4x32_10(i, j, 0, stream_word(tag, solve), k0, k1)
    u1 = unit53(o0, o1)
    u2 = unit53(o2, o3)
    return np.sqrt(-2.0 * np.log(u1)) * np.cos(2.0 * np.pi * u2)
