"""Philox4x32-10 counter-based generator, written from its published definition.

Test infrastructure only (see ``oracle/__init__.py``).

Reference: J. K. Salmon, M. A. Moraes, R. O. Dror, D. E. Shaw, "Parallel random
numbers: as easy as 1, 2, 3", SC'11, section on the Philox family.  One round maps
the counter (c0, c1, c2, c3) under key (k0, k1) to

    (hi(M1*c2) ^ c1 ^ k0,  lo(M1*c2),  hi(M0*c0) ^ c3 ^ k1,  lo(M0*c0))

with 32x32->64-bit products; between rounds the key is bumped by the Weyl
constants (W0, W1).  Ten rounds are used.

The paper draws its operators with ``std::minstd_rand`` (section "Results",
serial setup paragraph); a sequential LCG cannot be evaluated independently per
entry on a GPU, so this build replaces it with a counter-based generator whose
output for a given (counter, key) is fixed by the definition above.  The method
only needs independent uniform draws, which both generators supply.
"""
import numpy as np

M0 = 0xD2511F53
M1 = 0xCD9E8D57
W0 = 0x9E3779B9
W1 = 0xBB67AE85
_MASK = 0xFFFFFFFF


def philox4x32_10(c0, c1, c2, c3, key):
    """Evaluate Philox4x32-10 elementwise.

    c0..c3: integer arrays (broadcastable) holding 32-bit counter words.
    key: (k0, k1) python ints.
    Returns a tuple of four uint64 arrays, each holding a 32-bit output word.
    """
    u64 = np.uint64
    mask = u64(_MASK)
    x0 = np.asarray(c0, dtype=np.uint64) & mask
    x1 = np.asarray(c1, dtype=np.uint64) & mask
    x2 = np.asarray(c2, dtype=np.uint64) & mask
    x3 = np.asarray(c3, dtype=np.uint64) & mask
    x0, x1, x2, x3 = np.broadcast_arrays(x0, x1, x2, x3)
    k0 = int(key[0]) & _MASK
    k1 = int(key[1]) & _MASK
    for _ in range(10):
        p0 = u64(M0) * x0          # < 2^64: exact in uint64
        p1 = u64(M1) * x2
        hi0, lo0 = p0 >> u64(32), p0 & mask
        hi1, lo1 = p1 >> u64(32), p1 & mask
        x0, x1, x2, x3 = (hi1 ^ x1 ^ u64(k0), lo1, hi0 ^ x3 ^ u64(k1), lo0)
        k0 = (k0 + W0) & _MASK
        k1 = (k1 + W1) & _MASK
    return x0, x1, x2, x3


def key_from_seed(seed):
    """Split a 64-bit seed into the two 32-bit key words (low word first)."""
    seed = int(seed) & 0xFFFFFFFFFFFFFFFF
    return (seed & _MASK, seed >> 32)


def mulhi32(u, r):
    """floor(u * r / 2^32) for 32-bit u and 0 < r <= 2^32: a uniform draw from [0, r)."""
    return (np.asarray(u, dtype=np.uint64) * np.uint64(r)) >> np.uint64(32)
