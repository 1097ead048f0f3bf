"""Philox counter-based generator, written from its published definition.

Reference: J. K. Salmon, M. A. Moraes, R. O. Dror, D. E. Shaw, "Parallel random
numbers: as easy as 1, 2, 3", SC'11.  Philox-4xW-R maps a 4-word counter and a
2-word key to 4 output words through R rounds.  One round takes the counter
(x0, x1, x2, x3) and the round key (k0, k1) to

    (hi(M1*x2) ^ x1 ^ k0,  lo(M1*x2),  hi(M0*x0) ^ x3 ^ k1,  lo(M0*x0))

where hi/lo are the upper/lower W bits of the 2W-bit product.  Between rounds
the key is advanced by the Weyl constants (k0 += C0, k1 += C1); the first
round uses the key as given.

The sweep order of the mini-batch operator is drawn from Philox-4x32-10 (see
``permutation``).  The 4x64 variant is here only so that the round structure
can be checked against numpy's own Philox-4x64-10 implementation.

Test infrastructure only (see the package docstring).
"""

import numpy as np

_CONSTANTS = {
    32: dict(M=(0xD2511F53, 0xCD9E8D57), C=(0x9E3779B9, 0xBB67AE85)),
    64: dict(M=(0xD2E7470EE14C6C93, 0xCA5A826395121157),
             C=(0x9E3779B97F4A7C15, 0xBB67AE8584CAA73B)),
}


def philox_scalar(counter, key, width=32, rounds=10):
    """Philox-4x{width}-{rounds} on Python integers (slow, exact).

    ``counter`` is a 4-sequence and ``key`` a 2-sequence of unsigned integers
    below 2**width.  Returns the 4 output words as a list of ints.
    """
    consts = _CONSTANTS[width]
    mask = (1 << width) - 1
    x0, x1, x2, x3 = (int(v) & mask for v in counter)
    k0, k1 = (int(v) & mask for v in key)
    for r in range(rounds):
        if r > 0:
            k0 = (k0 + consts["C"][0]) & mask
            k1 = (k1 + consts["C"][1]) & mask
        p0 = consts["M"][0] * x0
        p1 = consts["M"][1] * x2
        x0, x1, x2, x3 = ((p1 >> width) ^ x1 ^ k0, p1 & mask,
                          (p0 >> width) ^ x3 ^ k1, p0 & mask)
    return [x0, x1, x2, x3]


def philox4x32_10(c0, c1, c2, c3, k0, k1):
    """Vectorised Philox-4x32-10.

    All arguments are numpy arrays (or scalars) of 32-bit values; they are
    broadcast together.  Products of two 32-bit words are formed exactly in
    uint64.  Returns the four output words as uint64 arrays holding 32-bit
    values.
    """
    mask = np.uint64(0xFFFFFFFF)
    shift = np.uint64(32)
    M0 = np.uint64(_CONSTANTS[32]["M"][0])
    M1 = np.uint64(_CONSTANTS[32]["M"][1])
    C0 = np.uint64(_CONSTANTS[32]["C"][0])
    C1 = np.uint64(_CONSTANTS[32]["C"][1])
    x0, x1, x2, x3, key0, key1 = np.broadcast_arrays(
        *(np.asarray(v, dtype=np.uint64) & mask for v in (c0, c1, c2, c3, k0, k1)))
    x0, x1, x2, x3 = x0.copy(), x1.copy(), x2.copy(), x3.copy()
    key0, key1 = key0.copy(), key1.copy()
    for r in range(10):
        if r > 0:
            key0 = (key0 + C0) & mask
            key1 = (key1 + C1) & mask
        p0 = M0 * x0
        p1 = M1 * x2
        x0, x1, x2, x3 = ((p1 >> shift) ^ x1 ^ key0, p1 & mask,
                          (p0 >> shift) ^ x3 ^ key1, p0 & mask)
    return x0, x1, x2, x3
