"""Seeded state order sigma_t of one sweep of the mini-batch operator.

The paper analyses the operator with the states processed in ascending order
and notes that one may first assign random indexes to the states and process
them in that order, re-randomised at every iteration (Sec. III-A); its
experiments shuffle the states before every operator evaluation (Sec. IV-A)
and the theory holds when states are drawn uniformly without replacement
(Sec. V).  The paper does not fix a generator, so this library defines one
(the same definition is implemented independently by the GPU library):

* ``h = half_bits(n)`` is the smallest h >= 1 with 4**h >= n; the Feistel
  domain is [0, 4**h).
* One Feistel encryption of x in that domain splits x into L = x >> h and
  R = x & (2**h - 1) and runs four rounds j = 0..3 of
  ``(L, R) <- (R, L ^ F_j(R))`` with the round function

      F_j(R) = word0(Philox-4x32-10(counter=(R, j, t_lo, t_hi),
                                    key=(seed_lo, seed_hi))) & (2**h - 1)

  where t is the sweep index and seed the 64-bit permutation seed, both split
  into 32-bit halves.  The result is (L << h) | R.  A Feistel network is a
  bijection of the domain whatever its round function (Luby & Rackoff 1988).
* Cycle walking (Black & Rogaway 2002) restricts it to [0, n): sigma_t(p) is
  the first value in E(p), E(E(p)), ... that is below n.  This is a bijection
  of [0, n) because the walk follows the cycle of E through p.

sigma_t(p) is the state processed at position p of sweep t; batch k holds the
positions k*b .. min((k+1)*b, n) - 1 (eq. (10): each batch is a block of b
consecutive positions in processing order, the last one possibly shorter).

Test infrastructure only (see the package docstring).
"""

import numpy as np

from .philox import philox4x32_10

FEISTEL_ROUNDS = 4


def half_bits(n):
    """Smallest h >= 1 such that the Feistel domain 4**h holds n positions."""
    if n < 1:
        raise ValueError("n must be >= 1")
    h = 1
    while (1 << (2 * h)) < n:
        h += 1
    return h


def feistel_encrypt(x, h, seed, t):
    """One encryption E of the values ``x`` (array) in the domain [0, 4**h)."""
    x = np.asarray(x, dtype=np.uint64)
    mask = np.uint64((1 << h) - 1)
    hh = np.uint64(h)
    seed = int(seed) & ((1 << 64) - 1)
    t = int(t) & ((1 << 64) - 1)
    s_lo, s_hi = seed & 0xFFFFFFFF, seed >> 32
    t_lo, t_hi = t & 0xFFFFFFFF, t >> 32
    left = x >> hh
    right = x & mask
    for j in range(FEISTEL_ROUNDS):
        f = philox4x32_10(right, j, t_lo, t_hi, s_lo, s_hi)[0] & mask
        left, right = right, left ^ f
    return (left << hh) | right


def sweep_permutation(n, seed, t):
    """sigma_t as an int64 array: entry p is the state at position p."""
    h = half_bits(n)
    pos = np.arange(n, dtype=np.uint64)
    y = feistel_encrypt(pos, h, seed, t)
    out_of_range = y >= np.uint64(n)
    while out_of_range.any():
        y[out_of_range] = feistel_encrypt(y[out_of_range], h, seed, t)
        out_of_range = y >= np.uint64(n)
    return y.astype(np.int64)
