"""Seeded synthetic MDP inputs.

This module only draws random MDPs; it contains none of the operator's
arithmetic.  The test suite, the smoke check and the benchmark all take their
inputs from here, so the GPU library and the CPU oracle always see the same
arrays.

Every array is drawn from numpy's Philox-4x64 generator keyed by
(seed, stream) with the counter set to the index of a fixed-size block of
states, so the result does not depend on how many threads generate it.

Shapes follow the paper's setting (Sec. II-A): transition row r = s*m + a.

* dense:  P [n, m, n] with rows ~ Dirichlet(alpha), c [n, m] ~ U[0, 1).
* CSR:    k distinct successor columns per row, sorted ascending, either
          uniform over all states or uniform in the clipped window
          [s - band, s + band]; weights ~ Dirichlet(alpha).

Rows are normalised in FP64 and then rounded to the storage dtype without
renormalising, so a stored FP32 row sums to 1 only up to rounding.
"""

import concurrent.futures as cf
import os

import numpy as np

_STREAM_P = 0
_STREAM_C = 1
_STREAM_COL = 2
_STREAM_VAL = 3
_STREAM_MISC = 4


def _rng(seed, stream, block):
    return np.random.Generator(
        np.random.Philox(key=[int(seed), int(stream)], counter=[int(block), 0, 0, 0]))


def _threads():
    return max(1, min(16, os.cpu_count() or 1))


def _parallel(fn, nblocks):
    if nblocks <= 1:
        for i in range(nblocks):
            fn(i)
        return
    with cf.ThreadPoolExecutor(_threads()) as ex:
        list(ex.map(fn, range(nblocks)))


def costs(n, m, seed, low=0.0, high=1.0, dtype=np.float32):
    """Stage costs c(s, a) ~ U[low, high)."""
    g = _rng(seed, _STREAM_C, 0)
    return (low + (high - low) * g.random((n, m))).astype(dtype)


def dense_dirichlet(n, m, alpha, seed, dtype=np.float32, block=64):
    """Dense transition tensor P[n, m, n] with each row ~ Dirichlet(alpha)."""
    P = np.empty((n, m, n), dtype=dtype)

    def fill(i):
        s0 = i * block
        s1 = min(n, s0 + block)
        g = _rng(seed, _STREAM_P, i)
        x = g.standard_gamma(alpha, size=(s1 - s0, m, n))
        tot = x.sum(axis=2, keepdims=True)
        empty = tot[..., 0] == 0.0
        if empty.any():  # every draw underflowed: fall back to a uniform row
            x[empty] = 1.0
            tot = x.sum(axis=2, keepdims=True)
        P[s0:s1] = (x / tot).astype(dtype)

    _parallel(fill, (n + block - 1) // block)
    return P


def dense_mdp(n, m, alpha, seed, dtype=np.float32):
    """(P, c) of a dense random MDP."""
    return dense_dirichlet(n, m, alpha, seed, dtype), costs(n, m, seed, dtype=dtype)


def _distinct_sorted(g, lo, width, k):
    """k distinct integers per row, uniform in [lo, lo + width), sorted.

    Duplicates are redrawn until none is left; by symmetry the resulting set
    is uniform over all k-subsets of the window."""
    rows = lo.shape[0]
    x = np.sort(lo[:, None] + np.floor(g.random((rows, k)) * width[:, None]).astype(np.int64), axis=1)
    while True:
        dup = np.zeros_like(x, dtype=bool)
        dup[:, 1:] = x[:, 1:] == x[:, :-1]
        if not dup.any():
            return x
        r, j = np.nonzero(dup)
        x[r, j] = lo[r] + np.floor(g.random(len(r)) * width[r]).astype(np.int64)
        x.sort(axis=1)


def csr_mdp(n, m, k, alpha, seed, band=None, val_dtype=np.float32, block=4096):
    """Sparse random MDP with exactly k successors per (s, a) row.

    band None: columns uniform over [0, n).  band w: columns uniform in
    [max(0, s - w), min(n - 1, s + w)].  Returns (row_ptr int64 [n*m + 1],
    col int32 [n*m*k], val [n*m*k], c float32 [n, m]).
    """
    if band is None and k > n:
        raise ValueError("k must not exceed n")
    if band is not None and k > min(n, band + 1):
        raise ValueError("window too small for k distinct columns")
    rows = n * m
    col = np.empty((rows, k), dtype=np.int32)
    val = np.empty((rows, k), dtype=val_dtype)

    def fill(i):
        s0 = i * block
        s1 = min(n, s0 + block)
        states = np.repeat(np.arange(s0, s1, dtype=np.int64), m)
        if band is None:
            lo = np.zeros_like(states)
            hi = np.full_like(states, n - 1)
        else:
            lo = np.maximum(0, states - band)
            hi = np.minimum(n - 1, states + band)
        gc = _rng(seed, _STREAM_COL, i)
        col[s0 * m:s1 * m] = _distinct_sorted(gc, lo, hi - lo + 1, k)
        gv = _rng(seed, _STREAM_VAL, i)
        w = gv.standard_gamma(alpha, size=(len(states), k))
        w /= w.sum(axis=1, keepdims=True)
        val[s0 * m:s1 * m] = w.astype(val_dtype)

    _parallel(fill, (n + block - 1) // block)
    row_ptr = np.arange(rows + 1, dtype=np.int64) * k
    return row_ptr, col.reshape(-1), val.reshape(-1), costs(n, m, seed)


def csr_ragged_mdp(n, m, k_min, k_max, alpha, seed, val_dtype=np.float32):
    """Sparse random MDP whose rows have between k_min and k_max distinct
    successors (uniform over [0, n)); k_min may be 0 to produce empty rows."""
    g = _rng(seed, _STREAM_MISC, 0)
    rows = n * m
    lengths = g.integers(k_min, k_max + 1, size=rows)
    row_ptr = np.concatenate(([0], np.cumsum(lengths))).astype(np.int64)
    col = np.empty(int(row_ptr[-1]), dtype=np.int32)
    val = np.empty(int(row_ptr[-1]), dtype=val_dtype)
    for r in range(rows):
        ln = int(lengths[r])
        if ln == 0:
            continue
        cols = np.sort(g.choice(n, size=ln, replace=False))
        w = g.standard_gamma(alpha, size=ln)
        col[row_ptr[r]:row_ptr[r + 1]] = cols
        val[row_ptr[r]:row_ptr[r + 1]] = (w / w.sum()).astype(val_dtype)
    return row_ptr, col, val, costs(n, m, seed)


def inadmissible(c, frac, seed):
    """Mark a fraction of (s, a) pairs as inadmissible (cost +inf), keeping
    at least one admissible action per state.  Returns a new array."""
    g = _rng(seed, _STREAM_MISC, 1)
    c = np.array(c, copy=True)
    n, m = c.shape
    mask = g.random((n, m)) < frac
    keep = g.integers(0, m, size=n)
    mask[np.arange(n), keep] = False
    c[mask] = np.inf
    return c


def multi_costs(n, m, r, seed, low=0.0, high=1.0, dtype=np.float32):
    """r cost vectors at once, C[s, a, j] ~ U[low, high), layout [n, m, r]."""
    g = _rng(seed, _STREAM_MISC, 3)
    return (low + (high - low) * g.random((n, m, r))).astype(dtype)


def values(n, seed, low=0.0, high=1.0, dtype=np.float32):
    """A random value vector V ~ U[low, high)."""
    g = _rng(seed, _STREAM_MISC, 2)
    return (low + (high - low) * g.random(n)).astype(dtype)


def policy(n, m, seed):
    """A random stationary policy, int32 [n]."""
    g = _rng(seed, _STREAM_MISC, 3)
    return g.integers(0, m, size=n).astype(np.int32)


# The workloads of the benchmark and the parity tests.  Data seed = workload
# index; permutation seed = 100 + workload index, shared by every batch size.
WORKLOADS = {
    "dense-64x4": dict(kind="dense", n=64, m=4, alpha=1.0, gamma=0.9,
                       data_seed=1, perm_seed=101, batch_sizes=(16,),
                       tol_dv=1e-8, p_dtype="float64"),
    "dense-8192x16": dict(kind="dense", n=8192, m=16, alpha=0.1, gamma=0.99,
                          data_seed=2, perm_seed=102,
                          batch_sizes=(256, 1024, 8192), K=5, eps=1e-6),
    "csr-1M-banded": dict(kind="csr", n=1_000_000, m=8, k=32, band=512, alpha=1.0,
                          gamma=0.995, data_seed=3, perm_seed=103,
                          batch_sizes=(4096, 65536, 1_000_000)),
    "csr-1M-uniform": dict(kind="csr", n=1_000_000, m=8, k=32, band=None, alpha=1.0,
                           gamma=0.995, data_seed=4, perm_seed=103,
                           batch_sizes=(4096, 65536, 1_000_000)),
}
