"""Several value vectors against one transition array, written from the
definitions.

The extension backs up r value vectors V[:, j] at once, one per cost vector
C[:, :, j], all sharing the transition probabilities P, the discount, the
batch size b and the sweep order sigma_t.  Column j follows MB-VI of the MDP
(P, C[:, :, j]) exactly: for the states of a batch

    Q[s, a, j] = C[s, a, j] + gamma * sum_{s'} P[s, a, s'] V[s', j]   (eqs. (6)-(7))
    V'[s, j]   = min_a Q[s, a, j]                                      (eq. (11))

with the batch committed after all its reads (eqs. (10)-(12)), and the
lowest minimising action on ties.  For one batch the expected values of all
columns are one matrix product, rows (s, a) of P against V [n, r]; that
product is the only step beyond the single-vector operator.

Test infrastructure only (see the package docstring).
"""

import numpy as np

from .permutation import sweep_permutation


def multi_q_values(P, C, gamma, states, V):
    """Q[k, a, j] for the given states: [len(states), m, r] (FP64)."""
    states = np.asarray(states, dtype=np.int64)
    rows = np.asarray(P)[states].astype(np.float64)          # [k, m, n]
    EV = rows @ np.asarray(V, dtype=np.float64)               # [k, m, r]
    return np.asarray(C, dtype=np.float64)[states] + gamma * EV


def multi_mb_sweep(P, C, gamma, V, b, order):
    """One sweep of the mini-batch operator on every column of V [n, r].

    Returns (V' [n, r], argmin [n, r], max |V' - V| per column [r])."""
    n = P.shape[0]
    if not 1 <= b <= n:
        raise ValueError("batch size must satisfy 1 <= b <= n")
    order = np.asarray(order, dtype=np.int64)
    V_old = np.asarray(V, dtype=np.float64)
    V_new = V_old.copy()
    arg = np.zeros(V_old.shape, dtype=np.int64)
    for start in range(0, n, b):
        batch = order[start:start + b]
        Q = multi_q_values(P, C, gamma, batch, V_new)        # reads before the commit
        V_new[batch] = Q.min(axis=1)
        arg[batch] = Q.argmin(axis=1)                         # first = lowest action
    dv = np.max(np.abs(V_new - V_old), axis=0) if n else np.zeros(V_old.shape[1])
    return V_new, arg, dv


def multi_value_iteration(P, C, gamma, b, seed, V0=None, tol_dv=1e-8, max_sweeps=100000,
                          first_sweep=0):
    """MB-VI on all columns with a common order per sweep; stops after the
    first sweep whose largest change over all columns is <= tol_dv (tol_dv < 0
    disables the rule).  Returns (V [n, r], greedy policy [n, r], sweeps,
    max |dV| of the last sweep)."""
    n, r = P.shape[0], C.shape[2]
    V = np.zeros((n, r)) if V0 is None else np.asarray(V0, dtype=np.float64).copy()
    sweeps, dv = 0, float("nan")
    for t in range(first_sweep, first_sweep + max_sweeps):
        V, _, dvs = multi_mb_sweep(P, C, gamma, V, b, sweep_permutation(n, seed, t))
        sweeps += 1
        dv = float(np.max(dvs)) if r else 0.0
        if tol_dv >= 0 and dv <= tol_dv:
            break
    Q = multi_q_values(P, C, gamma, np.arange(n), V)
    return V, Q.argmin(axis=1), sweeps, dv
