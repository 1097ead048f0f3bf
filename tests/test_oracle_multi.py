"""Pins of the oracle's multi-vector operator (CPU).

References other than the multi-vector code itself: the single-vector
operator and MB-VI (pinned in test_oracle_bellman.py) run column by column,
the Bellman operator written out with Python loops at b = n, policy
iteration's J* at the fixed point, linearity of the operator when there is a
single action, and equivariance under a permutation of the columns.
"""
import numpy as np

import oracle
from oracle import multi
from paper_2110_02901_amd import inputs


def _mdp(n, m, r, seed, alpha=1.0):
    P, _ = inputs.dense_mdp(n, m, alpha, seed, dtype=np.float64)
    C = inputs.multi_costs(n, m, r, seed + 1, dtype=np.float64)
    return P, C


def test_columns_follow_the_single_vector_operator():
    n, m, r = 37, 3, 5
    P, C = _mdp(n, m, r, 3)
    V0 = np.stack([inputs.values(n, 10 + j, 0.0, 3.0, dtype=np.float64) for j in range(r)], axis=1)
    for b in (1, 4, 7, 37):
        order = oracle.sweep_permutation(n, 9, 2)
        Vm, am, dvm = multi.multi_mb_sweep(P, C, 0.9, V0, b, order)
        for j in range(r):
            Vs, as_, dvs = oracle.mb_sweep(oracle.DenseMDP(P, C[:, :, j], 0.9), V0[:, j], b, order)
            assert np.allclose(Vm[:, j], Vs, rtol=0, atol=1e-13)
            assert np.array_equal(am[:, j], as_)
            assert abs(dvm[j] - dvs) <= 1e-13


def test_bellman_operator_written_out_at_b_equal_n():
    n, m, r = 6, 2, 3
    P, C = _mdp(n, m, r, 5)
    V = np.arange(n * r, dtype=np.float64).reshape(n, r) / 7.0
    gamma = 0.8
    Vn, arg, _ = multi.multi_mb_sweep(P, C, gamma, V, n, np.arange(n))
    for s in range(n):
        for j in range(r):
            best, best_a = None, None
            for a in range(m):
                q = C[s, a, j] + gamma * sum(P[s, a, t] * V[t, j] for t in range(n))
                if best is None or q < best:
                    best, best_a = q, a
            assert abs(Vn[s, j] - best) <= 1e-13
            assert arg[s, j] == best_a


def test_fixed_point_is_each_columns_optimum():
    n, m, r = 40, 4, 3
    P, C = _mdp(n, m, r, 8)
    V, pol, sweeps, dv = multi.multi_value_iteration(P, C, 0.9, 8, 4, tol_dv=1e-12)
    assert dv <= 1e-12
    for j in range(r):
        Vs, mu, _ = oracle.policy_iteration(oracle.DenseMDP(P, C[:, :, j], 0.9), improve_tol=1e-14)
        assert np.max(np.abs(V[:, j] - Vs)) <= 1e-10
        assert np.array_equal(pol[:, j], mu)


def test_single_action_operator_is_linear():
    n, r = 30, 4
    P, C = _mdp(n, 1, r, 12)
    g = np.random.Generator(np.random.Philox(3))
    V1, V2 = g.standard_normal((n, r)), g.standard_normal((n, r))
    C2 = g.standard_normal((n, 1, r))
    order = oracle.sweep_permutation(n, 1, 0)
    x, y = 0.7, -1.3
    L, _, _ = multi.multi_mb_sweep(P, x * C + y * C2, 0.95, x * V1 + y * V2, 6, order)
    A, _, _ = multi.multi_mb_sweep(P, C, 0.95, V1, 6, order)
    B, _, _ = multi.multi_mb_sweep(P, C2, 0.95, V2, 6, order)
    assert np.allclose(L, x * A + y * B, rtol=0, atol=1e-12)


def test_column_permutation_equivariance():
    n, m, r = 25, 3, 6
    P, C = _mdp(n, m, r, 14)
    V0 = np.random.Generator(np.random.Philox(4)).random((n, r))
    perm = np.array([3, 0, 5, 1, 4, 2])
    order = oracle.sweep_permutation(n, 2, 1)
    A, aa, da = multi.multi_mb_sweep(P, C, 0.9, V0, 5, order)
    B, ab, db = multi.multi_mb_sweep(P, C[:, :, perm], 0.9, V0[:, perm], 5, order)
    assert np.array_equal(A[:, perm], B) and np.array_equal(aa[:, perm], ab)
    assert np.array_equal(da[perm], db)


def test_value_iteration_matches_single_vector_runs():
    n, m, r = 50, 3, 4
    P, C = _mdp(n, m, r, 21)
    V, pol, sweeps, dv = multi.multi_value_iteration(P, C, 0.9, 13, 6, tol_dv=-1, max_sweeps=9)
    assert sweeps == 9
    for j in range(r):
        Vs, _, st = oracle.value_iteration(oracle.DenseMDP(P, C[:, :, j], 0.9), 13, 6, tol_dv=-1,
                                           max_sweeps=9)
        assert np.allclose(V[:, j], Vs, rtol=0, atol=1e-13)
