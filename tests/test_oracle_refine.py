"""Pins of the oracle's certified FP64 correction (CPU only).

Checked against things other than the correction itself:

* the input residual against a plain triple loop over states, actions and
  successors (eq. (7) written out);
* J* by brute force over all policies (eq. (2)) and by LAPACK policy
  iteration (eq. (4)): every returned bound must hold, and the result must be
  within eps of J*;
* the stop rule: the first sweep whose certified bound is <= eps (the
  previous one's was not), with the bound recomputed here from the sweep's
  change and the contraction factor;
* the b = n and b = 1 cases against the textbook operators T and F;
* planted mistakes: a bound without the 1/(1 - gamma) factor, and a
  correction that stops one sweep early, each fail the checks above.
"""
import numpy as np
import pytest

import oracle
from oracle import DenseMDP, brute_force_optimum, policy_iteration, sweep_permutation
from oracle.refine import certified_correction
from paper_2110_02901_amd import inputs


def dense_random(n, m, seed, alpha=1.0, gamma=0.9):
    P, c = inputs.dense_mdp(n, m, alpha, seed, dtype=np.float64)
    return DenseMDP(P, c.astype(np.float64), gamma)


def loop_residual(mdp, V):
    """max_s |min_a (c(s,a) + gamma sum_j P(s,a,j) V(j)) - V(s)|, plain loops."""
    worst = 0.0
    for s in range(mdp.n):
        best = float("inf")
        for a in range(mdp.m):
            q = float(mdp.c[s, a])
            acc = 0.0
            for j in range(mdp.n):
                acc += float(mdp.P[s, a, j]) * float(V[j])
            q += mdp.gamma * acc
            best = min(best, q)
        worst = max(worst, abs(best - float(V[s])))
    return worst


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_input_residual_matches_loops(seed):
    mdp = dense_random(12, 3, seed)
    V0 = np.random.default_rng(seed).uniform(0, 8, 12)
    _, _, st = certified_correction(mdp, V0, 4, 5, eps=1e-9, max_sweeps=0)
    assert st.sweeps == 0 and not st.converged
    assert abs(st.residual_in - loop_residual(mdp, V0)) <= 1e-13
    assert st.bound_in == pytest.approx(st.residual_in / (1 - mdp.gamma), rel=1e-15)


@pytest.mark.parametrize("n,m,seed", [(4, 2, 1), (5, 3, 2), (6, 2, 3)])
@pytest.mark.parametrize("b", [1, 2, 6])
def test_bounds_hold_against_brute_force(n, m, seed, b):
    b = min(b, n)
    mdp = dense_random(n, m, seed, gamma=0.95)
    Vs, _ = brute_force_optimum(mdp)
    V0 = Vs + np.random.default_rng(seed).uniform(-0.3, 0.3, n)
    assert np.max(np.abs(V0 - Vs)) <= loop_residual(mdp, V0) / (1 - mdp.gamma) + 1e-12
    trace = []
    V, pol, st = certified_correction(mdp, V0, b, 7, eps=1e-7, trace=trace)
    assert st.converged and st.sweeps == len(trace) > 0
    err = float(np.max(np.abs(V - Vs)))
    assert err <= st.bound_out + 1e-12 and st.bound_out <= 1e-7
    # every intermediate bound holds too: replay the sweeps from V0
    Vt = V0.copy()
    for t, (dv, bound, _) in enumerate(trace):
        Vt, _, _ = oracle.mb_sweep(mdp, Vt, b, sweep_permutation(n, 7, t))
        assert np.max(np.abs(Vt - Vs)) <= bound + 1e-12
    # the greedy policy at the result is optimal
    Q = oracle.q_values(mdp, np.arange(n), Vs)
    assert np.all(Q[np.arange(n), pol] <= Q.min(axis=1) + 1e-6)


def test_stop_is_the_first_certified_sweep():
    mdp = dense_random(40, 4, 9, gamma=0.97)
    Vs, _, _ = policy_iteration(mdp)
    V0 = Vs + 1e-3 * np.random.default_rng(1).standard_normal(40)
    trace = []
    V, _, st = certified_correction(mdp, V0, 10, 3, eps=1e-9, first_sweep=5, trace=trace)
    g = mdp.gamma
    bound = st.bound_in
    Vt = V0.copy()
    for i, (dv, b_t, _) in enumerate(trace):
        Vn, _, dv_here = oracle.mb_sweep(mdp, Vt, 10, sweep_permutation(40, 3, 5 + i))
        assert dv == dv_here
        bound = min(g * dv_here / (1 - g), g * bound)
        assert b_t == bound
        assert (bound <= 1e-9) == (i == len(trace) - 1)
        Vt = Vn
    assert np.array_equal(V, Vt)
    assert np.max(np.abs(V - Vs)) <= 1e-9


def test_already_certified_input_is_returned_unchanged():
    mdp = dense_random(30, 3, 4)
    Vs, _, _ = policy_iteration(mdp)
    V, _, st = certified_correction(mdp, Vs, 7, 1, eps=1e-6)
    assert st.converged and st.sweeps == 0
    assert np.array_equal(V, Vs)
    assert st.bound_out == st.bound_in <= 1e-6


@pytest.mark.parametrize("b", [1, 30])
def test_sweeps_are_the_textbook_operators_at_the_ends(b):
    """b = n: each sweep is T (eq. (7)); b = 1: the Gauss-Seidel F in the
    sweep's order (Sec. II-D)."""
    mdp = dense_random(30, 3, 5)
    V0 = np.random.default_rng(2).uniform(0, 10, 30)
    V, _, st = certified_correction(mdp, V0, b, 8, eps=1e-30, max_sweeps=3)
    assert st.sweeps == 3 and not st.converged
    W = V0.copy()
    for t in range(3):
        if b == 30:
            W = np.min(mdp.c + mdp.gamma * np.einsum("san,n->sa", mdp.P, W), axis=1)
        else:
            for s in sweep_permutation(30, 8, t):
                W[s] = np.min(mdp.c[s] + mdp.gamma * mdp.P[s] @ W)
    assert np.max(np.abs(V - W)) <= 1e-12


def test_measurement_mode_stops_at_first_crossing():
    mdp = dense_random(25, 3, 6, gamma=0.9)
    Vs, _, _ = policy_iteration(mdp)
    V0 = np.zeros(25)
    trace = []
    V, _, st = certified_correction(mdp, V0, 5, 2, eps=1e-6, V_ref=Vs, trace=trace)
    errs = [e for _, _, e in trace]
    assert st.converged and errs[-1] <= 1e-6 and all(e > 1e-6 for e in errs[:-1])
    assert st.final_err_ref == pytest.approx(float(np.max(np.abs(V - Vs))), abs=0)
    assert np.max(np.abs(V - Vs)) <= st.bound_out + 1e-12


def test_planted_mistakes_are_caught():
    """A bound that drops the 1/(1 - gamma) factor claims more than holds, and
    a correction stopping one sweep early leaves the error above eps."""
    mdp = dense_random(50, 4, 11, gamma=0.99)
    Vs, _, _ = policy_iteration(mdp)
    V0 = Vs + 1e-3
    trace = []
    V, _, st = certified_correction(mdp, V0, 10, 4, eps=1e-8, trace=trace)
    # wrong bound: gamma * dv alone
    dv_last = trace[-1][0]
    assert np.max(np.abs(V - Vs)) > mdp.gamma * dv_last
    # one sweep early: the certificate does not hold there and the error is larger
    V_early, _, _ = certified_correction(mdp, V0, 10, 4, eps=1e-30, max_sweeps=st.sweeps - 1)
    assert trace[-2][1] > 1e-8
    assert np.max(np.abs(V_early - Vs)) > np.max(np.abs(V - Vs))


# ---- the same correction by Algorithm 1 (certified at improvement steps)

from oracle.refine import certified_correction_mpi  # noqa: E402


def loop_greedy(mdp, V):
    """(residual max|TV - V|, lowest minimising action per state), plain loops."""
    worst, pol = 0.0, np.zeros(mdp.n, dtype=np.int64)
    for s in range(mdp.n):
        best, arg = float("inf"), 0
        for a in range(mdp.m):
            q = float(mdp.c[s, a]) + mdp.gamma * sum(
                float(mdp.P[s, a, j]) * float(V[j]) for j in range(mdp.n))
            if q < best:
                best, arg = q, a
        pol[s] = arg
        worst = max(worst, abs(best - float(V[s])))
    return worst, pol


@pytest.mark.parametrize("n,m,seed", [(4, 2, 1), (5, 3, 2), (6, 2, 3)])
@pytest.mark.parametrize("K,b", [(1, 1), (3, 2), (5, 6)])
def test_mpi_bounds_hold_against_brute_force(n, m, seed, K, b):
    b = min(b, n)
    mdp = dense_random(n, m, seed, gamma=0.95)
    Vs, _ = brute_force_optimum(mdp)
    V0 = Vs + np.random.default_rng(seed).uniform(-0.3, 0.3, n)
    trace = []
    V, pol, st = certified_correction_mpi(mdp, V0, K, b, 7, eps=1e-7, trace=trace)
    assert st.converged and st.bound_out <= 1e-7
    assert np.max(np.abs(V - Vs)) <= st.bound_out + 1e-12
    assert len(trace) == st.outer_iters + 1 and st.sweeps == K * st.outer_iters
    # the residuals are those of plain loops, and the returned policy is greedy
    res, lp = loop_greedy(mdp, V)
    assert abs(res - st.residual_out) <= 1e-13
    assert np.array_equal(lp, pol)
    assert abs(loop_greedy(mdp, V0)[0] - st.residual_in) <= 1e-13


def test_mpi_replays_algorithm_1():
    """Improvement (greedy at V, plain loops), then K sweeps of B_{mu,b} with
    that policy; the stop is the first improvement whose certificate is <= eps."""
    mdp = dense_random(12, 3, 4, gamma=0.9)
    Vs, _, _ = policy_iteration(mdp)
    V0 = Vs + np.random.default_rng(3).uniform(-0.05, 0.05, 12)
    K, b, seed, eps = 2, 5, 9, 1e-8
    trace = []
    V, _, st = certified_correction_mpi(mdp, V0, K, b, seed, eps, first_sweep=4, trace=trace)
    Vt, t = V0.copy(), 4
    for i, (res, bound) in enumerate(trace):
        r, mu = loop_greedy(mdp, Vt)
        assert abs(r - res) <= 1e-13 and bound == res / (1 - mdp.gamma)
        assert (bound <= eps) == (i == len(trace) - 1)
        if i == len(trace) - 1:
            break
        for _ in range(K):
            Vt, _, _ = oracle.mb_sweep(mdp, Vt, b, sweep_permutation(12, seed, t), policy=mu)
            t += 1
    assert np.array_equal(V, Vt)
    assert np.max(np.abs(V - Vs)) <= eps


def test_mpi_measurement_mode_and_final_certificate():
    mdp = dense_random(20, 3, 6, gamma=0.9)
    Vs, _, _ = policy_iteration(mdp)
    V, _, st = certified_correction_mpi(mdp, np.zeros(20), 3, 4, 2, eps=1e-6, V_ref=Vs)
    assert st.converged and st.final_err_ref <= 1e-6
    assert st.final_err_ref == float(np.max(np.abs(V - Vs)))
    # the output's certificate comes from an improvement step at the output itself
    assert abs(loop_greedy(mdp, V)[0] - st.residual_out) <= 1e-13
    assert np.max(np.abs(V - Vs)) <= st.bound_out + 1e-12


def test_mpi_planted_mistake_evaluation_changes_certify_nothing():
    """Certifying with the evaluation sweeps' changes (as the VI form may)
    would stop at J_mu of a suboptimal policy: the changes vanish while the
    error does not."""
    mdp = dense_random(8, 3, 12, gamma=0.9)
    Vs, _ = brute_force_optimum(mdp)
    # a start whose greedy policy is not optimal
    V0 = np.zeros(8)
    _, mu0 = loop_greedy(mdp, V0)
    Q = oracle.q_values(mdp, np.arange(8), Vs)
    assert np.any(Q[np.arange(8), mu0] > Q.min(axis=1) + 1e-9)
    V = V0.copy()
    for t in range(300):
        V, _, dv = oracle.mb_sweep(mdp, V, 3, sweep_permutation(8, 1, t), policy=mu0)
    assert mdp.gamma * dv / (1 - mdp.gamma) <= 1e-9      # the wrong certificate fires
    assert np.max(np.abs(V - Vs)) > 1e-3                 # but V is far from J*
    _, _, st = certified_correction_mpi(mdp, V0, 300, 3, 1, eps=1e-9)
    assert st.outer_iters >= 1 and st.converged          # the right one goes on improving
