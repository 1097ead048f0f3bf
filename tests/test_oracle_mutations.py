"""Planted mistakes: each plausible slip in the oracle's sweep must be caught
by at least one of the pins used in test_oracle_bellman.py.

The mistakes are planted in copies of the oracle's sweep, on the CPU; the
pins below are the same independent checks (hand-worked values, the b = n
and b = 1 textbook operators, the closed form of a policy sweep, the fixed
point J*)."""
import numpy as np
import pytest

from oracle import DenseMDP, policy_iteration, sweep_permutation
from oracle.bellman import mb_sweep as correct_sweep
from paper_2110_02901_amd import inputs

from test_oracle_bellman import (_hand, policy_sweep_closed_form, textbook_F,
                                 textbook_T)


def _sweep_variant(mistake):
    """A state-by-state restatement of the sweep with one planted mistake
    ("none" plants nothing)."""
    def sweep(mdp, V, b, order, policy=None):
        n, m = mdp.n, mdp.m
        P = np.asarray(mdp.P, dtype=np.float64)
        c = np.asarray(mdp.c, dtype=np.float64)
        gamma = 1.0 if mistake == "dropped-gamma" else mdp.gamma
        order = np.asarray(order)
        V_old = np.asarray(V, dtype=np.float64)
        V_new = V_old.copy()
        arg = np.zeros(n, dtype=np.int64)
        width = b + 1 if mistake == "overlapping-batches" else b
        for start in range(0, n, b):
            pending = {}
            for s in order[start:start + width]:
                src = V_old if mistake == "jacobi-across-batches" else V_new
                if mistake == "transposed-P":
                    ev = np.array([P[:, a, s] @ src for a in range(m)])
                else:
                    ev = P[s] @ src
                Q = c[s] - gamma * ev if mistake == "wrong-sign" else c[s] + gamma * ev
                if policy is not None:
                    a = int(policy[start] if mistake == "policy-by-position" else policy[s])
                elif mistake == "max-not-min":
                    a = int(np.argmax(Q))
                else:
                    a = int(np.argmin(Q))
                arg[s] = a
                if mistake == "in-batch-gauss-seidel":
                    V_new[s] = Q[a]
                else:
                    pending[s] = Q[a]
            for s, val in pending.items():
                V_new[s] = val
        return V_new, arg, float(np.max(np.abs(V_new - V_old)))
    return sweep


def _pins_pass(sweep):
    ex = _hand()
    # hand example A
    P = np.zeros((3, 1, 3))
    P[0, 0, 2] = P[1, 0, 0] = P[2, 0, 1] = 1.0
    hand = DenseMDP(P, np.array([[1.0], [2.0], [3.0]]), 0.5)
    for b in (3, 1, 2):
        if not np.allclose(sweep(hand, np.zeros(3), b, np.arange(3))[0], ex[("A", "b=%d" % b)]):
            return False
    # random MDP: b = n, b = 1, closed-form policy sweep, fixed point
    n, m = 24, 3
    Pr, cr = inputs.dense_mdp(n, m, 1.0, 5, dtype=np.float64)
    mdp = DenseMDP(Pr, cr, 0.9)
    V = inputs.values(n, 1, 0, 5, dtype=np.float64)
    order = sweep_permutation(n, 2, 0)
    if not np.allclose(sweep(mdp, V, n, order)[0], textbook_T(Pr, cr, 0.9, V), rtol=1e-12):
        return False
    if not np.allclose(sweep(mdp, V, 1, order)[0], textbook_F(Pr, cr, 0.9, V, order), rtol=1e-12):
        return False
    mu = inputs.policy(n, m, 3).astype(np.int64)
    got = sweep(mdp, V, 5, order, policy=mu)[0]
    if not np.allclose(got, policy_sweep_closed_form(Pr, cr, 0.9, V, 5, order, mu), rtol=1e-12):
        return False
    Vstar, _, _ = policy_iteration(mdp)
    if not np.allclose(sweep(mdp, Vstar, 7, order)[0], Vstar, atol=1e-11):
        return False
    return True


def test_pins_accept_the_correct_sweep():
    assert _pins_pass(correct_sweep)
    assert _pins_pass(_sweep_variant("none"))


@pytest.mark.parametrize("mistake", [
    "in-batch-gauss-seidel", "jacobi-across-batches", "dropped-gamma",
    "max-not-min", "transposed-P", "overlapping-batches", "wrong-sign",
    "policy-by-position",
])
def test_pins_reject_planted_mistake(mistake):
    assert not _pins_pass(_sweep_variant(mistake))
