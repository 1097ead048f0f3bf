"""Certified FP64 correction of an approximate solution, in plain FP64.

The reduced-precision extension solves the MDP with its transition rows
stored in BF16 or FP8.  That MDP's solution differs from the solution of the
MDP as given (FP32 rows, widened to FP64 exactly) by the quantisation error.
This module states the final step that closes the gap, written from the
contraction property of the mini-batch operator:

* Every operator B_{sigma,b} of eq. (11) is a gamma-contraction in the max
  norm with the fixed point J*, for any order sigma and batch size b
  (Sec. III-B, the contraction lemma and the fixed-point result).  So is the
  Bellman operator T of eq. (7) (the case b = n).
* Hence, for any V:  max|V - J*| <= max|TV - V| / (1 - gamma).
* And for V' = B_{sigma,b} V:  max|V' - J*| <= gamma max|V' - V| / (1 - gamma)
  and max|V' - J*| <= gamma max|V - J*|.

The correction first evaluates the residual max|TV - V| of the input (one
pass of eq. (7) over all states, V fixed).  If the bound it gives is already
<= eps, V is returned unchanged.  Otherwise it applies sweeps of B_{sigma_t,b}
(eqs. (10)-(11), sigma_t the sweep order of ``permutation``) and stops after
the first sweep whose certified bound

    bound_t = min(gamma * max|V_t - V_{t-1}| / (1 - gamma), gamma * bound_{t-1})

is <= eps.  In measurement mode (a reference V_ref given) the stop is instead
the first iterate with max|V - V_ref| <= eps, and the bounds are still
reported.  All arithmetic is FP64; the bounds are those of exact arithmetic
(the rounding of one FP64 backup is of order (row length) * 2^-53 * max|V|).

``certified_correction_mpi`` is the same correction done by Algorithm 1
(modified policy iteration) with B_{mu,b} for its K evaluation steps: the
improvement step at V is one pass of eq. (7), so it yields the residual and
with it the certificate max|V - J*| <= max|TV - V| / (1 - gamma); the loop
stops at the first improvement whose certificate is <= eps.  The evaluation
sweeps move V towards J_mu, not J*, so their changes certify nothing.

Test infrastructure only (see the package docstring).
"""

from dataclasses import dataclass

import numpy as np

from .bellman import greedy, mb_sweep
from .permutation import sweep_permutation


@dataclass
class RefineStats:
    residual_in: float = float("nan")   # max|TV - V| of the input
    bound_in: float = float("nan")      # residual_in / (1 - gamma)
    residual_out: float = float("nan")  # max|TV - V| of the output
    sweeps: int = 0
    outer_iters: int = 0                # improvement steps after the input's (MPI form)
    final_dv_inf: float = float("nan")  # max|V_t - V_{t-1}| of the last sweep
    bound_out: float = float("nan")     # certified max|V_out - J*|
    final_err_ref: float = float("nan") # max|V_out - V_ref| (measurement mode)
    converged: bool = False


def certified_correction(mdp, V0, b, seed, eps, first_sweep=0, max_sweeps=100000, V_ref=None,
                         trace=None):
    """Returns (V, greedy policy at V, RefineStats).

    Sweep t uses the order ``sweep_permutation(n, seed, t)`` for t =
    first_sweep, first_sweep + 1, ...  ``trace``, if a list, receives
    (dv, bound, err) after each sweep.
    """
    gamma = float(mdp.gamma)
    V = np.asarray(V0, dtype=np.float64).copy()
    st = RefineStats()
    TV, _ = greedy(mdp, V)                                  # eq. (7), V fixed
    st.residual_in = float(np.max(np.abs(TV - V))) if mdp.n else 0.0
    st.bound_in = st.residual_in / (1.0 - gamma)
    bound = st.bound_in
    if V_ref is not None:
        st.final_err_ref = float(np.max(np.abs(V - V_ref)))
        done = st.final_err_ref <= eps
    else:
        done = bound <= eps
    t = first_sweep
    while not done and st.sweeps < max_sweeps:
        V, _, dv = mb_sweep(mdp, V, b, sweep_permutation(mdp.n, seed, t))
        t += 1
        st.sweeps += 1
        st.final_dv_inf = dv
        bound = min(gamma * dv / (1.0 - gamma), gamma * bound)
        if V_ref is not None:
            st.final_err_ref = float(np.max(np.abs(V - V_ref)))
            done = st.final_err_ref <= eps
        else:
            done = bound <= eps
        if trace is not None:
            trace.append((dv, bound, st.final_err_ref))
    st.bound_out = bound
    st.converged = bool(done)
    TV, pol = greedy(mdp, V)
    st.residual_out = float(np.max(np.abs(TV - V))) if mdp.n else 0.0
    return V, pol, st


def certified_correction_mpi(mdp, V0, K, b, seed, eps, first_sweep=0, max_outer=100000,
                             V_ref=None, trace=None):
    """Returns (V, greedy policy at V, RefineStats), by Algorithm 1.

    Outer iteration: the improvement step at V (eq. (7) over all states, V
    fixed) gives the greedy policy mu and the residual max|TV - V|; stop if
    residual / (1 - gamma) <= eps; else K sweeps of B_{mu,sigma_t,b} (eq.
    (12)) from V, sweep t using ``sweep_permutation(n, seed, t)`` for t =
    first_sweep, first_sweep + 1, ...  In measurement mode the stop is the
    first V (the input or an evaluation sweep's result) with max|V - V_ref|
    <= eps.  bound_out is the certificate of the output, from a last
    improvement step at it; ``trace``, if a list, receives (residual, bound)
    per improvement step.
    """
    gamma = float(mdp.gamma)
    V = np.asarray(V0, dtype=np.float64).copy()
    st = RefineStats()
    TV, mu = greedy(mdp, V)                                 # improvement at the input
    residual = float(np.max(np.abs(TV - V))) if mdp.n else 0.0
    st.residual_in = residual
    st.bound_in = residual / (1.0 - gamma)
    if trace is not None:
        trace.append((residual, st.bound_in))
    fresh = True                                            # mu and residual belong to V
    if V_ref is not None:
        st.final_err_ref = float(np.max(np.abs(V - V_ref)))
        done = st.final_err_ref <= eps
    else:
        done = st.bound_in <= eps
    t = first_sweep
    while not done and st.outer_iters < max_outer:
        for _ in range(K):
            V, _, dv = mb_sweep(mdp, V, b, sweep_permutation(mdp.n, seed, t), policy=mu)
            t += 1
            st.sweeps += 1
            st.final_dv_inf = dv
            fresh = False
            if V_ref is not None:
                st.final_err_ref = float(np.max(np.abs(V - V_ref)))
                if st.final_err_ref <= eps:
                    done = True
                    break
        if done:
            break
        TV, mu = greedy(mdp, V)
        st.outer_iters += 1
        residual = float(np.max(np.abs(TV - V)))
        fresh = True
        if trace is not None:
            trace.append((residual, residual / (1.0 - gamma)))
        if V_ref is None:
            done = residual / (1.0 - gamma) <= eps
    if not fresh:                                           # certificate of the output
        TV, mu = greedy(mdp, V)
        residual = float(np.max(np.abs(TV - V)))
    st.residual_out = residual
    st.bound_out = residual / (1.0 - gamma)
    st.converged = bool(done)
    return V, mu, st
