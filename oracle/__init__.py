"""Plain FP64 CPU oracle for the randomized mini-batch Bellman operator.

TEST INFRASTRUCTURE ONLY.  This package is the slow, obviously correct
reference that the GPU library is checked against.  Only the test suite, the
smoke check and the CPU-baseline leg of the benchmark may import it; the
product path (the HIP library and its Python binding) never does, and shares
no code with it.

Everything here follows the paper "Parallel and Flexible Dynamic Programming
via the Randomized Mini-Batch Operator" (Gargiani, Martinelli, Ruts Martinez,
Lygeros; arXiv 2110.02901):

* ``philox``      -- the counter-based generator (Salmon et al., SC'11) used to
                     draw the per-sweep state order.
* ``permutation`` -- the seeded state order sigma_t of one sweep (the paper
                     shuffles the states before every operator evaluation,
                     Sec. IV-A, uniformly without replacement, Sec. V).
* ``bellman``     -- Q-values, the mini-batch operators B_b and B_{mu,b}
                     (Sec. III-A, eqs. (10)-(12)), value iteration, modified
                     policy iteration (Algorithm 1), exact policy evaluation
                     (eq. (4)), Howard policy iteration and brute-force
                     enumeration of J* (eq. (2)).
* ``adjoint``     -- gradients of L = w^T J* with respect to the costs and the
                     stored transition values at the optimal policy, via the
                     adjoint equation (I - gamma P_mu)^T lambda = w.
* ``multi``       -- r value vectors (one per cost vector) backed up against
                     one P with a shared order: MB-VI column by column,
                     one matrix product per batch.
* ``quantize``    -- BF16 / FP8 E4M3 storage of transition rows with one
                     scale per row renormalising it to sum 1 (the reduced-
                     precision variant; the paper fixes no precision).
* ``refine``      -- the certified FP64 correction that closes the gap between
                     the stored MDP's solution and the given MDP's: the input
                     residual max|TV - V| and mini-batch sweeps until the
                     contraction bound (Sec. III-B) certifies eps, or the
                     same by Algorithm 1, certified at its improvement steps.

Notation: the paper's batch size ``m`` is called ``b`` here, because ``m`` is
the number of actions; the paper's cost-to-go ``J`` is ``V`` and its discount
``alpha`` is ``gamma``.  The problem is cost minimisation.

Parity status: every public function is pinned by the CPU tests in
``tests/test_oracle_*.py`` (known-answer vectors, library routines, closed
forms, brute force and the paper's lemmas); none is "parity unpinned".
"""

from .philox import philox4x32_10, philox_scalar
from .permutation import half_bits, feistel_encrypt, sweep_permutation
from .bellman import (
    DenseMDP,
    CsrMDP,
    q_values,
    mb_sweep,
    greedy,
    value_iteration,
    modified_policy_iteration,
    policy_value,
    policy_iteration,
    brute_force_optimum,
    row_sums,
    shifted_costs,
)

__all__ = [
    "philox4x32_10",
    "philox_scalar",
    "half_bits",
    "feistel_encrypt",
    "sweep_permutation",
    "DenseMDP",
    "CsrMDP",
    "q_values",
    "mb_sweep",
    "greedy",
    "value_iteration",
    "modified_policy_iteration",
    "policy_value",
    "policy_iteration",
    "brute_force_optimum",
    "row_sums",
    "shifted_costs",
]
