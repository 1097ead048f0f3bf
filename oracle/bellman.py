"""Mini-batch Bellman operators, VI, MPI and exact references in plain FP64.

Paper: Gargiani, Martinelli, Ruts Martinez, Lygeros, "Parallel and Flexible
Dynamic Programming via the Randomized Mini-Batch Operator" (arXiv
2110.02901).  Section and equation numbers below are the paper's.

Model (Sec. II-A): n states, m actions in every state, transition
probabilities P(s, a, s') (the paper's p_ij(u)), stage cost c(s, a) (g(i, u))
and discount gamma in (0, 1) (alpha).  A cost of +inf marks an action that is
not admissible in that state (the paper's U(i) is a non-empty subset of the
controls).  The stored arrays *are* the MDP: FP32 inputs are widened to FP64
exactly and never renormalised.

Two storage forms, both with transition row r = s*m + a:

* ``DenseMDP``: P is an [n, m, n] array.
* ``CsrMDP``:   CSR over the n*m rows (row_ptr int64[n*m + 1], col, val); a
                repeated column contributes once per entry.

Every floating-point result is computed in FP64 from the widened inputs.
Large inputs are processed in chunks of states; each Q-value is an
independent sum, so chunking changes nothing but memory use.

Test infrastructure only (see the package docstring).
"""

from dataclasses import dataclass
import itertools

import numpy as np

from .permutation import sweep_permutation

_CHUNK_ELEMS = 1 << 25  # elements of P widened at once (256 MB of FP64)


@dataclass
class DenseMDP:
    P: np.ndarray  # [n, m, n], any float dtype
    c: np.ndarray  # [n, m]
    gamma: float

    @property
    def n(self):
        return self.P.shape[0]

    @property
    def m(self):
        return self.P.shape[1]


@dataclass
class CsrMDP:
    row_ptr: np.ndarray  # int64 [n*m + 1]
    col: np.ndarray      # int [nnz]
    val: np.ndarray      # float [nnz]
    c: np.ndarray        # [n, m]
    gamma: float

    @property
    def n(self):
        return self.c.shape[0]

    @property
    def m(self):
        return self.c.shape[1]


def _expected_values(mdp, states, V, actions):
    """sum_{s'} P(s, a, s') * V(s') for the given states (FP64).

    ``actions`` None: all m actions, result [len(states), m].
    ``actions`` array: one action per state, result [len(states)].
    """
    V = np.asarray(V, dtype=np.float64)
    states = np.asarray(states, dtype=np.int64)
    if isinstance(mdp, DenseMDP):
        n, m = mdp.n, mdp.m
        per_state = n * (m if actions is None else 1)
        step = max(1, _CHUNK_ELEMS // max(per_state, 1))
        parts = []
        for i in range(0, len(states), step):
            s = states[i:i + step]
            if actions is None:
                rows = mdp.P[s].astype(np.float64)               # [k, m, n]
            else:
                rows = mdp.P[s, np.asarray(actions)[i:i + step]].astype(np.float64)  # [k, n]
            parts.append(rows @ V)
        if not parts:
            return np.zeros((0, m) if actions is None else (0,))
        return np.concatenate(parts, axis=0)
    # CSR: row r = s*m + a holds entries row_ptr[r] .. row_ptr[r+1]-1.
    m = mdp.m
    if actions is None:
        rows = (states[:, None] * m + np.arange(m)[None, :]).reshape(-1)
    else:
        rows = states * m + np.asarray(actions, dtype=np.int64)
    out = np.zeros(len(rows), dtype=np.float64)
    starts = mdp.row_ptr[rows]
    lengths = mdp.row_ptr[rows + 1] - starts
    step_rows = max(1, _CHUNK_ELEMS // max(int(lengths.max(initial=1)), 1))
    for i in range(0, len(rows), step_rows):
        st = starts[i:i + step_rows]
        ln = lengths[i:i + step_rows]
        seg = np.repeat(np.arange(len(st)), ln)
        # entry index of every nonzero of these rows, in ascending order per row
        first = np.repeat(st - np.concatenate(([0], np.cumsum(ln)[:-1])), ln)
        idx = first + np.arange(int(ln.sum()))
        prod = mdp.val[idx].astype(np.float64) * V[mdp.col[idx]]
        out[i:i + step_rows] = np.bincount(seg, weights=prod, minlength=len(st))
    return out.reshape(-1, m) if actions is None else out


def q_values(mdp, states, V, actions=None):
    """Q(s, a) = c(s, a) + gamma * sum_{s'} P(s, a, s') V(s')  (eqs. (6), (7)).

    With ``actions`` None returns [len(states), m]; otherwise the Q-value of
    the given action of each state.
    """
    states = np.asarray(states, dtype=np.int64)
    c = np.asarray(mdp.c, dtype=np.float64)
    ev = _expected_values(mdp, states, V, actions)
    if actions is None:
        return c[states] + mdp.gamma * ev
    return c[states, np.asarray(actions, dtype=np.int64)] + mdp.gamma * ev


def mb_sweep(mdp, V, b, order, policy=None):
    """One application of the mini-batch operator, eqs. (11) and (12).

    ``order`` is the processing order (order[p] = state at position p).  The
    positions are cut into consecutive batches of ``b`` (the last one may be
    shorter).  By eq. (10), M_b(i) -- the states already updated when state
    i is processed -- is the union of the earlier batches.  So each state of
    a batch sees the new values of earlier batches and the old values of its
    own and later batches, itself included; the batch is committed only after
    all its values are computed.

    policy None: B_b, V'(s) = min_a Q(s, a), argmin = lowest minimising action.
    policy given: B_{mu,b}, V'(s) = Q(s, mu(s)), argmin = mu.
    Returns (V' float64 [n], argmin int64 [n], max_s |V'(s) - V(s)|).
    """
    n = mdp.n
    if not 1 <= b <= n:
        raise ValueError("batch size must satisfy 1 <= b <= n")
    order = np.asarray(order, dtype=np.int64)
    V_old = np.asarray(V, dtype=np.float64)
    V_new = V_old.copy()
    arg = np.zeros(n, dtype=np.int64)
    for start in range(0, n, b):
        batch = order[start:start + b]
        if policy is None:
            Q = q_values(mdp, batch, V_new)
            new_vals = Q.min(axis=1)
            arg[batch] = Q.argmin(axis=1)  # first occurrence = lowest index
        else:
            mu = np.asarray(policy, dtype=np.int64)[batch]
            new_vals = q_values(mdp, batch, V_new, actions=mu)
            arg[batch] = mu
        V_new[batch] = new_vals
    dv = float(np.max(np.abs(V_new - V_old))) if n else 0.0
    return V_new, arg, dv


def greedy(mdp, V):
    """(TV, greedy policy): eq. (7) over all states, lowest index on ties.

    This is also the policy-improvement step of Algorithm 1.
    """
    Q = q_values(mdp, np.arange(mdp.n), V)
    return Q.min(axis=1), Q.argmin(axis=1)


@dataclass
class SolveStats:
    sweeps: int = 0
    outer_iters: int = 0
    policy_changes_last: int = -1
    final_dv_inf: float = float("nan")
    final_err_ref: float = float("nan")
    converged: bool = False


def value_iteration(mdp, b, seed, V0=None, tol_dv=1e-8, max_sweeps=100000,
                    V_ref=None, eps=None, first_sweep=0, trace=None):
    """MB-VI (Sec. III-B): V_{t+1} = B_b V_t with a fresh order sigma_t per sweep.

    V_0 = 0 unless given (the paper's experiments start from zero, Sec. IV-A).
    Stops after the first sweep with max|V_{t+1} - V_t| <= tol_dv (tol_dv < 0
    disables this rule) or, when V_ref is given, with max|V_{t+1} - V_ref| <=
    eps.  Sweep t uses sigma_t from ``sweep_permutation(n, seed, t)`` with
    t = first_sweep, first_sweep + 1, ...  Returns (V, greedy policy, stats).
    ``trace``, if a list, receives (dv, err) per sweep.
    """
    n = mdp.n
    V = np.zeros(n) if V0 is None else np.asarray(V0, dtype=np.float64).copy()
    st = SolveStats()
    for t in range(first_sweep, first_sweep + max_sweeps):
        V, _, dv = mb_sweep(mdp, V, b, sweep_permutation(n, seed, t))
        st.sweeps += 1
        st.final_dv_inf = dv
        stop = tol_dv >= 0 and dv <= tol_dv
        if V_ref is not None:
            st.final_err_ref = float(np.max(np.abs(V - V_ref)))
            stop = stop or st.final_err_ref <= eps
        if trace is not None:
            trace.append((dv, st.final_err_ref))
        if stop:
            st.converged = True
            break
    _, pol = greedy(mdp, V)
    return V, pol, st


def modified_policy_iteration(mdp, K, b, seed, V0=None, mu0=None, tol_dv=1e-8,
                              max_outer=10000, V_ref=None, eps=None,
                              first_sweep=0):
    """MB-MPI: Algorithm 1 with the K evaluation steps done by B_{mu,b}.

    Policy evaluation warm-starts from the current V (Sec. II-C).  When no
    initial policy is given it is the greedy policy at V_0.  Each outer
    iteration runs K sweeps of B_{mu,b} (sweep t uses sigma_t, t counting all
    evaluation sweeps from ``first_sweep``), then the improvement step over
    all states with V fixed (no V update).  The loop stops when an
    improvement leaves the policy unchanged and the Bellman residual
    max|TV - V| is <= tol_dv, or -- when V_ref is given -- after the first
    evaluation sweep with max|V - V_ref| <= eps.  Returns (V, mu, stats).
    """
    n = mdp.n
    V = np.zeros(n) if V0 is None else np.asarray(V0, dtype=np.float64).copy()
    st = SolveStats()
    if mu0 is None:
        _, mu = greedy(mdp, V)
    else:
        mu = np.asarray(mu0, dtype=np.int64).copy()
    t = first_sweep
    for _ in range(max_outer):
        for _k in range(K):
            V, _, dv = mb_sweep(mdp, V, b, sweep_permutation(n, seed, t), policy=mu)
            t += 1
            st.sweeps += 1
            st.final_dv_inf = dv
            if V_ref is not None:
                st.final_err_ref = float(np.max(np.abs(V - V_ref)))
                if st.final_err_ref <= eps:
                    st.converged = True
                    return V, mu, st
        TV, mu_new = greedy(mdp, V)
        st.outer_iters += 1
        st.policy_changes_last = int(np.count_nonzero(mu_new != mu))
        residual = float(np.max(np.abs(TV - V)))
        mu = mu_new
        if st.policy_changes_last == 0 and tol_dv >= 0 and residual <= tol_dv:
            st.final_dv_inf = residual
            st.converged = True
            break
    return V, mu, st


def _policy_matrix(mdp, mu):
    """Rows of P selected by the policy, as a dense [n, n] FP64 matrix or a
    scipy sparse matrix (CSR storage)."""
    n = mdp.n
    mu = np.asarray(mu, dtype=np.int64)
    if isinstance(mdp, DenseMDP):
        return mdp.P[np.arange(n), mu].astype(np.float64)
    import scipy.sparse as sp
    rows = np.arange(n) * mdp.m + mu
    starts = mdp.row_ptr[rows]
    lengths = mdp.row_ptr[rows + 1] - starts
    first = np.repeat(starts - np.concatenate(([0], np.cumsum(lengths)[:-1])), lengths)
    idx = first + np.arange(int(lengths.sum()))
    indptr = np.concatenate(([0], np.cumsum(lengths)))
    # duplicate columns are summed by the conversion, as in the operator
    return sp.csr_matrix((mdp.val[idx].astype(np.float64), mdp.col[idx], indptr),
                         shape=(n, n))


def policy_value(mdp, mu, iterative_tol=None):
    """J_mu from the Bellman equation of mu, eq. (4): (I - gamma P_mu) V = c_mu.

    Dense storage: LAPACK solve.  CSR storage: sparse LU, or -- when
    ``iterative_tol`` is given -- BiCGSTAB to that relative residual.
    """
    n = mdp.n
    mu = np.asarray(mu, dtype=np.int64)
    c_mu = np.asarray(mdp.c, dtype=np.float64)[np.arange(n), mu]
    Pm = _policy_matrix(mdp, mu)
    if isinstance(mdp, DenseMDP):
        return np.linalg.solve(np.eye(n) - mdp.gamma * Pm, c_mu)
    import scipy.sparse as sp
    import scipy.sparse.linalg as spla
    A = (sp.identity(n, format="csr") - mdp.gamma * Pm).tocsc()
    if iterative_tol is None:
        return spla.spsolve(A, c_mu)
    x, info = spla.bicgstab(A.tocsr(), c_mu, rtol=iterative_tol, atol=0.0,
                            maxiter=100000)
    if info != 0:
        raise RuntimeError("BiCGSTAB did not converge (info=%d)" % info)
    return x


def policy_iteration(mdp, mu0=None, max_iter=1000, improve_tol=1e-12,
                     iterative_tol=None):
    """Howard policy iteration (Sec. II-C): exact evaluation by eq. (4), then
    greedy improvement.  A state switches action only when some action
    improves on its current value by more than ``improve_tol`` times
    max(1, |V|), so rounding-level ties cannot make it cycle.  Returns
    (J*, optimal policy, iterations)."""
    n = mdp.n
    mu = greedy(mdp, np.zeros(n))[1] if mu0 is None else np.asarray(mu0).copy()
    for it in range(1, max_iter + 1):
        V = policy_value(mdp, mu, iterative_tol=iterative_tol)
        TV, mu_g = greedy(mdp, V)
        better = TV < V - improve_tol * np.maximum(1.0, np.abs(V))
        if not better.any():
            return V, mu, it
        mu = np.where(better, mu_g, mu)
    raise RuntimeError("policy iteration did not terminate")


def brute_force_optimum(mdp):
    """J* by definition, eq. (2): the elementwise minimum of J_mu over all
    m**n stationary policies (each J_mu from eq. (4)).  Only for tiny MDPs.
    Returns (J*, list of policies mu with J_mu == J* to 1e-12)."""
    n, m = mdp.n, mdp.m
    c = np.asarray(mdp.c, dtype=np.float64)
    values = []
    policies = []
    for mu in itertools.product(range(m), repeat=n):
        mu = np.array(mu)
        if not np.all(np.isfinite(c[np.arange(n), mu])):
            continue  # uses an inadmissible action
        values.append(policy_value(mdp, mu))
        policies.append(mu)
    values = np.array(values)
    J = values.min(axis=0)
    optimal = [p for p, v in zip(policies, values)
               if np.max(np.abs(v - J)) <= 1e-12 * max(1.0, np.max(np.abs(J)))]
    return J, optimal


def row_sums(mdp):
    """rho(s, a) = sum_{s'} P(s, a, s') in FP64, shape [n, m]."""
    n, m = mdp.n, mdp.m
    if isinstance(mdp, DenseMDP):
        out = np.empty((n, m))
        step = max(1, _CHUNK_ELEMS // (m * n))
        for i in range(0, n, step):
            out[i:i + step] = mdp.P[i:i + step].astype(np.float64).sum(axis=2)
        return out
    lengths = np.diff(mdp.row_ptr)
    seg = np.repeat(np.arange(n * m), lengths)
    return np.bincount(seg, weights=mdp.val.astype(np.float64),
                       minlength=n * m).reshape(n, m)


def shifted_costs(mdp, r):
    """Costs c' for iterating W = V - r instead of V, r a scalar or a vector.

    Every value a state reads in eq. (11) -- old or new -- is V(j) = W(j) + r(j),
    so each bracket c(s,a) + gamma * sum_j P(s,a,j) V(j) equals
    [c(s,a) - r(s) + gamma * (P r)(s,a)] + r(s) + gamma * sum_j P(s,a,j) W(j).
    With c'(s,a) = c(s,a) - r(s) + gamma * (P r)(s,a) the operator with costs
    c' maps W to B(V) - r for any order and batch size (exact in real
    arithmetic).  For a scalar r, P r = r * rho (the row sums), which is the
    shift of the shift-invariance lemma (Sec. III-B.1) with rho = 1 for
    stochastic rows.
    """
    c = np.asarray(mdp.c, dtype=np.float64)
    n = mdp.n
    if np.ndim(r) == 0:
        return c - r + mdp.gamma * r * row_sums(mdp)
    r = np.asarray(r, dtype=np.float64)
    Pr = _expected_values(mdp, np.arange(n), r, None)  # (P r)(s, a)
    return c - r[:, None] + mdp.gamma * Pr
