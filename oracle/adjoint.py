"""Gradients of a linear functional of the optimal cost-to-go, written from
the definitions.

The paper stops at computing J*; this is the differentiation extension of
the method.  For L = w^T J* with a unique optimal policy mu (no ties), J*
is locally the value of mu, J* = (I - gamma P_mu)^-1 c_mu (eq. (4)), so by
the chain rule with the adjoint lambda = (I - gamma P_mu)^-T w:

    dL/dc(s, a)       = lambda(s) [a == mu(s)]
    dL/dP(s, a, s')   = gamma lambda(s) J*(s') [a == mu(s)]

where dL/dP is the partial derivative with respect to the stored entry
(P is not re-projected onto the simplex).  Entries of rows that mu does not
select have zero gradient.

Test infrastructure only (see the package docstring).
"""

import numpy as np

from .bellman import CsrMDP, DenseMDP, _policy_matrix


def adjoint(mdp, mu, w, iterative_tol=None, dense=False):
    """lambda solving (I - gamma P_mu)^T lambda = w (FP64): LAPACK for dense
    storage (and for CSR storage with ``dense``: the matrix is formed densely
    and solved by LU), sparse LU for CSR, or -- when ``iterative_tol`` is
    given -- BiCGSTAB to that relative residual (for large random sparse
    matrices, whose LU fills in)."""
    n = mdp.n
    Pm = _policy_matrix(mdp, mu)
    w = np.asarray(w, dtype=np.float64)
    if isinstance(mdp, DenseMDP):
        return np.linalg.solve((np.eye(n) - mdp.gamma * Pm).T, w)
    if dense:
        A = -mdp.gamma * Pm.T.toarray()
        A[np.arange(n), np.arange(n)] += 1.0
        return np.linalg.solve(A, w)
    import scipy.sparse as sp
    import scipy.sparse.linalg as spla
    A = (sp.identity(n, format="csr") - mdp.gamma * Pm).T.tocsr()
    if iterative_tol is None:
        return spla.spsolve(A.tocsc(), w)
    x, info = spla.bicgstab(A, w, rtol=iterative_tol, atol=0.0, maxiter=100000)
    if info != 0:
        raise RuntimeError("BiCGSTAB did not converge (info=%d)" % info)
    return x


def value_gradients(mdp, mu, V, w, iterative_tol=None, dense=False):
    """(lambda, dL/dc [n, m], dL/dP) for L = w^T V at the policy mu with
    V = J_mu.  dL/dP has P's shape for dense storage and one entry per stored
    value for CSR storage."""
    n, m = mdp.n, mdp.m
    mu = np.asarray(mu, dtype=np.int64)
    V = np.asarray(V, dtype=np.float64)
    lam = adjoint(mdp, mu, w, iterative_tol, dense)
    gc = np.zeros((n, m))
    gc[np.arange(n), mu] = lam
    if isinstance(mdp, DenseMDP):
        gP = np.zeros((n, m, n))
        gP[np.arange(n), mu, :] = mdp.gamma * lam[:, None] * V[None, :]
        return lam, gc, gP
    gv = np.zeros(len(mdp.val))
    for s in range(n):
        r = s * m + mu[s]
        e0, e1 = mdp.row_ptr[r], mdp.row_ptr[r + 1]
        gv[e0:e1] = mdp.gamma * lam[s] * V[mdp.col[e0:e1]]
    return lam, gc, gv


def transpose_policy_rows(mdp, mu):
    """P_mu^T as CSR arrays (row_ptr int64 [n+1], col int32, val), each row's
    entries in increasing source state: row j lists every (s, P(s, mu(s), j))
    with an entry j in the row of (s, mu(s))."""
    assert isinstance(mdp, CsrMDP)
    n, m = mdp.n, mdp.m
    mu = np.asarray(mu, dtype=np.int64)
    src, dst, val = [], [], []
    for s in range(n):
        r = s * m + mu[s]
        e0, e1 = mdp.row_ptr[r], mdp.row_ptr[r + 1]
        src.append(np.full(e1 - e0, s, dtype=np.int64))
        dst.append(mdp.col[e0:e1].astype(np.int64))
        val.append(mdp.val[e0:e1])
    src = np.concatenate(src)
    dst = np.concatenate(dst)
    val = np.concatenate(val)
    order = np.lexsort((src, dst))  # by destination, then source
    counts = np.bincount(dst, minlength=n)
    row_ptr = np.concatenate(([0], np.cumsum(counts))).astype(np.int64)
    return row_ptr, src[order].astype(np.int32), val[order]
