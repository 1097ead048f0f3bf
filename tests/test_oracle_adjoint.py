"""Pins of the oracle's gradients of L = w^T J* (CPU).

References other than the oracle's adjoint itself: central finite
differences of L through policy iteration and through brute-force
enumeration (eq. (2)), the duality identity lambda^T c_mu = w^T J*, a
dense LAPACK solve against the sparse LU, and scipy's own transpose.
"""
import numpy as np
import pytest

import oracle
from oracle import adjoint as adj
from paper_2110_02901_amd import inputs


def _w(n, seed):
    return np.random.Generator(np.random.Philox(seed)).standard_normal(n)


def _solve(mdp):
    V, mu, _ = oracle.policy_iteration(mdp, improve_tol=1e-14)
    return V, mu


def _csr(n, m, k, seed, gamma):
    rp, col, val, c = inputs.csr_mdp(n, m, k, 1.0, seed)
    return oracle.CsrMDP(rp, col, val.astype(np.float64), c.astype(np.float64), gamma)


def _margin(mdp, V, mu):
    """Smallest Q-gap between the optimal action and the next best."""
    Q = oracle.q_values(mdp, np.arange(mdp.n), V)
    srt = np.sort(Q, axis=1)
    return float(np.min(srt[:, 1] - srt[:, 0]))


def test_gradients_match_central_differences_sparse():
    mdp = _csr(40, 3, 6, 11, 0.9)
    w = _w(40, 1)
    V, mu = _solve(mdp)
    assert _margin(mdp, V, mu) > 1e-3
    lam, gc, gv = adj.value_gradients(mdp, mu, V, w)
    h = 1e-5
    g = np.random.Generator(np.random.Philox(2))
    for s in g.choice(40, 6, replace=False):
        for a in range(3):
            cp, cm = mdp.c.copy(), mdp.c.copy()
            cp[s, a] += h
            cm[s, a] -= h
            Lp = w @ _solve(oracle.CsrMDP(mdp.row_ptr, mdp.col, mdp.val, cp, mdp.gamma))[0]
            Lm = w @ _solve(oracle.CsrMDP(mdp.row_ptr, mdp.col, mdp.val, cm, mdp.gamma))[0]
            assert abs((Lp - Lm) / (2 * h) - gc[s, a]) <= 1e-6 * max(1.0, abs(gc[s, a]))
    for e in g.choice(len(mdp.val), 12, replace=False):
        vp, vm = mdp.val.copy(), mdp.val.copy()
        vp[e] += h
        vm[e] -= h
        Lp = w @ _solve(oracle.CsrMDP(mdp.row_ptr, mdp.col, vp, mdp.c, mdp.gamma))[0]
        Lm = w @ _solve(oracle.CsrMDP(mdp.row_ptr, mdp.col, vm, mdp.c, mdp.gamma))[0]
        assert abs((Lp - Lm) / (2 * h) - gv[e]) <= 1e-6 * max(1.0, abs(gv[e]))


def test_gradients_match_brute_force_differences_dense():
    P, c = inputs.dense_mdp(4, 2, 1.0, 5, dtype=np.float64)
    mdp = oracle.DenseMDP(P, c, 0.8)
    w = _w(4, 3)
    V, mus = oracle.brute_force_optimum(mdp)
    assert len(mus) == 1
    mu = np.array(mus[0])
    lam, gc, gP = adj.value_gradients(mdp, mu, V, w)
    h = 1e-6
    for s in range(4):
        for a in range(2):
            for j in range(4):
                Pp, Pm = P.copy(), P.copy()
                Pp[s, a, j] += h
                Pm[s, a, j] -= h
                Lp = w @ oracle.brute_force_optimum(oracle.DenseMDP(Pp, c, 0.8))[0]
                Lm = w @ oracle.brute_force_optimum(oracle.DenseMDP(Pm, c, 0.8))[0]
                assert abs((Lp - Lm) / (2 * h) - gP[s, a, j]) <= 1e-6


def test_adjoint_duality_and_dense_against_sparse():
    P, c = inputs.dense_mdp(60, 3, 1.0, 7, dtype=np.float64)
    dense = oracle.DenseMDP(P, c, 0.95)
    V, mu = _solve(dense)
    w = _w(60, 4)
    lam = adj.adjoint(dense, mu, w)
    c_mu = c[np.arange(60), mu]
    assert abs(lam @ c_mu - w @ V) <= 1e-10 * abs(w @ V) + 1e-12
    # the same MDP in CSR storage: sparse LU against LAPACK
    rp = np.arange(0, 60 * 3 * 60 + 1, 60, dtype=np.int64)
    col = np.tile(np.arange(60, dtype=np.int32), 60 * 3)
    csr = oracle.CsrMDP(rp, col, P.reshape(-1), c, 0.95)
    assert np.allclose(adj.adjoint(csr, mu, w), lam, rtol=1e-11, atol=1e-11)


def test_transpose_policy_rows_matches_scipy():
    import scipy.sparse as sp
    mdp = _csr(50, 4, 8, 13, 0.9)
    mu = np.random.Generator(np.random.Philox(5)).integers(0, 4, 50)
    rp, col, val = adj.transpose_policy_rows(mdp, mu)
    T = sp.csr_matrix((val, col, rp), shape=(50, 50)).toarray()
    ref = oracle.bellman._policy_matrix(mdp, mu).T.toarray()
    assert np.array_equal(T, ref)
    for j in range(50):
        assert np.all(np.diff(col[rp[j]:rp[j + 1]]) > 0)


def test_iterative_adjoint_matches_sparse_lu():
    mdp = _csr(500, 3, 10, 17, 0.98)
    mu = np.random.Generator(np.random.Philox(6)).integers(0, 3, 500)
    w = _w(500, 7)
    direct = adj.adjoint(mdp, mu, w)
    iterative = adj.adjoint(mdp, mu, w, iterative_tol=1e-13)
    assert np.max(np.abs(direct - iterative)) <= 1e-10 * np.max(np.abs(direct))


def test_dense_lu_adjoint_of_csr_storage():
    """The dense FP64 LU solve of a CSR MDP's adjoint equation against sparse
    LU and against the dense MDP's LAPACK solve (the same matrix), and
    against a planted transpose mistake (the non-transposed system)."""
    mdp = _csr(300, 4, 12, 19, 0.97)
    mu = np.random.Generator(np.random.Philox(8)).integers(0, 4, 300)
    w = _w(300, 9)
    lu = adj.adjoint(mdp, mu, w)
    dn = adj.adjoint(mdp, mu, w, dense=True)
    assert np.max(np.abs(dn - lu)) <= 1e-11 * np.max(np.abs(lu))
    Pm = oracle.bellman._policy_matrix(mdp, mu).toarray()
    wrong = np.linalg.solve(np.eye(300) - 0.97 * Pm, w)
    assert np.max(np.abs(wrong - dn)) > 1e-3 * np.max(np.abs(dn))
    # the defining equation, written out
    assert np.max(np.abs(dn - 0.97 * Pm.T @ dn - w)) <= 1e-11 * np.max(np.abs(dn))
