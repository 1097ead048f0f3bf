"""GPU parity of the differentiation extension against the oracle: the
transposed policy rows, the adjoint lambda = (I - gamma P_mu)^-T w from the
mini-batch sweep on the transpose, the gradients of L = w^T J* with respect
to the costs and the stored transition values, and the torch autograd
wrapper against central finite differences of the oracle's J*."""
import time

import numpy as np
import pytest
import torch

import oracle
from oracle import adjoint as adj
from paper_2110_02901_amd import binding as mb
from paper_2110_02901_amd import inputs
from paper_2110_02901_amd.autograd import OptimalValue

from gpu_util import dev, up

pytestmark = pytest.mark.gpu


def say(msg):
    print("[adjoint] " + msg, flush=True)


def case(n, m, k, seed, gamma, band=None):
    rp, col, val, c = inputs.csr_mdp(n, m, k, 1.0, seed, band=band)
    mdp = oracle.CsrMDP(rp, col, val, c, gamma)
    return rp, col, val, c, mdp


def solve_gpu(h, n, b, tol=1e-11):
    ws = mb.workspace(h, b)
    V = torch.zeros(n, dtype=torch.float32, device=dev())
    V64 = torch.zeros(n, dtype=torch.float64, device=dev())
    pol = torch.zeros(n, dtype=torch.int32, device=dev())
    st = mb.mpi_solve(h, V, pol, 5, b, 3, ws, policy_is_init=False, tol_dv=tol, max_outer=100000,
                      V64_out=V64)
    assert st["converged"], st
    return V64, pol, ws


@pytest.mark.parametrize("band", [None, 40])
def test_policy_transpose_matches_oracle(band):
    n, m, k = 900, 3, 12
    rp, col, val, c, mdp = case(n, m, k, 21, 0.95, band)
    h = mb.mdp_create_csr(up(rp), up(col), up(val), up(c), 0.95)
    mu = inputs.policy(n, m, 22)
    rp_t, col_t, val_t = mb.mdp_policy_transpose(h, up(mu), k, mb.workspace(h, 1))
    r_ref, c_ref, v_ref = adj.transpose_policy_rows(mdp, mu)
    assert np.array_equal(rp_t.cpu().numpy(), r_ref)
    assert np.array_equal(col_t.cpu().numpy(), c_ref)
    assert np.array_equal(val_t.cpu().numpy(), v_ref)
    # a policy entry out of range is an argument error, read nowhere
    bad = mu.copy()
    bad[5] = m
    with pytest.raises(mb.MbdpError) as e:
        mb.mdp_policy_transpose(h, up(bad), k, mb.workspace(h, 1))
    assert e.value.status == mb.MBDP_ERR_INVALID_ARG


@pytest.mark.parametrize("b_frac", [1, 8])
def test_adjoint_and_gradients_match_oracle(b_frac):
    n, m, k, gamma = 2000, 4, 16, 0.98
    rp, col, val, c, mdp = case(n, m, k, 23, gamma)
    h = mb.mdp_create_csr(up(rp), up(col), up(val), up(c), gamma)
    b = n // b_frac
    V64, pol, ws = solve_gpu(h, n, b)
    Vs, mus, _ = oracle.policy_iteration(mdp, improve_tol=1e-14)
    assert np.array_equal(pol.cpu().numpy(), mus)
    w = np.random.Generator(np.random.Philox(24)).standard_normal(n)
    lam_ref, gc_ref, gv_ref = adj.value_gradients(mdp, mus, Vs, w)
    # the adjoint by the mini-batch sweep on the transpose
    rp_t, col_t, val_t = mb.mdp_policy_transpose(h, pol, k, ws)
    h_t = mb.mdp_create_csr(rp_t, col_t, val_t, up(w.astype(np.float32).reshape(n, 1)), gamma)
    ws_t = mb.workspace(h_t, b)
    lam32 = torch.zeros(n, dtype=torch.float32, device=dev())
    lam = torch.zeros(n, dtype=torch.float64, device=dev())
    st = mb.vi_solve(h_t, lam32, b, 5, ws_t, tol_dv=1e-11, max_sweeps=200000, V64_out=lam)
    assert st["converged"], st
    say("adjoint sweep b=%d: %s" % (b, st))
    # reference adjoint for the FP32-rounded right-hand side the GPU solved
    lam_w32 = adj.adjoint(mdp, mus, w.astype(np.float32).astype(np.float64))
    scale = float(np.max(np.abs(lam_w32)))
    assert np.max(np.abs(lam.cpu().numpy() - lam_w32)) <= 1e-6 * scale
    assert np.max(np.abs(lam_w32 - lam_ref)) <= 1e-6 * scale
    gc, gv = mb.mdp_value_gradients(h, pol, lam, V64, ws, k=k)
    gc = gc.cpu().numpy().reshape(n, m)
    gv = gv.cpu().numpy()
    assert np.max(np.abs(gc - gc_ref)) <= 2e-6 * scale
    assert np.max(np.abs(gv - gv_ref)) <= 2e-6 * scale * float(np.max(np.abs(Vs)))
    off = np.ones((n, m), dtype=bool)
    off[np.arange(n), mus] = False
    assert np.all(gc[off] == 0.0)


def _oracle_L(rp, col, val, c, gamma, w, iterative_tol=None):
    V, _, _ = oracle.policy_iteration(oracle.CsrMDP(rp, col, val, c, gamma), improve_tol=1e-14,
                                      iterative_tol=iterative_tol)
    return float(w @ V)


def _clear_states(mdp, n_pick, seed, gap=1e-2, iterative_tol=None):
    """States whose best action wins by more than `gap` (finite differences
    of size 1e-4 there cannot switch the optimal policy)."""
    V, _, _ = oracle.policy_iteration(mdp, improve_tol=1e-14, iterative_tol=iterative_tol)
    Q = oracle.q_values(mdp, np.arange(mdp.n), V)
    srt = np.sort(Q, axis=1)
    ok = np.flatnonzero(srt[:, 1] - srt[:, 0] > gap)
    return np.random.Generator(np.random.Philox(seed)).choice(ok, n_pick, replace=False)


def test_autograd_against_finite_differences():
    n, m, k, gamma = 300, 3, 8, 0.95
    rp, col, val, c, mdp = case(n, m, k, 25, gamma)
    w = np.random.Generator(np.random.Philox(26)).standard_normal(n)
    probes = _clear_states(mdp, 8, 27)
    c_t = up(c).requires_grad_(True)
    v_t = up(val).requires_grad_(True)
    J = OptimalValue.apply(c_t, v_t, up(rp), up(col), gamma, n // 4, 7, 1e-11, 5)
    L = (J * up(w)).sum()
    L.backward()
    gc = c_t.grad.cpu().numpy().astype(np.float64)
    gv = v_t.grad.cpu().numpy().astype(np.float64)
    c64, v64 = c.astype(np.float64), val.astype(np.float64)
    h = 1e-4
    for s in probes[:5]:
        for a in range(m):
            cp, cm = c64.copy(), c64.copy()
            cp[s, a] += h
            cm[s, a] -= h
            fd = (_oracle_L(rp, col, v64, cp, gamma, w) - _oracle_L(rp, col, v64, cm, gamma, w)) / (2 * h)
            assert abs(fd - gc[s, a]) <= 1e-5 * max(1.0, abs(fd)), (s, a, fd, gc[s, a])
    for s in probes[5:]:
        r = s * m + int(np.argmin(oracle.q_values(mdp, [s], _oracle_V(mdp))[0]))
        e = int(rp[r]) + 3  # an entry of the state's optimal row (and one of another row)
        e2 = int(rp[s * m + (r - s * m + 1) % m]) + 2
        for e in (e, e2):
            vp, vm = v64.copy(), v64.copy()
            vp[e] += h
            vm[e] -= h
            fd = (_oracle_L(rp, col, vp, c64, gamma, w) -
                  _oracle_L(rp, col, vm, c64, gamma, w)) / (2 * h)
            assert abs(fd - gv[e]) <= 1e-5 * max(1.0, abs(fd)), (e, fd, gv[e])


def _oracle_V(mdp):
    return oracle.policy_iteration(mdp, improve_tol=1e-14)[0]


def test_adjoint_at_the_differentiation_workload():
    """n = 16384, m = 8, k = 64 uniform successors, Dirichlet(1), gamma 0.98,
    L = w^T J* with w ~ N(0, 1): gradients against the oracle's sparse-LU
    adjoint on every entry and against central differences on a few."""
    n, m, k, gamma = 16384, 8, 64, 0.98
    rp, col, val, c, mdp = case(n, m, k, 5, gamma)
    w = np.random.Generator(np.random.Philox(28)).standard_normal(n)
    c_t = up(c).requires_grad_(True)
    v_t = up(val).requires_grad_(True)
    torch.cuda.synchronize()
    t0 = time.time()
    J = OptimalValue.apply(c_t, v_t, up(rp), up(col), gamma, n, 7, 1e-11, 5)
    torch.cuda.synchronize()
    t1 = time.time()
    (J * up(w)).sum().backward()
    torch.cuda.synchronize()
    t2 = time.time()
    say("n=16384 forward (MB-MPI to 1e-11) %.1f ms, backward (transpose + adjoint sweep + "
        "gradients) %.1f ms" % ((t1 - t0) * 1e3, (t2 - t1) * 1e3))
    # the oracle with iterative solves (random sparse rows fill in under LU)
    t0 = time.time()
    Vs, mus, _ = oracle.policy_iteration(mdp, improve_tol=1e-14, iterative_tol=1e-14)
    say("oracle J* in %.1f s" % (time.time() - t0))
    assert np.max(np.abs(J.detach().cpu().numpy() - Vs)) <= 1e-8
    lam, gc_ref, gv_ref = adj.value_gradients(mdp, mus, Vs, w, iterative_tol=1e-14)
    say("oracle gradients in %.1f s" % (time.time() - t0))
    scale = float(np.max(np.abs(lam)))
    gc = c_t.grad.cpu().numpy().astype(np.float64)
    gv = v_t.grad.cpu().numpy().astype(np.float64)
    err_c = float(np.max(np.abs(gc - gc_ref)))
    err_v = float(np.max(np.abs(gv - gv_ref)))
    say("max |dL/dc - oracle| = %.3g, max |dL/dP - oracle| = %.3g (max |lambda| %.3g)"
        % (err_c, err_v, scale))
    assert err_c <= 1e-5 * scale
    assert err_v <= 1e-5 * scale * float(np.max(np.abs(Vs)))
    # and against the dense FP64 linear solve of the adjoint equation (LU of the
    # 16384 x 16384 matrix (I - gamma P_mu)^T)
    t0 = time.time()
    lam_d, gc_d, gv_d = adj.value_gradients(mdp, mus, Vs, w, dense=True)
    say("dense FP64 LU adjoint in %.1f s: max |lambda_dense - lambda_iterative| = %.3g"
        % (time.time() - t0, float(np.max(np.abs(lam_d - lam)))))
    assert np.max(np.abs(lam_d - lam)) <= 1e-10 * scale
    assert np.max(np.abs(gc - gc_d)) <= 1e-5 * scale
    assert np.max(np.abs(gv - gv_d)) <= 1e-5 * scale * float(np.max(np.abs(Vs)))
    h = 1e-4
    c64, v64 = c.astype(np.float64), val.astype(np.float64)
    for s in _clear_states(mdp, 2, 29, iterative_tol=1e-14):
        a = int(mus[s])
        cp, cm = c64.copy(), c64.copy()
        cp[s, a] += h
        cm[s, a] -= h
        fd = (_oracle_L(rp, col, v64, cp, gamma, w, 1e-14) -
              _oracle_L(rp, col, v64, cm, gamma, w, 1e-14)) / (2 * h)
        say("central difference at state %d: %.6g vs %.6g" % (s, fd, gc[s, a]))
        assert abs(fd - gc[s, a]) <= 1e-4 * max(1.0, abs(fd)), (s, a, fd, gc[s, a])
