"""GPU parity at the benchmark's full sizes, in the launch configurations the
benchmark times.

* dense 8192 x 16 (4.3 GB, Dirichlet(0.1), gamma 0.99): one sweep at each
  benchmarked batch size against a full oracle sweep from the same seeded
  V; vi_solve and mpi_solve to eps = 1e-6 against J* from policy iteration.
* sparse 1M x 8, k = 32 (banded s +- 512 and uniform, gamma 0.995): one
  sweep at b = 4096, 65536 and n against a full oracle sweep; the solve's
  limit checked by the oracle's Bellman residual (a property that holds at
  any size), and J* itself to eps at n = 50000 with the same structure.

At n = 1M (banded) VI also reaches eps against J* from the oracle's policy
iteration (half a minute of host time).
"""
import time

import numpy as np
import pytest
import torch

import oracle
from paper_2110_02901_amd import binding as mb
from paper_2110_02901_amd import inputs

from gpu_util import csr_case, dense_case, dev, run_sweep, up

pytestmark = pytest.mark.gpu


def say(msg):
    print("[fullsize] " + msg, flush=True)


def out_tol(eps, Vstar):
    return eps + 0.5 * float(np.spacing(np.float32(np.max(np.abs(Vstar)))))


@pytest.fixture(scope="module")
def c2():
    wl = inputs.WORKLOADS["dense-8192x16"]
    t0 = time.time()
    P, c = inputs.dense_mdp(wl["n"], wl["m"], wl["alpha"], wl["data_seed"], dtype=np.float32)
    h, mdp = dense_case(P, c, wl["gamma"])
    say("dense-8192x16 generated and uploaded in %.1f s" % (time.time() - t0))
    t0 = time.time()
    Vstar, _, it = oracle.policy_iteration(mdp)
    say("oracle J* by policy iteration: %d iterations, %.1f s" % (it, time.time() - t0))
    return wl, h, mdp, Vstar


@pytest.mark.parametrize("b", [256, 1024, 8192])
def test_dense_8192x16_sweep(c2, b):
    wl, h, mdp, Vstar = c2
    V0 = inputs.values(wl["n"], 20, 5.8, 6.4)
    t0 = time.time()
    run_sweep(h, mdp, V0, b, wl["perm_seed"], 0, check_arg=(b == 1024))
    say("sweep b=%d checked in %.1f s" % (b, time.time() - t0))


@pytest.mark.parametrize("b", [256, 1024, 8192])
def test_dense_8192x16_vi_reaches_eps(c2, b):
    wl, h, mdp, Vstar = c2
    ws = mb.workspace(h, b)
    V = torch.zeros(wl["n"], dtype=torch.float32, device=dev())
    V64 = torch.zeros(wl["n"], dtype=torch.float64, device=dev())
    st = mb.vi_solve(h, V, b, wl["perm_seed"], ws, tol_dv=-1.0, eps=1e-6, V_ref=up(Vstar),
                     max_sweeps=5000, V64_out=V64)
    say("VI b=%d: %s" % (b, st))
    assert st["converged"]
    assert np.max(np.abs(V64.cpu().numpy() - Vstar)) <= 1e-6
    assert np.max(np.abs(V.cpu().numpy() - Vstar)) <= out_tol(1e-6, Vstar)


@pytest.mark.parametrize("b", [256, 1024, 8192])
def test_dense_8192x16_mpi_reaches_eps(c2, b):
    wl, h, mdp, Vstar = c2
    ws = mb.workspace(h, b)
    V = torch.zeros(wl["n"], dtype=torch.float32, device=dev())
    V64 = torch.zeros(wl["n"], dtype=torch.float64, device=dev())
    pol = torch.zeros(wl["n"], dtype=torch.int32, device=dev())
    st = mb.mpi_solve(h, V, pol, wl["K"], b, wl["perm_seed"], ws, policy_is_init=False,
                      tol_dv=-1.0, eps=1e-6, V_ref=up(Vstar), max_outer=5000, V64_out=V64)
    say("MPI K=5 b=%d: %s" % (b, st))
    assert st["converged"]
    assert np.max(np.abs(V64.cpu().numpy() - Vstar)) <= 1e-6
    assert np.max(np.abs(V.cpu().numpy() - Vstar)) <= out_tol(1e-6, Vstar)


@pytest.mark.parametrize("dtype", ["bf16", "fp8"])
def test_dense_8192x16_lowprec_sweep(c2, dtype):
    """BF16 / FP8 storage at full size: one sweep at b = 1024 against the
    oracle on the stored MDP (codes and scales from the oracle's quantiser;
    the library's codes must equal them)."""
    from oracle import quantize as qz
    wl, h32, mdp32, _ = c2
    n, m = wl["n"], wl["m"]
    P32 = mdp32.P.reshape(n * m, n)
    t0 = time.time()
    q_ref, s_ref = qz.quantize_rows(P32, dtype)
    q_gpu, s_gpu = mb.mdp_quantize_rows(up(P32), dtype)
    torch.cuda.synchronize()
    assert np.array_equal(q_gpu.cpu().numpy().view(q_ref.dtype), q_ref)
    assert np.all(np.abs(s_gpu.cpu().numpy() - s_ref) <= np.spacing(s_ref))
    h = mb.mdp_create_dense_q(q_gpu.reshape(-1), dtype, s_gpu, up(mdp32.c), wl["gamma"])
    mdp = oracle.DenseMDP(qz.dequantized(q_ref, s_ref, dtype).reshape(n, m, n), mdp32.c,
                          wl["gamma"])
    say("%s codes checked in %.1f s" % (dtype, time.time() - t0))
    V0 = inputs.values(n, 24, 5.8, 6.4)
    run_sweep(h, mdp, V0, 1024, wl["perm_seed"], 0, check_arg=False)


def _sparse(name):
    wl = inputs.WORKLOADS[name]
    t0 = time.time()
    rp, col, val, c = inputs.csr_mdp(wl["n"], wl["m"], wl["k"], wl["alpha"], wl["data_seed"],
                                     band=wl["band"])
    h, mdp = csr_case(rp, col, val, c, wl["gamma"])
    say("%s generated and uploaded in %.1f s; engine at b = 65536: %s"
        % (name, time.time() - t0, mb.mdp_engine(h, 65536)))
    return wl, h, mdp


@pytest.fixture(scope="module", params=["csr-1M-banded", "csr-1M-uniform"])
def c3(request):
    out = _sparse(request.param)
    yield out
    out[1].close()


@pytest.mark.parametrize("b", [4096, 65536, 1_000_000])
def test_sparse_1M_sweep(c3, b):
    wl, h, mdp = c3
    V0 = inputs.values(wl["n"], 21, 21.0, 23.0)
    t0 = time.time()
    run_sweep(h, mdp, V0, b, wl["perm_seed"], 0, check_arg=False)
    say("sweep b=%d checked in %.1f s" % (b, time.time() - t0))


def test_sparse_1M_policy_sweep(c3):
    wl, h, mdp = c3
    V0 = inputs.values(wl["n"], 22, 21.0, 23.0)
    run_sweep(h, mdp, V0, 65536, wl["perm_seed"], 1, policy=inputs.policy(wl["n"], wl["m"], 23))


@pytest.mark.parametrize("dtype", ["bf16", "fp8"])
def test_sparse_1M_lowprec_sweep(c3, dtype):
    from oracle import quantize as qz
    wl, h32, mdp32 = c3
    n, m, k = wl["n"], wl["m"], wl["k"]
    rows = mdp32.val.reshape(n * m, k)
    q_ref, s_ref = qz.quantize_rows(rows, dtype)
    q_gpu, s_gpu = mb.mdp_quantize_rows(up(rows), dtype)
    torch.cuda.synchronize()
    assert np.array_equal(q_gpu.cpu().numpy().view(q_ref.dtype), q_ref)
    h = mb.mdp_create_csr_q(up(mdp32.row_ptr), up(mdp32.col), q_gpu.reshape(-1), dtype, s_gpu,
                            up(mdp32.c), wl["gamma"])
    mdp = oracle.CsrMDP(mdp32.row_ptr, mdp32.col, qz.dequantized(q_ref, s_ref, dtype).reshape(-1),
                        mdp32.c, wl["gamma"])
    say("%s storage, engine at b = 65536: %s" % (dtype, mb.mdp_engine(h, 65536)))
    V0 = inputs.values(n, 25, 21.0, 23.0)
    run_sweep(h, mdp, V0, 65536, wl["perm_seed"], 0, check_arg=False)


def _certify(mdp, V64, gamma):
    """The oracle's Bellman residual of the solve's FP64 iterate, which
    certifies its accuracy at any size: max|V - J*| <= max|TV - V| / (1 -
    gamma) (contraction, Sec. III-B)."""
    Vg = V64.cpu().numpy()
    TV, _ = oracle.greedy(mdp, Vg)
    resid = float(np.max(np.abs(TV - Vg)))
    bound = resid / (1.0 - gamma)
    say("oracle residual %.3g -> certified max|V - J*| <= %.3g" % (resid, bound))
    return bound


@pytest.mark.parametrize("b", [4096, 65536, 1_000_000])
def test_sparse_1M_vi_certified_eps(c3, b):
    """MB-VI at each benchmarked b until max|dV| <= 1e-11, certified by the
    oracle's residual of the result."""
    wl, h, mdp = c3
    n = wl["n"]
    ws = mb.workspace(h, b)
    V = torch.zeros(n, dtype=torch.float32, device=dev())
    V64 = torch.zeros(n, dtype=torch.float64, device=dev())
    t0 = time.time()
    st = mb.vi_solve(h, V, b, wl["perm_seed"], ws, tol_dv=1e-11, max_sweeps=30000,
                     V64_out=V64)
    say("VI b=%d to max|dV| <= 1e-11: %s in %.1f s" % (b, st, time.time() - t0))
    assert st["converged"]
    assert _certify(mdp, V64, wl["gamma"]) <= 1e-6


def test_sparse_1M_mpi_certified_eps(c3):
    """MB-MPI (K = 5) at b = 65536 until the policy is stable and the
    residual of its improvement step is <= 1e-11, certified by the oracle's
    residual of the result."""
    wl, h, mdp = c3
    n, b = wl["n"], 65536
    ws = mb.workspace(h, b)
    V = torch.zeros(n, dtype=torch.float32, device=dev())
    V64 = torch.zeros(n, dtype=torch.float64, device=dev())
    pol = torch.zeros(n, dtype=torch.int32, device=dev())
    t0 = time.time()
    st = mb.mpi_solve(h, V, pol, 5, b, wl["perm_seed"], ws, policy_is_init=False, tol_dv=1e-11,
                      max_outer=10000, V64_out=V64)
    say("MPI K=5 b=%d: %s in %.1f s" % (b, st, time.time() - t0))
    assert st["converged"] and st["policy_changes_last"] == 0
    assert _certify(mdp, V64, wl["gamma"]) <= 1e-6


def test_sparse_50k_reaches_eps():
    """J* to eps = 1e-6 with the 1M workload's structure at n = 50000."""
    n, m, k = 50_000, 8, 32
    rp, col, val, c = inputs.csr_mdp(n, m, k, 1.0, 3, band=512)
    h, mdp = csr_case(rp, col, val, c, 0.995)
    t0 = time.time()
    Vstar, _, it = oracle.policy_iteration(mdp)
    say("oracle J* (n=50000): %d iterations, %.1f s" % (it, time.time() - t0))
    for b in (4096, n):
        ws = mb.workspace(h, b)
        V = torch.zeros(n, dtype=torch.float32, device=dev())
        V64 = torch.zeros(n, dtype=torch.float64, device=dev())
        st = mb.vi_solve(h, V, b, 103, ws, tol_dv=-1.0, eps=1e-6, V_ref=up(Vstar),
                         max_sweeps=20000, V64_out=V64)
        say("VI b=%d: %s" % (b, st))
        assert st["converged"]
        assert np.max(np.abs(V64.cpu().numpy() - Vstar)) <= 1e-6
        assert np.max(np.abs(V.cpu().numpy() - Vstar)) <= out_tol(1e-6, Vstar)


def test_sparse_1M_banded_reaches_eps_against_policy_iteration():
    """The full-size banded workload (10^6 states): VI at b = 65 536 to
    eps = 1e-6 against J* from the oracle's policy iteration (sparse
    iterative policy evaluation to 1e-14; about half a minute on the host)."""
    wl, h, mdp = _sparse("csr-1M-banded")
    Vstar, _, it = oracle.policy_iteration(mdp, iterative_tol=1e-14)
    ws = mb.workspace(h, 65536)
    V = torch.zeros(wl["n"], dtype=torch.float32, device=dev())
    st = mb.vi_solve(h, V, 65536, wl["perm_seed"], ws, tol_dv=-1.0, eps=1e-6, V_ref=up(Vstar),
                     max_sweeps=20000)
    assert st["converged"]
    assert np.max(np.abs(V.cpu().numpy() - Vstar)) <= out_tol(1e-6, Vstar)
