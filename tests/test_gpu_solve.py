"""GPU parity of the drivers (vi_solve, mpi_solve) against the oracle:
the limit J* (policy iteration on the stored MDP), the greedy policy (up to
near-ties), the first sweep that crosses eps in measurement mode, resuming
at a sweep index, and MPI's stopping rule."""
import numpy as np
import pytest
import torch

import oracle
from paper_2110_02901_amd import binding as mb
from paper_2110_02901_amd import inputs

from gpu_util import check_argmin, csr_case, dense_case, dev, up

pytestmark = pytest.mark.gpu


def out_tol(eps, Vstar):
    """eps plus half an FP32 ulp: the solve stops on the FP64 value W + r,
    and the returned V is that value rounded to FP32."""
    return eps + 0.5 * float(np.spacing(np.float32(np.max(np.abs(Vstar)))))


def zeros(n, dtype=torch.float32):
    return torch.zeros(n, dtype=dtype, device=dev())


def assert_optimal_policy(mdp, Vstar, pol, tol):
    Q = oracle.q_values(mdp, np.arange(mdp.n), Vstar)
    check_argmin(Q, pol, tol)


@pytest.fixture(scope="module")
def c1():
    # 64 states, 4 actions, Dirichlet(1) rows drawn in FP64, stored FP32
    P64, c64 = inputs.dense_mdp(64, 4, 1.0, 1, dtype=np.float64)
    P, c = P64.astype(np.float32), c64.astype(np.float32)
    h, mdp = dense_case(P, c, 0.9)
    Vstar, mustar, _ = oracle.policy_iteration(mdp)
    return h, mdp, Vstar


def test_vi_64x4_to_tolerance(c1):
    h, mdp, Vstar = c1
    ws = mb.workspace(h, 16)
    V = zeros(64)
    pol = torch.zeros(64, dtype=torch.int32, device=dev())
    st = mb.vi_solve(h, V, 16, 101, ws, tol_dv=1e-8, max_sweeps=5000, policy_out=pol)
    assert st["converged"] and st["final_dv_inf"] <= 1e-8
    Vg = V.cpu().numpy()
    assert np.max(np.abs(Vg - Vstar)) <= out_tol(1e-6, Vstar)
    assert_optimal_policy(mdp, Vstar, pol.cpu().numpy(), 1e-5 * np.max(np.abs(Vstar)))
    # The dV rule reads FP32 differences of W = V - R.  The anchor R absorbs
    # W whenever max|W| > 2^14 max|dW| (at most every 8 sweeps), so at the
    # stop max|W| <= 2^14 dV and the FP32 change is resolved to 2 ulp(W) <=
    # 2^-8 dV; the trajectory's rounding, contracted over 1 / (1 - rho)
    # sweeps (rho ~ 0.86 per sweep here), stays a few per cent of dV.  A
    # relative error delta moves the crossing of 1e-8 by at most
    # ceil(ln(1 + delta) / -ln(rho)) = 1 sweep; one more for the trajectory.
    _, _, ost = oracle.value_iteration(mdp, 16, 101, tol_dv=1e-8, max_sweeps=5000)
    assert abs(st["sweeps"] - ost.sweeps) <= 2, (st["sweeps"], ost.sweeps)


@pytest.mark.parametrize("b", [1, 16, 64])
def test_vi_first_crossing_matches_oracle(c1, b):
    h, mdp, Vstar = c1
    ws = mb.workspace(h, b)
    V = zeros(64)
    V64 = zeros(64, torch.float64)
    st = mb.vi_solve(h, V, b, 101, ws, tol_dv=-1.0, eps=1e-6, V_ref=up(Vstar), max_sweeps=5000,
                     V64_out=V64)
    _, _, ost = oracle.value_iteration(mdp, b, 101, tol_dv=-1, V_ref=Vstar, eps=1e-6)
    assert st["converged"] and st["final_err_ref"] <= 1e-6
    assert np.max(np.abs(V64.cpu().numpy() - Vstar)) <= 1e-6
    assert np.max(np.abs(V.cpu().numpy() - Vstar)) <= out_tol(1e-6, Vstar)
    assert abs(st["sweeps"] - ost.sweeps) <= 2, (st["sweeps"], ost.sweeps)


@pytest.mark.parametrize("b", [1, 16, 64])
def test_vi_tight_tolerance_beyond_fp32(c1, b):
    """With the FP64 anchor the iterate keeps converging far below FP32
    resolution of V: max|dV| <= 1e-12 certifies max|V - J*| <= 9e-12."""
    h, mdp, Vstar = c1
    ws = mb.workspace(h, b)
    V = zeros(64)
    V64 = zeros(64, torch.float64)
    st = mb.vi_solve(h, V, b, 101, ws, tol_dv=1e-12, max_sweeps=5000, V64_out=V64)
    assert st["converged"], st
    assert np.max(np.abs(V64.cpu().numpy() - Vstar)) <= 1e-11
    assert np.array_equal(V.cpu().numpy(), V64.cpu().numpy().astype(np.float32))


# "ell": the band-local engine; "ell-gather": the same MDP with V gathered
# from memory (band window off).
_ENGINE = {"dense": "dense", "ell": "ell-band", "ell-gather": "ell", "csr": "csr"}
_WINDOW = {"ell-gather": -1}


def _trajectory_case(storage):
    if storage == "dense":
        P, c = inputs.dense_mdp(1024, 16, 0.1, 2, dtype=np.float32)
        h, mdp = dense_case(P, c, 0.99)
    elif storage.startswith("ell"):
        rp, col, val, c = inputs.csr_mdp(3000, 8, 32, 1.0, 3, band=64)
        h, mdp = csr_case(rp, col, val, c, 0.995)
    else:
        rp, col, val, c = inputs.csr_ragged_mdp(500, 3, 1, 12, 1.0, 80)
        h, mdp = csr_case(rp, col, val, c, 0.95)
    _tune(h, storage)
    assert mb.mdp_engine(h, 37) == _ENGINE[storage]
    return h, mdp


def _tune(h, storage, **kw):
    mb.mdp_set_tuning(h, band_window=_WINDOW.get(storage, 0), **kw)


@pytest.mark.parametrize("storage,b", [("dense", 1024), ("dense", 100), ("dense", 7),
                                       ("ell", 3000), ("ell", 1000), ("ell", 37),
                                       ("ell-gather", 3000), ("ell-gather", 37),
                                       ("csr", 500), ("csr", 33)])
@pytest.mark.parametrize("anchor", [False, True])
def test_vi_trajectory_matches_oracle(storage, b, anchor):
    """Several sweeps in one launch against the oracle's MB-VI from the same
    seeded V0 and orders.  Every sweep boundary is crossed (the first batch
    of a sweep may hold states of the previous sweep's last batch, all of
    them when b = n); a lost or stale update there shows up as an error of
    the size of one sweep's change."""
    h, mdp = _trajectory_case(storage)
    n, T = mdp.n, 6
    _tune(h, storage, recentre_every=(1 if anchor else -1))
    try:
        V0 = inputs.values(n, 31, 0.0, 3.0)
        ws = mb.workspace(h, b)
        V = up(V0)
        V64 = zeros(n, torch.float64)
        st = mb.vi_solve(h, V, b, 55, ws, tol_dv=-1.0, max_sweeps=T, V64_out=V64)
        assert st["sweeps"] == T
        ref, _, _ = oracle.value_iteration(mdp, b, 55, V0=V0, tol_dv=-1, max_sweeps=T)
        scale = float(np.max(np.abs(ref)))
        assert np.max(np.abs(V64.cpu().numpy() - ref)) <= 1e-5 * scale
        assert np.max(np.abs(V.cpu().numpy() - ref)) <= 1e-5 * scale
    finally:
        _tune(h, storage)


@pytest.mark.parametrize("storage,b", [("dense", 1024), ("dense", 100), ("ell", 3000),
                                       ("ell", 37), ("ell-gather", 37), ("csr", 33)])
def test_vi_trajectory_with_recentring_every_sweep(storage, b):
    """Start next to J* and fold the iterate into the FP64 anchor after every
    sweep: the trajectory must still be the oracle's (which needs no
    re-centring in FP64)."""
    h, mdp = _trajectory_case(storage)
    n, T = mdp.n, 5
    Vstar, _, _ = oracle.policy_iteration(mdp)
    V0 = (Vstar + inputs.values(n, 33, -1e-3, 1e-3, dtype=np.float64)).astype(np.float32)
    _tune(h, storage, recentre_every=1, recentre_force=1)
    try:
        ws = mb.workspace(h, b)
        V = up(V0)
        V64 = zeros(n, torch.float64)
        st = mb.vi_solve(h, V, b, 57, ws, tol_dv=-1.0, max_sweeps=T, V64_out=V64)
        assert st["recentrings"] == T - 1, st
        ref, _, _ = oracle.value_iteration(mdp, b, 57, V0=V0, tol_dv=-1, max_sweeps=T)
        # A lost update or a wrong shift would be as large as the change
        # itself; FP32 rounding of the first sweep (before the first fold,
        # on W ~ V0) stays near 1e-7 * max|V|.
        change = float(np.max(np.abs(ref - V0)))
        assert np.max(np.abs(V64.cpu().numpy() - ref)) <= 1e-2 * change
    finally:
        _tune(h, storage)


@pytest.mark.parametrize("storage,b", [("dense", 1024), ("dense", 100), ("ell", 3000),
                                       ("ell", 37), ("ell-gather", 3000), ("ell-gather", 37),
                                       ("csr", 33)])
def test_mpi_trajectory_matches_oracle(storage, b):
    """Three outer iterations of MB-MPI (K = 2) in one launch against the
    oracle: values and policies after the last improvement."""
    h, mdp = _trajectory_case(storage)
    n = mdp.n
    V0 = inputs.values(n, 32, 0.0, 3.0)
    ws = mb.workspace(h, b)
    V = up(V0)
    pol = torch.zeros(n, dtype=torch.int32, device=dev())
    st = mb.mpi_solve(h, V, pol, 2, b, 56, ws, policy_is_init=False, tol_dv=-1.0, max_outer=3)
    assert st["sweeps"] == 6 and st["outer_iters"] == 3
    ref, mu, _ = oracle.modified_policy_iteration(mdp, 2, b, 56, V0=V0, tol_dv=-1, max_outer=3)
    scale = float(np.max(np.abs(ref)))
    assert np.max(np.abs(V.cpu().numpy() - ref)) <= 1e-5 * scale
    Q = oracle.q_values(mdp, np.arange(n), ref)
    check_argmin(Q, pol.cpu().numpy(), 1e-5 * scale)


def test_vi_resume_reproduces_uninterrupted_run(c1):
    h, mdp, _ = c1
    mb.mdp_set_tuning(h, recentre_every=-1)
    try:
        ws = mb.workspace(h, 16)
        full = zeros(64)
        mb.vi_solve(h, full, 16, 7, ws, max_sweeps=20)
        part = zeros(64)
        mb.vi_solve(h, part, 16, 7, ws, max_sweeps=12)
        mb.vi_solve(h, part, 16, 7, ws, first_sweep=12, max_sweeps=8)
        assert torch.equal(full, part)
    finally:
        mb.mdp_set_tuning(h)


def test_vi_not_converged_is_soft(c1):
    h, _, _ = c1
    ws = mb.workspace(h, 16)
    V = zeros(64)
    st = mb.vi_solve(h, V, 16, 1, ws, tol_dv=0.0, max_sweeps=3)
    assert not st["converged"] and st["sweeps"] == 3


@pytest.mark.parametrize("K,b,init", [(5, 16, False), (1, 64, False), (5, 1, True)])
def test_mpi_64x4(c1, K, b, init):
    h, mdp, Vstar = c1
    ws = mb.workspace(h, b)
    V = zeros(64)
    pol = up(inputs.policy(64, 4, 3)) if init else torch.zeros(64, dtype=torch.int32, device=dev())
    st = mb.mpi_solve(h, V, pol, K, b, 101, ws, policy_is_init=init, tol_dv=1e-7,
                      max_outer=2000)
    assert st["converged"] and st["policy_changes_last"] == 0
    assert np.max(np.abs(V.cpu().numpy() - Vstar)) <= out_tol(1e-6, Vstar)
    assert_optimal_policy(mdp, Vstar, pol.cpu().numpy(), 1e-5 * np.max(np.abs(Vstar)))


def test_mpi_first_crossing_matches_oracle(c1):
    h, mdp, Vstar = c1
    ws = mb.workspace(h, 16)
    V = zeros(64)
    pol = torch.zeros(64, dtype=torch.int32, device=dev())
    st = mb.mpi_solve(h, V, pol, 5, 16, 101, ws, policy_is_init=False, tol_dv=-1.0, eps=1e-6,
                      V_ref=up(Vstar), max_outer=2000)
    _, _, ost = oracle.modified_policy_iteration(mdp, 5, 16, 101, tol_dv=-1, V_ref=Vstar,
                                                 eps=1e-6)
    assert st["converged"] and abs(st["sweeps"] - ost.sweeps) <= 2, (st, ost)


@pytest.fixture(scope="module")
def dense_1024():
    P, c = inputs.dense_mdp(1024, 16, 0.1, 2, dtype=np.float32)
    h, mdp = dense_case(P, c, 0.99)
    Vstar, _, _ = oracle.policy_iteration(mdp)
    return h, mdp, Vstar


@pytest.mark.parametrize("b", [1024, 128, 32])
def test_vi_dense_1024x16_reaches_eps(dense_1024, b):
    """gamma = 0.99 and V* ~ 6: eps = 1e-6 needs the re-centred iterate."""
    h, mdp, Vstar = dense_1024
    ws = mb.workspace(h, b)
    V = zeros(1024)
    V64 = zeros(1024, torch.float64)
    pol = torch.zeros(1024, dtype=torch.int32, device=dev())
    st = mb.vi_solve(h, V, b, 102, ws, tol_dv=-1.0, eps=1e-6, V_ref=up(Vstar),
                     max_sweeps=4000, policy_out=pol, V64_out=V64)
    assert st["converged"], st
    assert np.max(np.abs(V64.cpu().numpy() - Vstar)) <= 1e-6
    assert np.max(np.abs(V.cpu().numpy() - Vstar)) <= out_tol(1e-6, Vstar)
    assert st["recentrings"] >= 1
    # the same orders in FP64 cross eps within a few sweeps of the GPU
    _, _, ost = oracle.value_iteration(mdp, b, 102, tol_dv=-1, V_ref=Vstar, eps=1e-6)
    assert abs(st["sweeps"] - ost.sweeps) <= 3, (st["sweeps"], ost.sweeps)
    assert_optimal_policy(mdp, Vstar, pol.cpu().numpy(), 1e-5 * np.max(np.abs(Vstar)))


def test_mpi_dense_1024x16_reaches_eps(dense_1024):
    h, mdp, Vstar = dense_1024
    ws = mb.workspace(h, 128)
    V = zeros(1024)
    pol = torch.zeros(1024, dtype=torch.int32, device=dev())
    st = mb.mpi_solve(h, V, pol, 5, 128, 102, ws, policy_is_init=False, tol_dv=-1.0, eps=1e-6,
                      V_ref=up(Vstar), max_outer=2000)
    assert st["converged"], st
    assert np.max(np.abs(V.cpu().numpy() - Vstar)) <= out_tol(1e-6, Vstar)


@pytest.mark.parametrize("window", [0, -1])
@pytest.mark.parametrize("band", [64, None])
def test_vi_and_mpi_sparse_reach_eps(band, window):
    n, m, k = 3000, 8, 32
    rp, col, val, c = inputs.csr_mdp(n, m, k, 1.0, 3, band=band)
    h, mdp = csr_case(rp, col, val, c, 0.995)
    mb.mdp_set_tuning(h, band_window=window)
    Vstar, _, _ = oracle.policy_iteration(mdp)
    for b in (3000, 300):
        ws = mb.workspace(h, b)
        V = zeros(n)
        pol = torch.zeros(n, dtype=torch.int32, device=dev())
        st = mb.vi_solve(h, V, b, 103, ws, tol_dv=-1.0, eps=1e-6, V_ref=up(Vstar),
                         max_sweeps=20000, policy_out=pol)
        assert st["converged"], st
        assert np.max(np.abs(V.cpu().numpy() - Vstar)) <= out_tol(1e-6, Vstar)
        assert_optimal_policy(mdp, Vstar, pol.cpu().numpy(), 1e-5 * np.max(np.abs(Vstar)))
    ws = mb.workspace(h, 300)
    V = zeros(n)
    pol = torch.zeros(n, dtype=torch.int32, device=dev())
    st = mb.mpi_solve(h, V, pol, 5, 300, 103, ws, policy_is_init=False, tol_dv=-1.0, eps=1e-6,
                      V_ref=up(Vstar), max_outer=20000)
    assert st["converged"], st


def test_general_csr_vi():
    n, m = 500, 3
    rp, col, val, c = inputs.csr_ragged_mdp(n, m, 1, 12, 1.0, 80)
    h, mdp = csr_case(rp, col, val, c, 0.95)
    Vstar, _, _ = oracle.policy_iteration(mdp)
    ws = mb.workspace(h, 50)
    V = zeros(n)
    st = mb.vi_solve(h, V, 50, 3, ws, tol_dv=-1.0, eps=1e-6, V_ref=up(Vstar), max_sweeps=5000)
    assert st["converged"] and np.max(np.abs(V.cpu().numpy() - Vstar)) <= out_tol(1e-6, Vstar)
