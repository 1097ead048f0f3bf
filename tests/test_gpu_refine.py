"""GPU parity of the certified FP64 correction (mdp_refine) against the
oracle's ``certified_correction`` (sweeps of B_{sigma_t,b}, K = 0) and
``certified_correction_mpi`` (Algorithm 1, K >= 1).

The correction starts where it is used: at J* of the BF16 / FP8-stored MDP
(the oracle's policy iteration on P' built from the oracle's own codes), or
at a seeded perturbation of the FP32 MDP's J*.  From the same input, both
sides do the same FP64 steps, so the GPU must match the oracle element by
element up to FP64 summation order: the input residual, the number of
sweeps and improvement steps (the same stop rule on the same quantities),
the output V, its certified bound and residual, and the greedy policy.  The
output is then checked against J* of the FP32 MDP itself: max|V - J*| <=
bound <= eps.  At the full 8192 x 16 size the first sweep is compared with
an oracle sweep from the same input and the limit by its properties.
"""
import time

import numpy as np
import pytest
import torch

import oracle
from oracle import quantize as qz
from oracle.refine import certified_correction, certified_correction_mpi
from paper_2110_02901_amd import binding as mb
from paper_2110_02901_amd import inputs

from gpu_util import check_argmin, csr_case, dense_case, dev, up

pytestmark = pytest.mark.gpu

# FP64 on both sides, summed in different orders: a backup differs by a few
# units of 2^-53 max|V| per term level; the contraction keeps the sum of
# these over a correction below ~1e-12 max|V| at these sizes.
V_ATOL = 1e-10
RES_ATOL = 1e-12


def say(msg):
    print("[refine] " + msg, flush=True)


def stored_solution(mdp32, dtype, rows_shape):
    """J* of the BF16 / FP8-stored MDP (oracle codes, oracle policy iteration)."""
    rows = (mdp32.P.reshape(rows_shape) if isinstance(mdp32, oracle.DenseMDP)
            else mdp32.val.reshape(rows_shape))
    q, s = qz.quantize_rows(rows.astype(np.float32), dtype)
    vp = qz.dequantized(q, s, dtype)
    if isinstance(mdp32, oracle.DenseMDP):
        mdpq = oracle.DenseMDP(vp.reshape(mdp32.P.shape), mdp32.c, mdp32.gamma)
    else:
        mdpq = oracle.CsrMDP(mdp32.row_ptr, mdp32.col, vp.reshape(-1), mdp32.c, mdp32.gamma)
    Vq, _, _ = oracle.policy_iteration(mdpq)
    return Vq


def run_refine(h, mdp, V0, K, b, seed, eps, V_ref=None, first_sweep=0, max_iters=100000,
               want_policy=True):
    ws = mb.workspace(h, b)
    V = up(np.asarray(V0, dtype=np.float64))
    pol = torch.full((mdp.n,), -1, dtype=torch.int32, device=dev()) if want_policy else None
    st = mb.mdp_refine(h, V, b, seed, ws, K=K, eps=eps,
                       V_ref=None if V_ref is None else up(V_ref), first_sweep=first_sweep,
                       max_iters=max_iters, policy_out=pol)
    return V.cpu().numpy(), (pol.cpu().numpy() if want_policy else None), st


def oracle_refine(mdp, V0, K, b, seed, eps, V_ref=None, first_sweep=0, max_iters=100000):
    if K == 0:
        return certified_correction(mdp, V0, b, seed, eps, first_sweep=first_sweep,
                                    max_sweeps=max_iters, V_ref=V_ref)
    return certified_correction_mpi(mdp, V0, K, b, seed, eps, first_sweep=first_sweep,
                                    max_outer=max_iters, V_ref=V_ref)


def compare(mdp, V0, K, b, seed, eps, Vstar=None, V_ref=None, first_sweep=0, max_iters=100000):
    """Runs both sides from V0 and checks every output; returns the GPU stats."""
    t0 = time.time()
    Vg, pg, st = run_refine(mdp.h, mdp, V0, K, b, seed, eps, V_ref, first_sweep, max_iters)
    t1 = time.time()
    Vo, po, so = oracle_refine(mdp, V0, K, b, seed, eps, V_ref, first_sweep, max_iters)
    say("n=%d K=%d b=%d: GPU %s (%.2f s); oracle sweeps %d outer %d (%.2f s)"
        % (mdp.n, K, b, st, t1 - t0, so.sweeps, so.outer_iters, time.time() - t1))
    scale = max(1.0, float(np.max(np.abs(Vo))))
    assert abs(st["residual_in"] - so.residual_in) <= RES_ATOL * scale
    assert st["sweeps"] == so.sweeps
    assert st["outer_iters"] == so.outer_iters
    assert bool(st["converged"]) == so.converged
    assert np.max(np.abs(Vg - Vo)) <= V_ATOL * scale
    assert abs(st["residual_out"] - so.residual_out) <= RES_ATOL * scale
    # the bounds are the residual (K >= 1) or the last sweep's change (K = 0)
    # times 1 / (1 - gamma) or gamma / (1 - gamma): their tolerance is the
    # residual's, amplified by that factor (twice it for a difference of Vs)
    g = mdp.gamma
    if K == 0:
        tol_b = 2 * RES_ATOL * scale * g / (1 - g)
        assert abs(st["bound_out"] - so.bound_out) <= tol_b
        if so.sweeps:
            assert abs(st["final_dv_inf"] - so.final_dv_inf) <= 2 * RES_ATOL * scale
    else:
        assert abs(st["bound_out"] - so.bound_out) <= RES_ATOL * scale / (1 - g)
    if V_ref is not None:
        assert st["final_err_ref"] == pytest.approx(so.final_err_ref, rel=1e-9, abs=1e-13)
    Q = oracle.q_values(mdp, np.arange(mdp.n), Vo)
    check_argmin(Q, pg, 1e-9 * scale)
    if Vstar is not None and so.converged:
        err = float(np.max(np.abs(Vg - Vstar)))
        assert err <= st["bound_out"] * (1 + 1e-9) + 1e-12
        if V_ref is None:
            assert st["bound_out"] <= eps
        else:
            assert err <= eps
    return st


class Case:
    """GPU handle + oracle MDP of one FP32 MDP, with its J*."""

    def __init__(self, h, mdp, Vstar=None):
        self.h, self.mdp, self.Vstar = h, mdp, Vstar
        mdp.h = h


@pytest.fixture(scope="module")
def dense1024():
    P, c = inputs.dense_mdp(1024, 16, 0.1, 2, dtype=np.float32)
    h, mdp = dense_case(P, c, 0.99)
    Vstar, _, _ = oracle.policy_iteration(mdp)
    return Case(h, mdp, Vstar)


@pytest.mark.parametrize("dtype", ["bf16", "fp8"])
@pytest.mark.parametrize("K,b", [(0, 256), (5, 256), (0, 1024), (3, 77)])
def test_dense_from_stored_solution(dense1024, dtype, K, b):
    cs = dense1024
    V0 = stored_solution(cs.mdp, dtype, (1024 * 16, 1024))
    say("%s: max|J*(stored) - J*| = %.3g" % (dtype, float(np.max(np.abs(V0 - cs.Vstar)))))
    compare(cs.mdp, V0, K, b, 401, 1e-6, Vstar=cs.Vstar, first_sweep=3)


def test_dense_measurement_mode(dense1024):
    cs = dense1024
    V0 = stored_solution(cs.mdp, "bf16", (1024 * 16, 1024))
    for K in (0, 5):
        compare(cs.mdp, V0, K, 512, 402, 1e-6, Vstar=cs.Vstar, V_ref=cs.Vstar)


def test_certified_input_is_returned_unchanged(dense1024):
    cs = dense1024
    Vg, _, st = run_refine(cs.h, cs.mdp, cs.Vstar, 0, 256, 1, 1e-6)
    assert st["converged"] and st["sweeps"] == 0 and st["outer_iters"] == 0
    assert np.array_equal(Vg, cs.Vstar)
    assert st["residual_out"] == st["residual_in"]
    assert st["bound_out"] == pytest.approx(st["residual_in"] / (1 - 0.99), rel=1e-12)


def test_dense_ragged_width_and_limit():
    """n not a multiple of 4 (scalar row loads), m > 8 rows per pass, and a
    sweep limit that stops the correction before it certifies."""
    P, c = inputs.dense_mdp(999, 11, 0.5, 7, dtype=np.float32)
    h, mdp = dense_case(P, c, 0.95)
    cs = Case(h, mdp)
    V0 = inputs.values(999, 60, 0.0, 15.0).astype(np.float64)
    st = compare(mdp, V0, 0, 100, 403, 1e-9, max_iters=7)
    assert not st["converged"] and st["sweeps"] == 7
    compare(mdp, V0, 2, 999, 404, 1e-9, max_iters=4)
    Vstar, _, _ = oracle.policy_iteration(mdp)
    V1 = Vstar + inputs.values(999, 64, -1e-3, 1e-3).astype(np.float64)
    compare(mdp, V1, 0, 1, 405, 1e-7, Vstar=Vstar)
    del cs


def test_dense_wider_than_lds_stage():
    """n > 8192: V is read from memory instead of the LDS stage."""
    P, c = inputs.dense_mdp(8200, 2, 1.0, 8, dtype=np.float32)
    h, mdp = dense_case(P, c, 0.9)
    Case(h, mdp)
    V0 = inputs.values(8200, 61, 0.0, 10.0).astype(np.float64)
    compare(mdp, V0, 0, 4100, 406, 0.0, max_iters=3)
    compare(mdp, V0, 1, 999, 407, 0.0, max_iters=2)


@pytest.fixture(scope="module", params=[64, None], ids=["banded", "uniform"])
def ell3000(request):
    rp, col, val, c = inputs.csr_mdp(3000, 8, 32, 1.0, 3, band=request.param)
    h, mdp = csr_case(rp, col, val, c, 0.98)
    Vstar, _, _ = oracle.policy_iteration(mdp)
    return Case(h, mdp, Vstar)


@pytest.mark.parametrize("dtype,K,b", [("bf16", 0, 3000), ("fp8", 0, 500), ("fp8", 5, 300),
                                       ("bf16", 2, 60)])
def test_ell_from_stored_solution(ell3000, dtype, K, b):
    cs = ell3000
    V0 = stored_solution(cs.mdp, dtype, (3000 * 8, 32))
    say("%s: max|J*(stored) - J*| = %.3g" % (dtype, float(np.max(np.abs(V0 - cs.Vstar)))))
    compare(cs.mdp, V0, K, b, 408, 1e-6, Vstar=cs.Vstar)


@pytest.mark.parametrize("K", [0, 3])
def test_csr_ragged_rows(K):
    rp, col, val, c = inputs.csr_ragged_mdp(700, 3, 1, 70, 1.0, 81)
    h, mdp = csr_case(rp, col, val, c, 0.97)
    Vstar, _, _ = oracle.policy_iteration(mdp)
    Case(h, mdp, Vstar)
    V0 = Vstar + inputs.values(700, 62, -1e-3, 1e-3).astype(np.float64)
    compare(mdp, V0, K, 64, 409, 1e-8, Vstar=Vstar)


def test_rejections():
    P, c = inputs.dense_mdp(64, 4, 1.0, 1, dtype=np.float32)
    h, mdp = dense_case(P, c, 0.9)
    ws = mb.workspace(h, 16)
    V = torch.zeros(64, dtype=torch.float64, device=dev())
    for kw in (dict(K=-1), dict(eps=-1.0), dict(max_iters=-1)):
        with pytest.raises(mb.MbdpError) as e:
            mb.mdp_refine(h, V, 16, 1, ws, **kw)
        assert e.value.status == mb.MBDP_ERR_INVALID_ARG
    with pytest.raises(mb.MbdpError) as e:
        mb.mdp_refine(h, V, 65, 1, ws)
    assert e.value.status == mb.MBDP_ERR_INVALID_ARG
    q, s = mb.mdp_quantize_rows(up(P.reshape(256, 64)), "bf16")
    hq = mb.mdp_create_dense_q(q.reshape(-1), "bf16", s, up(c), 0.9)
    with pytest.raises(mb.MbdpError) as e:
        mb.mdp_refine(hq, V, 16, 1, mb.workspace(hq, 16))
    assert e.value.status == mb.MBDP_ERR_UNSUPPORTED


# ------------------------------------------------------------ full size

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


@pytest.mark.parametrize("K", [0, 5])
def test_dense_8192x16_full_size(c2, K):
    """From J* plus a seeded error of the size BF16 storage leaves (2e-5), at
    the benchmark's b = 1024: the input residual and the first sweep against
    the oracle from the same input, then the certified limit against J*."""
    wl, h, mdp, Vstar = c2
    n, b, seed = wl["n"], 1024, wl["perm_seed"]
    V0 = Vstar + inputs.values(n, 63, -2e-5, 2e-5).astype(np.float64)
    t0 = time.time()
    Vg, _, st1 = run_refine(h, mdp, V0, K, b, seed, 0.0, max_iters=1, want_policy=False)
    TV, _ = oracle.greedy(mdp, V0)
    assert abs(st1["residual_in"] - float(np.max(np.abs(TV - V0)))) <= RES_ATOL * 8
    if K == 0:
        ref, _, _ = oracle.mb_sweep(mdp, V0, b, oracle.sweep_permutation(n, seed, 0))
    else:
        _, mu = oracle.greedy(mdp, V0)
        ref = V0
        for t in range(K):
            ref, _, _ = oracle.mb_sweep(mdp, ref, b, oracle.sweep_permutation(n, seed, t),
                                        policy=mu)
    assert np.max(np.abs(Vg - ref)) <= V_ATOL * 8
    say("K=%d first step checked in %.1f s" % (K, time.time() - t0))
    Vg, pg, st = run_refine(h, mdp, V0, K, b, seed, 1e-6)
    say("K=%d certified: %s" % (K, st))
    assert st["converged"] and st["bound_out"] <= 1e-6
    assert np.max(np.abs(Vg - Vstar)) <= st["bound_out"]
    Q = oracle.q_values(mdp, np.arange(n), Vstar)
    check_argmin(Q, pg, 3e-6)
