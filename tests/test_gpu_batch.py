"""GPU parity of the batched solve (many independent dense MDPs in one
launch) against the oracle: each MDP's iterate after a fixed number of
sweeps equals the oracle's FP64 MB-VI from the same V0, seed and batch size
(the kernel computes in FP64 too), the greedy policies, the limit J*, and
replays of a hipGraph-captured launch."""
import numpy as np
import pytest
import torch

import oracle
from oracle import quantize as qz
from paper_2110_02901_amd import binding as mb
from paper_2110_02901_amd import inputs

from gpu_util import check_argmin, dev, up

pytestmark = pytest.mark.gpu


def say(msg):
    print("[batch] " + msg, flush=True)


def make_item(n, m, dtype, gamma, b, seed, data_seed, lanes=0, alpha=1.0, with_oracle=True):
    """(item dict for the library, oracle MDP of the stored rows or None, V0)."""
    ld = (n + 15) // 16 * 16
    P, c = inputs.dense_mdp(n, m, alpha, data_seed, dtype=np.float32)
    Ppad = np.zeros((n, m, ld), dtype=np.float32)
    Ppad[:, :, :n] = P
    rows = up(Ppad.reshape(n * m, ld))
    Pstored = None
    if dtype == "f32":
        Pd, scale = rows, None
        if with_oracle:
            Pstored = P.astype(np.float64)
    else:
        Pd, scale = mb.mdp_quantize_rows(rows, dtype)
        del rows
        if with_oracle:
            q_ref, s_ref = qz.quantize_rows(Ppad.reshape(n * m, ld), dtype)
            Pstored = qz.dequantized(q_ref, s_ref, dtype).reshape(n, m, ld)[:, :, :n]
    V0 = inputs.values(n, data_seed + 1000, 0.0, 2.0, dtype=np.float64)
    item = {"n": n, "m": m, "dtype": dtype, "ld": ld, "P": Pd, "row_scale": scale,
            "c": up(c), "gamma": gamma, "b": b, "seed": seed,
            "V": up(V0.copy()), "policy": torch.zeros(n, dtype=torch.int32, device=dev()),
            "lanes": lanes}
    return item, (oracle.DenseMDP(Pstored, c, gamma) if with_oracle else (Ppad, c)), V0


def mixed_batch():
    specs = [(16, 3, "f32", 0.9, 4, 0), (100, 5, "bf16", 0.85, 13, 16), (256, 8, "fp8", 0.95, 32, 32),
             (333, 2, "f32", 0.93, 42, 64), (700, 8, "bf16", 0.9, 88, 0), (64, 1, "fp8", 0.8, 64, 16),
             (500, 10, "f32", 0.97, 63, 32), (1000, 4, "fp8", 0.9, 125, 64), (7, 2, "bf16", 0.5, 3, 16),
             (900, 8, "f32", 0.99, 113, 0)]
    out = []
    for i, (n, m, dt, g, b, lanes) in enumerate(specs):
        out.append(make_item(n, m, dt, g, b, 500 + i, 40 + i, lanes))
    return out


def test_batch_iterates_match_oracle_after_fixed_sweeps():
    batch = mixed_batch()
    items = [x[0] for x in batch]
    ws = mb.batch_workspace(len(items))
    mb.mdp_batch_upload(items, ws)
    T = 25
    mb.mdp_batch_launch(len(items), -1.0, T, ws)
    stats = mb.mdp_batch_read_stats(ws, len(items))
    for (item, mdp, V0), st in zip(batch, stats):
        assert st["sweeps"] == T and not st["converged"]
        ref, _, _ = oracle.value_iteration(mdp, item["b"], item["seed"], V0=V0, tol_dv=-1,
                                           max_sweeps=T)
        Vg = item["V"].cpu().numpy()
        err = float(np.max(np.abs(Vg - ref)))
        say("n=%d m=%d %s b=%d lanes=%d: max err %.3g" % (item["n"], item["m"], item["dtype"],
                                                         item["b"], item["lanes"], err))
        assert err <= 1e-11 * max(1.0, float(np.max(np.abs(ref))))
        Q = oracle.q_values(mdp, np.arange(mdp.n), Vg)
        check_argmin(Q, item["policy"].cpu().numpy(), 1e-10)


def test_batch_solves_reach_the_limit():
    batch = mixed_batch()
    items = [x[0] for x in batch]
    ws = mb.batch_workspace(len(items))
    mb.mdp_batch_upload(items, ws)
    mb.mdp_batch_launch(len(items), 1e-11, 100000, ws)
    stats = mb.mdp_batch_read_stats(ws, len(items))
    for (item, mdp, _), st in zip(batch, stats):
        assert st["converged"], st
        Vs, _, _ = oracle.policy_iteration(mdp, improve_tol=1e-14)
        bound = 1e-11 * item["gamma"] / (1 - item["gamma"]) + 1e-12 * float(np.max(np.abs(Vs)))
        assert np.max(np.abs(item["V"].cpu().numpy() - Vs)) <= 10 * bound


def test_batch_launch_replays_from_a_hip_graph():
    batch = mixed_batch()[:6]
    items = [x[0] for x in batch]
    V0s = [x[2] for x in batch]
    ws = mb.batch_workspace(len(items))
    mb.mdp_batch_upload(items, ws)
    T = 12
    # eager reference
    mb.mdp_batch_launch(len(items), -1.0, T, ws)
    torch.cuda.synchronize()
    eager = [it["V"].clone() for it in items]
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.stream(s):
        for it, V0 in zip(items, V0s):
            it["V"].copy_(up(V0))
        torch.cuda.synchronize()
        with torch.cuda.graph(graph, stream=s):
            mb.mdp_batch_launch(len(items), -1.0, T, ws)
    torch.cuda.current_stream().wait_stream(s)
    for rep in range(3):
        for it, V0 in zip(items, V0s):
            it["V"].copy_(up(V0))
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        for it, ref in zip(items, eager):
            assert torch.equal(it["V"], ref), rep
        # eager work between replays
        _ = torch.ones(1000, device=dev()).sum().item()


def test_batch_at_scale_sampled():
    """32 MDPs with n ~ U[256, 2048], m = 8, BF16, gamma ~ U[0.9, 0.99],
    b = ceil(n / 8): a fixed number of sweeps, three MDPs against the oracle."""
    g = np.random.Generator(np.random.Philox(77))
    count = 32
    ns = g.integers(256, 2049, count)
    gammas = g.uniform(0.9, 0.99, count)
    check = {int(np.argmax(ns)), int(np.argmin(ns)), 7}
    batch = [make_item(int(n), 8, "bf16", float(gm), int((n + 7) // 8), 900 + i, 300 + i,
                       with_oracle=(i in check))
             for i, (n, gm) in enumerate(zip(ns, gammas))]
    items = [x[0] for x in batch]
    ws = mb.batch_workspace(count)
    mb.mdp_batch_upload(items, ws)
    T = 10
    mb.mdp_batch_launch(count, -1.0, T, ws)
    stats = mb.mdp_batch_read_stats(ws, count)
    assert all(st["sweeps"] == T for st in stats)
    for i in sorted(check):
        item, mdp, V0 = batch[i]
        ref, _, _ = oracle.value_iteration(mdp, item["b"], item["seed"], V0=V0, tol_dv=-1,
                                           max_sweeps=T)
        err = float(np.max(np.abs(item["V"].cpu().numpy() - ref)))
        say("item %d n=%d: max err %.3g" % (i, item["n"], err))
        assert err <= 1e-11 * max(1.0, float(np.max(np.abs(ref))))


def test_batch_teams_match_single_workgroups():
    """A team of workgroups on one MDP computes the same iterates as one
    workgroup (the same arithmetic per state), for team sizes with members
    idle in some batches (b below the team's lane groups) and sizes that
    split every batch; both after a fixed number of sweeps and with the
    stop rule (the same sweep count)."""
    specs = [(700, 8, "bf16", 0.9, 88, 16), (1000, 4, "fp8", 0.95, 125, 64),
             (333, 2, "f32", 0.93, 42, 32), (2048, 8, "bf16", 0.97, 256, 16),
             (50, 3, "f32", 0.8, 7, 16)]
    for T, tol in ((9, -1.0), (100000, 1e-9)):
        base = [make_item(n, m, dt, g, b, 700 + i, 60 + i, lanes, with_oracle=False)
                for i, (n, m, dt, g, b, lanes) in enumerate(specs)]
        runs = {}
        for teams in ((1, 1, 1, 1, 1), (2, 3, 5, 16, 2), (16, 2, 3, 4, 7)):
            items = []
            for (it, _, V0), k in zip(base, teams):
                it = dict(it)
                it["V"] = up(V0.copy())
                it["policy"] = torch.zeros(it["n"], dtype=torch.int32, device=dev())
                it["team"] = k
                items.append(it)
            ws = mb.batch_workspace(len(items))
            mb.mdp_batch_upload(items, ws)
            mb.mdp_batch_launch(len(items), tol, T, ws)
            stats = mb.mdp_batch_read_stats(ws, len(items))
            assert [st["team"] for st in stats] == list(teams)
            assert all(0.0 <= st["start_us"] <= st["end_us"] for st in stats)
            runs[teams] = ([it["V"].cpu() for it in items], [it["policy"].cpu() for it in items],
                           [(st["sweeps"], st["converged"]) for st in stats])
            say("T=%d tol=%g teams %s: sweeps %s" % (T, tol, teams, [s[0] for s in runs[teams][2]]))
        ref = runs[(1, 1, 1, 1, 1)]
        for teams, (Vs, pols, sts) in runs.items():
            assert sts == ref[2], teams
            for i in range(len(specs)):
                assert torch.equal(Vs[i], ref[0][i]), (teams, i)
                assert torch.equal(pols[i], ref[1][i]), (teams, i)
        if tol > 0:
            assert all(c for _, c in ref[2])


def test_batch_rejects_bad_team_sizes():
    item, _, _ = make_item(64, 2, "f32", 0.9, 8, 1, 2, with_oracle=False)
    ws = mb.batch_workspace(1)
    for bad in (-1, 17):
        it = dict(item)
        it["team"] = bad
        with pytest.raises(RuntimeError):
            mb.mdp_batch_upload([it], ws)


def test_batch_teams_replay_from_a_hip_graph():
    """A captured launch with teams replays to the eager result, three times,
    with eager work in between (the team barrier counters are cleared by a
    fill kernel inside the capture)."""
    specs = [(700, 8, "bf16", 0.9, 88, 16, 3), (1000, 4, "fp8", 0.95, 125, 64, 2),
             (333, 2, "f32", 0.93, 42, 32, 1), (2048, 8, "bf16", 0.97, 256, 16, 4)]
    batch = [make_item(n, m, dt, g, b, 800 + i, 90 + i, lanes, with_oracle=False)
             for i, (n, m, dt, g, b, lanes, _) in enumerate(specs)]
    items = []
    for (it, _, V0), spec in zip(batch, specs):
        it = dict(it)
        it["team"] = spec[6]
        items.append(it)
    V0s = [x[2] for x in batch]
    ws = mb.batch_workspace(len(items))
    mb.mdp_batch_upload(items, ws)
    T = 7
    mb.mdp_batch_launch(len(items), -1.0, T, ws)
    torch.cuda.synchronize()
    eager = [it["V"].clone() for it in items]
    assert [st["team"] for st in mb.mdp_batch_read_stats(ws, len(items))] == [s[6] for s in specs]
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.stream(s):
        for it, V0 in zip(items, V0s):
            it["V"].copy_(up(V0.copy()))
        torch.cuda.synchronize()
        with torch.cuda.graph(graph, stream=s):
            mb.mdp_batch_launch(len(items), -1.0, T, ws)
    torch.cuda.current_stream().wait_stream(s)
    for rep in range(3):
        for it, V0 in zip(items, V0s):
            it["V"].copy_(up(V0.copy()))
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        for it, ref in zip(items, eager):
            assert torch.equal(it["V"], ref), rep
        _ = torch.ones(1000, device=dev()).sum().item()


def test_batch_size_tuner_keeps_the_fixed_point():
    """The b tuner picks a divisor per size class; the tuned solve still
    reaches every MDP's J* (policy iteration on the stored rows), and V is
    restored after tuning."""
    from paper_2110_02901_amd import tune
    specs = [(200, 4, "f32", 0.9), (260, 4, "f32", 0.95), (600, 8, "bf16", 0.9),
             (700, 8, "bf16", 0.97), (1100, 4, "fp8", 0.9)]
    batch = [make_item(n, m, dt, g, 8, 1500 + i, 700 + i) for i, (n, m, dt, g) in enumerate(specs)]
    items = [x[0] for x in batch]
    before = [it["V"].clone() for it in items]
    choice = tune.tune_batch_size(items, tol=1e-6, sample=4)
    say("b tuner: %s" % {"%s/%d" % k: v[0] for k, v in choice.items()})
    for it, V in zip(items, before):
        assert torch.equal(it["V"], V)
        assert 1 <= it["b"] <= min(it["n"], 4096)
        assert any(it["b"] == tune.batch_size(it["n"], d) for d in tune.DIVISORS)
    ws = mb.batch_workspace(len(items))
    mb.mdp_batch_upload(items, ws)
    mb.mdp_batch_launch(len(items), 1e-11, 100000, ws)
    stats = mb.mdp_batch_read_stats(ws, len(items))
    for (item, mdp, _), st in zip(batch, stats):
        assert st["converged"], st
        Vs, _, _ = oracle.policy_iteration(mdp, improve_tol=1e-14)
        bound = 1e-11 * item["gamma"] / (1 - item["gamma"]) + 1e-12 * float(np.max(np.abs(Vs)))
        assert np.max(np.abs(item["V"].cpu().numpy() - Vs)) <= 10 * bound


def test_batch_512_full_size_sampled():
    """The benchmark's batch: 512 MDPs, n ~ U[256, 4096], m = 8, Dirichlet(1)
    rows (torch's generator on the GPU, as the benchmark draws them) in BF16,
    gamma ~ U[0.9, 0.99], b = ceil(n/8), automatic teams; 3 sweeps, then the
    largest, the smallest, the heaviest (served by a team) and one more MDP
    against the oracle's MB-VI of rows it quantises itself from host copies
    of the same FP32 rows."""
    count, m, T = 512, 8, 3
    g = np.random.Generator(np.random.Philox(104))
    ns = g.integers(256, 4097, count)
    gammas = g.uniform(0.9, 0.99, count)
    heavy = int(np.argmax(ns.astype(np.float64) ** 2 / -np.log(gammas)))  # gets a team
    check = {int(np.argmax(ns)), int(np.argmin(ns)), 100, heavy}
    gen = torch.Generator(device=dev())
    gen.manual_seed(104)
    items, host = [], {}
    for i in range(count):
        n = int(ns[i])
        ld = (n + 63) // 64 * 64  # rows of whole 128-byte lines, as the benchmark lays them out
        rows = torch.zeros(n * m, ld, dtype=torch.float32, device=dev())
        w = torch._standard_gamma(torch.ones(n * m, n, device=dev()), generator=gen)
        rows[:, :n] = w / w.sum(dim=1, keepdim=True)
        del w
        if i in check:
            host[i] = rows.cpu().numpy()
        codes, scale = mb.mdp_quantize_rows(rows, "bf16")
        del rows
        c = torch.rand(n, m, device=dev(), generator=gen)
        items.append({"n": n, "m": m, "dtype": "bf16", "ld": ld, "P": codes.reshape(-1),
                      "row_scale": scale, "c": c, "gamma": float(gammas[i]), "b": (n + 7) // 8,
                      "seed": 2000 + i, "V": torch.zeros(n, dtype=torch.float64, device=dev()),
                      "policy": None, "lanes": 0})
    say("generated the 512 MDPs")
    ws = mb.batch_workspace(count)
    mb.mdp_batch_upload(items, ws)
    mb.mdp_batch_launch(count, -1.0, T, ws)
    stats = mb.mdp_batch_read_stats(ws, count)
    assert all(st["sweeps"] == T for st in stats)
    teams = [st["team"] for st in stats]
    say("teams: %d MDPs with more than one workgroup" % sum(t > 1 for t in teams))
    assert teams[heavy] > 1  # the heavy MDPs run as teams in this configuration
    for i in sorted(check):
        n, ld = int(ns[i]), items[i]["ld"]
        q, sc = qz.quantize_rows(host[i], "bf16")
        Pst = qz.dequantized(q, sc, "bf16").reshape(n, m, ld)[:, :, :n]
        c = items[i]["c"].cpu().numpy().astype(np.float64)
        mdp = oracle.DenseMDP(Pst, c, float(gammas[i]))
        ref, _, _ = oracle.value_iteration(mdp, (n + 7) // 8, 2000 + i, V0=np.zeros(n), tol_dv=-1,
                                           max_sweeps=T)
        err = float(np.max(np.abs(items[i]["V"].cpu().numpy() - ref)))
        say("item %d n=%d team=%d: max err %.3g" % (i, n, teams[i], err))
        assert err <= 1e-11 * max(1.0, float(np.max(np.abs(ref))))
