"""Autotuners of the batched solve.

`tune_lanes` picks the lane-group width (threads per state row).  The
batched kernel serves a state with a group of 16, 32 or 64 lanes; the best
width depends on the row length (ld), the value type and the batch size: too
wide and a workgroup has few lane groups for a batch's states, too narrow
and long rows take many steps per lane.  It times a few sweeps of each width
on a sample of the MDPs of every size class, on the device, and writes the
fastest into the items.

`tune_batch_size` picks b = ceil(n / d) per size class from a set of
divisors d by timing whole solves to a tolerance on a sample.  b changes the
iterates (more, smaller batches propagate new values sooner, eqs. (10)-(12))
but not the fixed point J*, so it is for callers who fix only the accuracy.

Both save and restore the MDPs' V, so tuning leaves the solve's start
unchanged.
"""
import torch

from . import binding as mb

CANDIDATES = (16, 32, 64)
# classes of row length (values): [lo, hi)
CLASSES = ((0, 512), (512, 1024), (1024, 2048), (2048, 1 << 30))


def _cu_time(items, sweeps, ws):
    """Compute-unit milliseconds of `sweeps` sweeps of every item, one
    workgroup per item (the sum of the solves' spans, after a warm-up)."""
    mb.mdp_batch_upload(items, ws)
    mb.mdp_batch_launch(len(items), -1.0, 1, ws)  # warm-up
    mb.mdp_batch_launch(len(items), -1.0, sweeps, ws)
    stats = mb.mdp_batch_read_stats(ws, len(items))
    return sum(st["end_us"] - st["start_us"] for st in stats) / 1e3


def _groups(items):
    groups = {}
    for it in items:
        cls = next(i for i, (lo, hi) in enumerate(CLASSES) if lo <= it["ld"] < hi)
        groups.setdefault((it.get("dtype", "f32"), cls), []).append(it)
    return groups


def tune_lanes(items, sweeps=3, sample=32, candidates=CANDIDATES):
    """Sets item['lanes'] for every item: per size class the width with the
    least compute-unit time for a few sweeps of up to `sample` MDPs of the
    class, run one workgroup per MDP as most MDPs of a large batch are (a
    few MDPs alone on the device would get teams, which change the balance).
    Returns {(dtype, class): (lanes, compute-unit ms by width)}."""
    saved = [(it["V"].clone(), it.get("team", 0)) for it in items]
    choice = {}
    try:
        for key, group in sorted(_groups(items).items()):
            probe = group[:sample]
            ws = mb.batch_workspace(len(probe))
            times = {}
            for lanes in candidates:
                for it in probe:
                    it["lanes"] = lanes
                    it["team"] = 1
                times[lanes] = _cu_time(probe, sweeps, ws)
            best = min(times, key=times.get)
            for it in group:
                it["lanes"] = best
            choice[key] = (best, times)
    finally:
        for it, (V, team) in zip(items, saved):
            it["V"].copy_(V)
            it["team"] = team
    return choice


DIVISORS = (2, 4, 8, 16, 32)
MAX_B = 4096  # the batched kernel's largest batch


def batch_size(n, d):
    return max(1, min(n, MAX_B, -(-n // d)))


def tune_batch_size(items, tol=1e-6, sample=8, divisors=DIVISORS, max_sweeps=100000):
    """Sets item['b'] = ceil(n / d) (at most 4096) for every item, d per size
    class the divisor with the least compute-unit time (the sum over the
    sample of each solve's span) for solves of up to `sample` MDPs of the
    class from their current V to max |dV| <= tol.  The probes run one
    workgroup per MDP, as most MDPs of a large batch do (a few MDPs alone on
    the device would all get teams, whose per-batch barrier favours few
    batches).  Returns {(dtype, class): (d, compute-unit ms by divisor)}."""
    saved = [(it["V"].clone(), it.get("team", 0)) for it in items]
    choice = {}
    try:
        for key, group in sorted(_groups(items).items()):
            probe = group[:sample]
            start = [it["V"].clone() for it in probe]
            ws = mb.batch_workspace(len(probe))
            times = {}
            for d in divisors:
                for it, V in zip(probe, start):
                    it["b"] = batch_size(int(it["n"]), d)
                    it["team"] = 1
                    it["V"].copy_(V)
                mb.mdp_batch_upload(probe, ws)
                mb.mdp_batch_launch(len(probe), tol, max_sweeps, ws)
                stats = mb.mdp_batch_read_stats(ws, len(probe))
                times[d] = sum(st["end_us"] - st["start_us"] for st in stats) / 1e3
            best = min(times, key=times.get)
            for it in group:
                it["b"] = batch_size(int(it["n"]), best)
            choice[key] = (best, times)
    finally:
        for it, (V, team) in zip(items, saved):
            it["V"].copy_(V)
            it["team"] = team
    return choice
