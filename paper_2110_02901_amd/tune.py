"""Autotuner of the batched solve's lane-group width (threads per state row).

The batched kernel serves a state with a group of 16, 32 or 64 lanes; the
best width depends on the row length (ld) and the value type: too wide and
lanes idle on short rows, too narrow and long rows take many steps per lane.
`tune_lanes` times a few sweeps of each width on a sample of the MDPs of
every size class, on the device, and writes the fastest into the items.
The MDPs' V are saved and restored, so tuning leaves the solve unchanged.
"""
import torch

from . import binding as mb

CANDIDATES = (16, 32, 64)
# classes of row length (values): [lo, hi)
CLASSES = ((0, 512), (512, 1024), (1024, 2048), (2048, 1 << 30))


def _time_launch(items, sweeps, ws):
    mb.mdp_batch_upload(items, ws)
    mb.mdp_batch_launch(len(items), -1.0, 1, ws)  # warm-up
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    mb.mdp_batch_launch(len(items), -1.0, sweeps, ws)
    e1.record()
    e1.synchronize()
    return e0.elapsed_time(e1)


def tune_lanes(items, sweeps=3, sample=32, candidates=CANDIDATES):
    """Sets item['lanes'] for every item; returns {(dtype, class): (lanes, ms by width)}."""
    saved = [it["V"].clone() for it in items]
    choice = {}
    try:
        groups = {}
        for it in items:
            cls = next(i for i, (lo, hi) in enumerate(CLASSES) if lo <= it["ld"] < hi)
            groups.setdefault((it.get("dtype", "f32"), cls), []).append(it)
        for key, group in sorted(groups.items()):
            probe = group[:sample]
            ws = mb.batch_workspace(len(probe))
            times = {}
            for lanes in candidates:
                for it in probe:
                    it["lanes"] = lanes
                times[lanes] = _time_launch(probe, sweeps, ws)
            best = min(times, key=times.get)
            for it in group:
                it["lanes"] = best
            choice[key] = (best, times)
    finally:
        for it, V in zip(items, saved):
            it["V"].copy_(V)
    return choice
