"""Autotuner of the scoring kernel's launch shape.

The scoring kernel takes three free parameters: candidates per work item
(32, 64 or 128), correspondences per work item (512 to 4,096, the
correspondence tile) and the number of workgroups (from a few per compute
unit, each striding over many work items, to about one per item).  None changes a
result (per-candidate scores are integer-accumulated over fixed 512-point
wave blocks), so the tuner simply times each shape on the caller's own
workload with HIP events (the library's per-stage timing) and keeps the
fastest on the context.
"""
from __future__ import annotations

import ctypes as C

from . import Context, lib


def candidate_shapes(cus: int):
    for ct in (32, 64, 128):
        for pts in (512, 1024, 2048, 4096):
            for per_cu in (4, 8, 16, 32, 64, 128, 256):
                yield ct, pts, per_cu * cus


def tune_scoring(ctx: Context, run, reps: int = 2, cus: int | None = None) -> dict:
    """run(ctx) must execute the workload once and return imloc stats (a dict,
    or a list of dicts or a stats array for a batch).  Returns the timing table and leaves the
    fastest shape set on ctx."""
    if cus is None:
        import torch
        cus = torch.cuda.get_device_properties(ctx.device).multi_processor_count
    lib().imloc_set_timing(ctx.h, 1)
    table = []
    try:
        for ct, pts, wg in candidate_shapes(cus):
            ctx.set_score_tuning(ct, wg)
            ctx.set_score_points(pts)
            best = None
            for _ in range(reps):
                st = run(ctx)
                st0 = st if isinstance(st, dict) else st[0]  # one query's stats, or a batch's (list or array)
                ms = float(st0["ms_score"])
                best = ms if best is None else min(best, ms)
            table.append(dict(candidates_per_item=ct, points_per_item=pts, workgroups=wg, score_ms=best))
    finally:
        lib().imloc_set_timing(ctx.h, 0)
    win = min(table, key=lambda r: r["score_ms"])
    ctx.set_score_tuning(win["candidates_per_item"], win["workgroups"])
    ctx.set_score_points(win["points_per_item"])
    return dict(best=win, table=table)
