"""Autotuner for the launch-shape knobs of a solve (orchestration only).

The knobs (see sgp_tune in include/sgp.h) and the elimination schedule of the
tree factor change launch shapes, never the method: check_every, tail_max
and graph leave every result bitwise unchanged; spmv_waves, light_height and
the schedule change only the order of roundings.  So the autotuner can pick
them by time alone, on the caller's own workload:

  1. schedule x light_height x tail_max: a factor per combination (the level
     schedule has no light phase), timed by fixed-iteration solves (the
     sweeps are the only part that differs);
  2. spmv_waves: fixed-iteration solves with the chosen factor;
  3. graph x check_every: full solves to the tolerance (the polling cadence
     and the launch path only show in the whole solve).

Each candidate is timed as the median of `repeats` runs after one warm-up
run.  Every run goes through libsgp; this module only keeps the clock.
"""
from __future__ import annotations

import time

import numpy as np
import torch

SCHEDULES = ("contract", "level")
TAIL_MAX = (0, 1024, 2200)
LIGHT_HEIGHT = (0, 16, 32, 64)
SPMV_WAVES = (2, 4, 8)
CHECK_EVERY = (1, 2, 4, 8, 16)
GRAPH = (0, 1)


def _timed(ctx, fn, repeats):
    fn()   # warm-up (allocations, graph capture paths)
    ts = []
    for _ in range(repeats):
        torch.cuda.synchronize(ctx.dev())
        t0 = time.perf_counter()
        fn()
        torch.cuda.synchronize(ctx.dev())
        ts.append(time.perf_counter() - t0)
    return float(np.median(ts))


def tune(ctx, g, T, A, F, offsets=None, fixed_iters=20, repeats=3, rtol=1e-8, log=None):
    """Choose the knobs for solving Gamma v = F on (g, T, A); F on the device,
    `offsets` (host int64) for a batch.  Applies the choice to ctx and returns
    {"schedule", "light_height", "tail_max", "spmv_waves", "check_every",
    "graph", "prec", "table"}: `prec` is the factor built with the chosen
    schedule, light_height and tail_max, `table` every timing (seconds)."""
    table = {}

    def solve(M, fixed):
        if offsets is None:
            return ctx.pcg_solve(A, M, F, rtol=rtol, fixed_iters=fixed)
        return ctx.pcg_solve_batched(A, M, offsets, F, rtol=rtol, fixed_iters=fixed)

    start = {k: ctx.tune_get(k) for k in ("check_every", "tail_max", "graph", "spmv_waves", "light_height")}
    ctx.tune("graph", 0)
    best = None
    for sched in SCHEDULES:
        for lh in (LIGHT_HEIGHT if sched == "contract" else (0,)):
            ctx.tune("light_height", lh)
            for tm in TAIL_MAX:
                ctx.tune("tail_max", tm)
                M = ctx.factor_tree(g, T, schedule=sched)
                t = _timed(ctx, lambda: solve(M, fixed_iters), repeats)
                table[f"schedule={sched},light_height={lh},tail_max={tm}"] = t
                if log:
                    log(f"autotune: schedule {sched} light_height {lh} tail_max {tm}: "
                        f"{t * 1e3:.2f} ms / {fixed_iters} iterations")
                if best is None or t < best[0]:
                    best = (t, sched, lh, tm, M)
    _, sched, lh, tm, M = best
    ctx.tune("light_height", lh)
    ctx.tune("tail_max", tm)
    best_w = None
    for wv in SPMV_WAVES:
        ctx.tune("spmv_waves", wv)
        t = _timed(ctx, lambda: solve(M, fixed_iters), repeats)
        table[f"spmv_waves={wv}"] = t
        if log:
            log(f"autotune: spmv_waves {wv}: {t * 1e3:.2f} ms / {fixed_iters} iterations")
        if best_w is None or t < best_w[0]:
            best_w = (t, wv)
    ctx.tune("spmv_waves", best_w[1])
    best_c = None
    for gr in GRAPH:
        for ce in CHECK_EVERY:
            ctx.tune("graph", gr)
            ctx.tune("check_every", ce)
            t = _timed(ctx, lambda: solve(M, 0), repeats)
            table[f"graph={gr},check_every={ce}"] = t
            if log:
                log(f"autotune: graph {gr} check_every {ce}: {t * 1e3:.2f} ms / solve")
            if best_c is None or t < best_c[0]:
                best_c = (t, gr, ce)
    ctx.tune("graph", best_c[1])
    ctx.tune("check_every", best_c[2])
    return {"schedule": sched, "light_height": lh, "tail_max": tm, "spmv_waves": best_w[1], "graph": best_c[1],
            "check_every": best_c[2], "prec": M, "table": table, "defaults": start}
