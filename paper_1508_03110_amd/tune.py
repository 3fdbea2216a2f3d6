"""Work-decomposition tuner for the half-sweep.

For each orientation of R it times the half-sweep (the dominant launch of
both algorithms) over a small grid of launch shapes and keeps the fastest:
  * chunk: the most ratings one wavefront takes from a row (longer rows are
    split with a fixed-order second stage); candidates around the plan's
    default of nnz / (8 x compute units);
  * grid: one workgroup per chunk, or a persistent grid of k workgroups per
    compute unit striding over the chunks (longest first).
Results do not depend on the choice (every chunk reduces into its own slot
in a fixed order); only time does.  The choice is returned as a dict and
applied to the problem's plans.
"""
from __future__ import annotations

import time

import torch


def _time_sweep(DP, side, Y, X, reps):
    DP.sweep(side, Y, X)  # warm (also sizes the workspace)
    torch.cuda.synchronize()
    a = torch.cuda.Event(enable_timing=True)
    b = torch.cuda.Event(enable_timing=True)
    best = float("inf")
    for _ in range(reps):
        a.record()
        DP.sweep(side, Y, X)
        b.record()
        torch.cuda.synchronize()
        best = min(best, a.elapsed_time(b))
    return best


def tune(DP, x, reps: int = 2, chunk_factors=(1.0, 0.25, 0.0625), grids_per_cu=(0, 4, 8, 16),
         log=None) -> dict:
    """Tune both plans of DeviceProblem DP on the iterate x ([U; M], its
    current values are used as the fixed side; X outputs go to scratch)."""
    say = log or (lambda *a: None)
    n_cu = torch.cuda.get_device_properties(DP.ctx.torch_device).multi_processor_count
    out = {}
    for side, A, Y, nrows in (("U", DP.R, DP.M(x), DP.n_u), ("M", DP.Rt, DP.U(x), DP.n_m)):
        X = torch.empty((nrows, DP.ld), dtype=DP.dtype, device=DP.ctx.torch_device)
        base = A.info()["chunk"]
        trials = []
        t0 = time.perf_counter()
        for f in chunk_factors:
            chunk = max(256, int(base * f) // 4 * 4)
            A.replan(chunk, 0)
            for gpc in grids_per_cu:
                A.set_grid(gpc * n_cu)
                ms = _time_sweep(DP, side, Y, X, reps)
                trials.append({"chunk": chunk, "grid": gpc * n_cu, "ms": round(ms, 4)})
        best = min(trials, key=lambda t: t["ms"])
        A.replan(best["chunk"], best["grid"])
        out[side] = {"best": best, "default_ms": trials[0]["ms"], "trials": trials,
                     "seconds": round(time.perf_counter() - t0, 2)}
        say("tuned %s half-sweep: %s (default %.3f ms)" % (side, best, trials[0]["ms"]))
        del X
    return out
