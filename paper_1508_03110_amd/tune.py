"""Work-decomposition tuner for the half-sweep and the streaming passes.

For each orientation of R it times the half-sweep (the dominant launch of
both algorithms) over a small grid of launch shapes and keeps the fastest:
  * chunk: the most ratings one wavefront takes from a row (longer rows are
    split with a fixed-order second stage); candidates at and below the
    plan's default (nnz / (8 x compute units), at most 8192);
  * sweep grid: one workgroup per chunk, or a persistent grid of k
    workgroups per compute unit striding over the chunks (longest first).
With that plan it then picks the length bins of the half-sweep: rows of at
most `dual_max` ratings take the dual form (an n_i x n_i system, one kernel
instance per 16-wide tile count), the rest the n_f x n_f form; candidates
0 (off) and 16 b - 2 for b = 1 .. 6 tiles, each timed (in FP32) with and
without the split copy of the fixed side for the n_f x n_f form.  Last it picks the persistent
grid of the orientation's streaming pass (coefficients for R, gradient for
R^T), whose per-chunk work is small enough for workgroup dispatch to matter,
and whether the M-block gradient takes a plan of R^T cut at column slices
(one slice of the user rows per die of the device at a time, so that each
die's L2 holds the rows it gathers).
Results do not depend on the chunk or the grids (every chunk reduces into
its own slot in a fixed order), only time does; the dual form and the
column slices reach the same result by a different rounding path.
"""
from __future__ import annotations

import time

import torch


def _best_ms(fn, reps):
    fn()  # warm (also sizes the workspace)
    torch.cuda.synchronize()
    a = torch.cuda.Event(enable_timing=True)
    b = torch.cuda.Event(enable_timing=True)
    best = float("inf")
    for _ in range(reps):
        a.record()
        fn()
        b.record()
        torch.cuda.synchronize()
        best = min(best, a.elapsed_time(b))
    return best


DUAL_CANDIDATES = (0, 14, 30, 46, 62, 78, 94)


def tune_dual(DP, side: str, Y, X, reps: int = 3, candidates=DUAL_CANDIDATES,
              split_modes=None) -> dict:
    """Pick the dual-form length bound of one orientation's plan together
    with (FP32) whether its n_f x n_f form gathers a split copy of the fixed
    side, by timing the half-sweep for every pair (Y: fixed side, X: output
    buffer); leaves the best pair set.  split_modes: the split-copy settings
    to try (default: off and on in FP32, the plan's default otherwise)."""
    A = DP.R if side == "U" else DP.Rt
    if split_modes is None:
        split_modes = (0, 1) if DP.dtype == torch.float32 else (-1,)
    trials = []
    for m in candidates:
        if m > 0 and m > A.info()["chunk"]:
            continue
        A.set_dual(m)
        for sc in split_modes:
            A.set_split_copy(sc)
            trials.append({"dual_max": m, "split_copy": sc, "dual_rows": A.info()["dual_rows"],
                           "ms": round(_best_ms(lambda: DP.sweep(side, Y, X), reps), 4)})
    best = min(trials, key=lambda t: t["ms"])
    A.set_dual(best["dual_max"])
    A.set_split_copy(best["split_copy"])
    return {"best": best, "trials": trials}


GRAD_SLICE_CANDIDATES = (0, 8)
SLICE_TABLE_MAX = 256 << 20  # bytes of gathered rows up to which slices are tried


def tune_grad_slices(DP, U, M, X, reps: int = 3, candidates=GRAD_SLICE_CANDIDATES) -> dict:
    """Pick the column slices of the M-block gradient's plan (0: the plan of
    the half-sweep) by timing that pass (X: output rows of M's shape);
    leaves the best one set."""
    trials = []
    for n in candidates:
        DP.Rt.set_grad_slices(n)
        trials.append({"slices": n, "ms": round(_best_ms(lambda: DP.gradient(U, M, None, X, None), reps), 4)})
    best = min(trials, key=lambda t: t["ms"])
    DP.Rt.set_grad_slices(best["slices"])
    return {"best": best, "trials": trials}


def tune(DP, x, reps: int = 2, chunk_factors=(1.0, 0.25), grids_per_cu=(0, 4, 8, 16),
         pass_grids_per_cu=(0, 4, 8, 16, 32), log=None) -> dict:
    """Tune both plans of DeviceProblem DP around the iterate x ([U; M]; its
    values are the inputs, outputs go to scratch buffers)."""
    say = log or (lambda *a: None)
    n_cu = torch.cuda.get_device_properties(DP.ctx.torch_device).multi_processor_count
    dev = DP.ctx.torch_device
    out = {}
    U, M = DP.U(x), DP.M(x)
    # a direction distinct from x: the coefficient pass gathers both, and
    # p = x would let the second gather hit the first one's cache lines
    pdir = torch.empty_like(x).normal_(0.0, 0.01)
    pU, pM = DP.U(pdir), DP.M(pdir)
    coef = torch.zeros(8, dtype=torch.float64, device=dev)
    for side, A, Y, nrows in (("U", DP.R, M, DP.n_u), ("M", DP.Rt, U, DP.n_m)):
        X = torch.empty((nrows, DP.ld), dtype=DP.dtype, device=dev)
        base = A.info()["chunk"]
        trials = []
        t0 = time.perf_counter()
        for f in chunk_factors:
            chunk = max(256, int(base * f) // 4 * 4)
            A.replan(chunk, 0, 0)
            for gpc in grids_per_cu:
                A.set_grid(gpc * n_cu, 0)
                ms = _best_ms(lambda: DP.sweep(side, Y, X), reps)
                trials.append({"chunk": chunk, "grid": gpc * n_cu, "ms": round(ms, 4)})
        best = min(trials, key=lambda t: t["ms"])
        A.replan(best["chunk"], best["grid"], 0)
        dual = tune_dual(DP, side, Y, X, reps=reps)
        best = dict(best, dual_max=dual["best"]["dual_max"], split_copy=dual["best"]["split_copy"],
                    dual_ms=dual["best"]["ms"])
        if side == "U":  # the coefficient pass runs over R
            run = lambda: DP.coeffs(U, M, pU, pM, coef)  # noqa: E731
        else:            # the M-block gradient pass runs over R^T
            run = lambda: DP.gradient(U, M, None, X, None)  # noqa: E731
        ptrials = []
        for gpc in pass_grids_per_cu:
            A.set_grid(best["grid"], gpc * n_cu)
            ptrials.append({"grid_pass": gpc * n_cu, "ms": round(_best_ms(run, reps), 4)})
        pbest = min(ptrials, key=lambda t: t["ms"])
        A.set_grid(best["grid"], pbest["grid_pass"])
        # slices are tried only while the gathered user rows fit the device's
        # 256 MB last-level cache: beyond it one die's slice is far larger
        # than its L2 and the extra pieces are not expected to pay
        table = DP.n_u * DP.ld * DP.zeros(1).element_size()
        if side == "M" and table <= SLICE_TABLE_MAX:
            sl = tune_grad_slices(DP, U, M, X, reps=reps)
            if sl["best"]["slices"] and sl["best"]["ms"] < pbest["ms"]:
                pbest = {"grid_pass": pbest["grid_pass"], "ms": sl["best"]["ms"]}
                best = dict(best, grad_slices=sl["best"]["slices"])
            else:
                DP.Rt.set_grad_slices(0)
                best = dict(best, grad_slices=0)
            ptrials = ptrials + [dict(t, grid_pass=0) for t in sl["trials"] if t["slices"]]
        elif side == "M":
            best = dict(best, grad_slices=0)
        out[side] = {"best": dict(best, grid_pass=pbest["grid_pass"], pass_ms=pbest["ms"]),
                     "default_ms": trials[0]["ms"], "default_pass_ms": ptrials[0]["ms"],
                     "trials": trials, "dual_trials": dual["trials"], "pass_trials": ptrials,
                     "seconds": round(time.perf_counter() - t0, 2)}
        say("tuned %s: %s (default sweep %.3f ms, pass %.3f ms)"
            % (side, out[side]["best"], trials[0]["ms"], ptrials[0]["ms"]))
        del X
    del pdir
    return out
