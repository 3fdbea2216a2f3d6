#!/usr/bin/env python3
"""Benchmark: ALS-NCG on the MovieLens-20M-shaped synthetic problem, one GPU.

Workload: 138,493 users x 26,744 items, exactly 20,000,263 ratings (Zipf item
popularity, log-normal user activity, half-star values from a planted rank-50
model), n_f = 100, lambda = 0.05, FP32 factors, FP64 reductions.  All inputs
are seeded and resident in HBM before the timed region.

One step = one full ALS-NCG iteration (Algorithm 2): quartic coefficients
(one pass over R), backtracking on the device, x += alpha p, the ALS
preconditioner P(x) = two half-sweeps (U block of the gradient fused into
the U half-sweep), the M block of the gradient (one pass over R^T), and the
direction update.  value = half-sweep ratings per second sustained by the
whole iteration: 2 * nnz * steps / elapsed.

Prints one JSON line (rank 0).
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "ALS half-sweep ratings/s + time-to-f-tol, ALS-NCG vs ALS; fold-in p99 ms"
PEAK_FP32_TFLOPS = 157.3   # MI355X dense FP32 matrix
PEAK_HBM_GBS = 8000.0


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def sweep_flops(nnz, n_rows, n_f):
    """Algorithmic flops of one half-sweep: symmetric Gram n_f(n_f+1) and RHS
    2 n_f per rating, Cholesky n_f^3/3 and two triangular solves 2 n_f^2 per row."""
    return nnz * (n_f * (n_f + 1) + 2 * n_f) + n_rows * (n_f ** 3 / 3.0 + 2 * n_f ** 2)


def sweep_flops_binned(counts, n_f, dual_max):
    """Algorithmic flops of one half-sweep with length bins: rows of
    1 <= n_i <= dual_max ratings in the dual form (symmetric K = Y_I Y_I^T
    n_i (n_i + 1) n_f, Cholesky n_i^3 / 3, two triangular solves 2 n_i^2,
    x = Y_I^T z 2 n_i n_f), the others as sweep_flops."""
    import numpy as np
    n = np.asarray(counts, dtype=np.float64)
    prim = n * (n_f * (n_f + 1) + 2 * n_f) + (n_f ** 3 / 3.0 + 2 * n_f ** 2)
    dual = n * (n + 1) * n_f + n ** 3 / 3.0 + 2 * n ** 2 + 2 * n * n_f
    use = (n >= 1) & (n <= dual_max)
    return float(np.where(use, dual, prim).sum())


def kernel_source_hash():
    """sha256 (first 16 hex) of the half-sweep's sources with // comments,
    trailing blanks and empty lines removed: the code the counters were
    taken on, not its commentary."""
    import hashlib
    m = hashlib.sha256()
    for f in ("sweep.hip", "sweep_dual.hip", "internal.h", "rowsolve.h"):
        with open(os.path.join(ROOT, "paper_1508_03110_amd", "csrc", f), encoding="utf-8") as fh:
            for line in fh:
                code = line.split("//", 1)[0].rstrip()
                if code:
                    m.update(code.encode() + b"\n")
    return m.hexdigest()[:16]


def profiled_traffic(dual_max, split_copy=0):
    """HBM bytes per U half-sweep (all its launches) from the committed
    rocprofv3 counter summary for this length bound and split-copy choice,
    or None when the kernel sources changed since it was taken or that
    configuration was not profiled."""
    path = os.path.join(ROOT, "profiles", "sweep_chunks_f32_nf100_ml20m_shape.md")
    try:
        for line in open(path):
            line = line.strip()
            if line.startswith("TRAFFIC "):
                d = json.loads(line[len("TRAFFIC "):])
                if (d.get("source_hash") == kernel_source_hash() and d.get("dual_max") == dual_max
                        and d.get("split_copy", 0) == split_copy):
                    return int(d["bytes"])
    except OSError:
        pass
    return None


def cpu_model():
    """The host CPU's model name (from /proc/cpuinfo, as lscpu reports it)."""
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def row_sample(A, n_rows):
    """Evenly spaced rows of a CSR (host arrays) as a CSR of their own."""
    import numpy as np
    from types import SimpleNamespace
    rows = np.linspace(0, A.n_rows - 1, n_rows).astype(np.int64)
    lo, hi = A.indptr[rows], A.indptr[rows + 1]
    take = np.concatenate([np.arange(a, b) for a, b in zip(lo, hi)])
    indptr = np.concatenate([[0], np.cumsum(hi - lo)]).astype(np.int64)
    return SimpleNamespace(n_rows=n_rows, n_cols=A.n_cols, indptr=indptr,
                           indices=A.indices[take], values=A.values[take])


def cpu_baseline(P, reps=3, sample_users=2000):
    """The FP64 oracle timed on the host.

    value: one full ALS-NCG iteration (the loop body of Algorithm 2: quartic
    pass, backtracking, x + alpha p, P(x) = two half-sweeps, gradient,
    direction) on the whole matrix, all threads, median of `reps` iterations
    after one untimed iteration, in the unit and definition of `value`
    (2 nnz half-sweep ratings per iteration).  one_thread / all_threads: the
    oracle's U half-sweep over evenly spaced sampled users, median of `reps`,
    at 1 thread and at all threads (half-sweep ratings per second)."""
    import numpy as np

    import oracle
    threads = oracle.set_threads(0)
    U0 = P.U0.astype(np.float32).astype(np.float64)
    M0 = P.M0.astype(np.float32).astype(np.float64)
    o = oracle.NcgOracle(P.R, P.Rt, P.n_f, P.lam)
    t = time.perf_counter()
    s = o.init(U0, M0)
    t_init = time.perf_counter() - t
    o.step(s)
    its = []
    for _ in range(reps):
        t = time.perf_counter()
        o.step(s)
        its.append(time.perf_counter() - t)
    dt = float(np.median(its))
    S = row_sample(P.R, sample_users)

    def sweep_rate(n_threads):
        oracle.set_threads(n_threads)
        ts = []
        for _ in range(reps):
            t = time.perf_counter()
            oracle.half_sweep(S, M0, P.lam)
            ts.append(time.perf_counter() - t)
        return len(S.indices) / float(np.median(ts))

    r_all = sweep_rate(threads)
    r_one = sweep_rate(1)
    oracle.set_threads(threads)
    return {"value": 2.0 * P.nnz / dt, "unit": "ratings/s", "cores": threads, "kind": "oracle",
            "cpu": cpu_model(),
            "sample": "FP64 oracle ALS-NCG iteration (Algorithm 2 loop body) on the full "
                      "%d-rating matrix, n_f=%d, %d threads: median of %d = %.2f s (runs %s; "
                      "one untimed iteration and set-up P(x0), g(x0) %.1f s before)"
                      % (P.nnz, P.n_f, threads, reps, dt, [round(x, 2) for x in its], t_init),
            "half_sweep_sample": "U half-sweep over %d evenly spaced users (%d ratings), "
                                 "median of %d" % (sample_users, len(S.indices), reps),
            "half_sweep_ratings_per_s": {"threads_%d" % threads: r_all, "threads_1": r_one}}


def load_fstar():
    path = os.path.join(ROOT, "tests", "golden", "fstar_ml20m_shape.json")
    try:
        with open(path) as fh:
            return json.load(fh)
    except OSError:
        return None


RANK_T = 20  # top-t of the ranking accuracy (Section IV uses t = 20)


def ranking_kernels(DP, x, reps=3):
    """Average time of rank_top_t and rank_accuracy (HIP events on torch's
    current stream, where the binding launches them) at the problem's shape."""
    import torch

    from paper_1508_03110_amd.solver import rank_accuracy, rank_top_t
    U, M = DP.U(x), DP.M(x)
    top = rank_top_t(DP.ctx, U, M, RANK_T, n_f=DP.n_f)
    rank_accuracy(DP.ctx, U, M, top, n_f=DP.n_f)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
    ev[0].record()
    for _ in range(reps):
        rank_top_t(DP.ctx, U, M, RANK_T, n_f=DP.n_f)
    ev[1].record()
    for _ in range(reps):
        q = rank_accuracy(DP.ctx, U, M, top, n_f=DP.n_f)
    ev[2].record()
    torch.cuda.synchronize()
    flops = 2.0 * DP.n_u * DP.n_m * DP.n_f
    t_top, t_acc = ev[0].elapsed_time(ev[1]) / reps, ev[1].elapsed_time(ev[2]) / reps
    return {"t": RANK_T, "users": DP.n_u, "items": DP.n_m, "top_t_ms": round(t_top, 3),
            "accuracy_ms": round(t_acc, 3), "self_accuracy": q.item(),
            "rating_tflops_fp64": {"top_t": round(flops / t_top / 1e9, 2),
                                   "accuracy": round(flops / t_acc / 1e9, 2), "peak": 78.6}}


def ranking_small(ctx, n_starts=20, gtol=1e-6, max_als=3000, max_ncg=1500):
    """Tables III/IV of Section IV on the 600 x 400 planted problem (FP64,
    n_f = 10): from n_starts random starting iterates (N(0, 0.1), seeds
    1000 + i), ALS and ALS-NCG run until (1/N)||g|| <= gtol (traced: every
    iterate kept on the device); each run's final iterate gives the reference
    top-20 lists; the first iterate reaching 70/80/90/100 % ranking accuracy
    is timed in a second run from the same start without diagnostics (ALS:
    eager sweeps, two launches each; ALS-NCG: the device-controlled iteration
    replayed as a HIP graph, the same iterates as the traced run).  Reported
    as mean +- standard deviation over the starts, and the acceleration
    factor as the ratio of the mean times."""
    import numpy as np
    import torch

    import synth
    from paper_1508_03110_amd.solver import Als, AlsNcg, DeviceProblem, rank_accuracy, rank_top_t
    P = synth.c0_tiny()
    DP = DeviceProblem(ctx, P.R, P.Rt, P.n_f, P.lam, torch.float64)
    N = P.n_f * (P.n_u + P.n_m)
    levels = (0.70, 0.80, 0.90, 1.00)
    runs = {"als": [], "als_ncg": []}
    for i in range(n_starts):
        rng = np.random.default_rng(1000 + i)
        U0 = rng.normal(0.0, 0.1, (P.n_u, P.n_f))
        M0 = rng.normal(0.0, 0.1, (P.n_m, P.n_f))
        for name in runs:
            def make():
                return Als(DP, DP.pack(U0, M0)) if name == "als" else AlsNcg(DP).init(U0, M0)

            def step(s):
                s.sweep() if name == "als" else s.step()
            s, keep, conv = make(), [], False
            for k in range(1, (max_als if name == "als" else max_ncg) + 1):
                step(s)
                g = DP.loss_and_gnorm(s.x)[1] if name == "als" else s.gnorm()
                keep.append(s.x.clone())
                if g / N <= gtol:
                    conv = True
                    break
            top = rank_top_t(ctx, DP.U(keep[-1]), DP.M(keep[-1]), RANK_T, n_f=P.n_f)
            q = torch.cat([rank_accuracy(ctx, DP.U(x), DP.M(x), top, n_f=P.n_f) for x in keep])
            q = q.cpu().numpy()
            del keep
            ks = {lv: int(np.argmax(q >= lv)) + 1 for lv in levels}  # the last iterate has q = 1
            marks = sorted(set(ks.values()))
            # the clock starts before the set-up (ALS-NCG: P(x0) and g(x0));
            # capturing the graphs runs no iteration and is left out
            torch.cuda.synchronize()
            t0, secs = time.perf_counter(), {}
            s = make()
            if name == "als_ncg":
                torch.cuda.synchronize()
                t_cap = time.perf_counter()
                s.capture()
                torch.cuda.synchronize()
                t0 += time.perf_counter() - t_cap
            for k in range(1, marks[-1] + 1):
                s.sweep() if name == "als" else s.replay()
                if k in marks:
                    torch.cuda.synchronize()
                    secs[k] = time.perf_counter() - t0
            runs[name].append({"converged": conv, "iterations": len(q),
                               "levels": {lv: (ks[lv], secs[ks[lv]]) for lv in levels}})
    out = {"problem": "600 x 400 planted, 20,000 ratings, n_f = 10, FP64", "t": RANK_T,
           "starts": n_starts, "gnorm_over_N_tol": gtol}
    for name, rs in runs.items():
        out[name] = {"converged": sum(r["converged"] for r in rs),
                     "mean_iterations": float(np.mean([r["iterations"] for r in rs]))}
        for lv in levels:
            t = np.array([r["levels"][lv][1] for r in rs])
            it = np.array([r["levels"][lv][0] for r in rs])
            out[name]["%d%%" % round(100 * lv)] = {"seconds_mean": float(t.mean()),
                                                   "seconds_std": float(t.std()),
                                                   "iterations_mean": float(it.mean())}
    out["acceleration"] = {k: out["als"][k]["seconds_mean"] / out["als_ncg"][k]["seconds_mean"]
                           for k in ("70%", "80%", "90%", "100%")}
    return out


def time_to_tol(DP, P, fstar, tol=1e-6, gtol=1e-6, max_als=2500, max_ncg=600):
    """Wall time for ALS (Algorithm 1) and ALS-NCG (Algorithm 2) from the same
    x0 to a relative f-gap (f - f*)/f* <= tol, and to the paper's stopping
    rule (1/N)||g|| <= gtol (Section IV).  As in the paper's timing method
    (Section VI), a traced run (f and ||g|| evaluated every iteration) finds the
    iteration counts and a separate run without the diagnostics is timed.

    Also the time to a top-20 ranking accuracy of 70/80/90/100 % (Section IV,
    Tables III and IV): the traced runs keep x on the device (every ALS-NCG
    iteration; every ALS sweep up to 100, then every 10th), each algorithm's
    final traced iterate gives the reference top-20 lists, and the first kept
    iteration at each accuracy level is timed in the runs without
    diagnostics."""
    import numpy as np
    import torch

    from paper_1508_03110_amd.solver import Als, AlsNcg, rank_accuracy, rank_top_t
    U0 = P.U0.astype(np.float32)
    M0 = P.M0.astype(np.float32)
    N = P.n_f * (P.n_u + P.n_m)
    out = {"f_gap_tol": tol, "gnorm_over_N_tol": gtol, "f_star": fstar}

    def crossing(trace):
        kf = next((k for k, f, g in trace if (f - fstar) / fstar <= tol), None)
        kg = next((k for k, f, g in trace if g / N <= gtol), None)
        return kf, kg

    # ALS trace: f and ||g|| by one gradient pass per orientation after every sweep
    als = Als(DP, DP.pack(U0, M0))
    trace = []
    keep_als = []
    for k in range(1, max_als + 1):
        als.sweep()
        f, g = DP.loss_and_gnorm(als.x)
        trace.append((k, f, g))
        if k <= 100 or k % 10 == 0:
            keep_als.append((k, als.x.clone()))
        kf, kg = crossing(trace)
        if kf is not None and kg is not None:
            break
    k_als = crossing(trace)
    # ALS-NCG traces (backtracking of Algorithm 4, and the exact minimiser of
    # the same quartic): f(x_k) = Q(alpha_k) and ||g_k|| come with every iteration
    def ncg_trace(search, keep=None):
        ncg = AlsNcg(DP, search=search).init(U0, M0)
        tr = []
        for k in range(1, max_ncg + 1):
            ncg.step()
            f = ncg.f if ncg.f == ncg.f else DP.loss_and_gnorm(ncg.x)[0]  # NaN after an ALS point
            tr.append((k, f, ncg.gnorm()))
            if keep is not None:
                keep.append((k, ncg.x.clone()))
            kf, kg = crossing(tr)
            if kf is not None and kg is not None:
                break
        return tr

    keep_ncg = []
    trace_n = ncg_trace("backtracking", keep_ncg)
    k_ncg = crossing(trace_n)
    trace_e = ncg_trace("exact")
    k_exact = crossing(trace_e)

    def timed(make, step, marks):
        # the clock starts before make(): ALS-NCG's set-up (P(x0) and the
        # gradient at x0) is part of its time, as is ALS's upload of x0
        marks = sorted({m for m in marks if m})
        if not marks:
            return {}
        torch.cuda.synchronize()
        t = time.perf_counter()
        s = make()
        got = {}
        for k in range(1, marks[-1] + 1):
            step(s)
            if k in marks:
                torch.cuda.synchronize()
                got[k] = time.perf_counter() - t
        return got

    # ranking accuracy of the kept iterates against each run's final one
    levels = (0.70, 0.80, 0.90, 0.99, 0.999, 0.9999, 1.00)

    def rank_levels(keep):
        x_ref = keep[-1][1]
        top = rank_top_t(DP.ctx, DP.U(x_ref), DP.M(x_ref), RANK_T, n_f=DP.n_f)
        qs = [(k, rank_accuracy(DP.ctx, DP.U(x), DP.M(x), top, n_f=DP.n_f)) for k, x in keep]
        torch.cuda.synchronize()
        qs = [(k, float(q.item())) for k, q in qs]
        keep.clear()
        return qs, {lv: next((k for k, q in qs if q >= lv), None) for lv in levels}

    q_als, r_als = rank_levels(keep_als)
    q_ncg, r_ncg = rank_levels(keep_ncg)
    ta = timed(lambda: Als(DP, DP.pack(U0, M0)), lambda s: s.sweep(),
               list(k_als) + list(r_als.values()))
    tn = timed(lambda: AlsNcg(DP).init(U0, M0), lambda s: s.step(),
               list(k_ncg) + list(r_ncg.values()))
    te = timed(lambda: AlsNcg(DP, search="exact").init(U0, M0), lambda s: s.step(), k_exact)
    for name, ks, ts, tr in (("als", k_als, ta, trace), ("als_ncg", k_ncg, tn, trace_n),
                             ("als_ncg_exact_search", k_exact, te, trace_e)):
        out[name] = {"iterations_to_f_tol": ks[0], "seconds_to_f_tol": ts.get(ks[0]),
                     "iterations_to_g_tol": ks[1], "seconds_to_g_tol": ts.get(ks[1]),
                     "final_f": tr[-1][1], "final_gnorm_over_N": tr[-1][2] / N,
                     "traced_iterations": len(tr)}
    rank = {"t": RANK_T, "reference": "each algorithm's own final traced iterate",
            "kept_iterates": "ALS: sweeps 1-100, then every 10th; ALS-NCG: every iteration"}
    for name, qs, r, ts in (("als", q_als, r_als, ta), ("als_ncg", q_ncg, r_ncg, tn)):
        rank[name] = {"%.4g%%" % (100 * lv): {"iterations": r[lv], "seconds": ts.get(r[lv])}
                      for lv in levels}
        rank[name]["accuracy_at"] = {str(k): round(q, 6) for k, q in qs
                                     if k in (1, 2, 5, 10, 20, 50, 100, 200, 500, 1000)}
    rank["acceleration"] = {}
    for lv in levels:
        key = "%.4g%%" % (100 * lv)
        a, b = rank["als"][key]["seconds"], rank["als_ncg"][key]["seconds"]
        rank["acceleration"][key] = (a / b) if (a and b) else None
    out["ranking_accuracy"] = rank
    for crit in ("f_tol", "g_tol"):
        a, b = out["als"]["seconds_to_" + crit], out["als_ncg"]["seconds_to_" + crit]
        e = out["als_ncg_exact_search"]["seconds_to_" + crit]
        out["speedup_" + crit] = (a / b) if (a and b) else None
        out["speedup_exact_search_" + crit] = (a / e) if (a and e) else None
    return out


C3_NF = (64, 128)
HOLDOUT_FRAC, HOLDOUT_SEED = 0.01, 3


def load_c3_ref():
    path = os.path.join(ROOT, "tests", "golden", "c3_ml20m_holdout_ref.json")
    try:
        with open(path) as fh:
            return json.load(fh)
    except OSError:
        return None


def c3_bench(ctx, steps=20, gtol=1e-6, max_iter=400):
    """Reduced-precision form at the ML-20M shape with 1% of the ratings held
    out, n_f = 64 and 128: plain FP32, BF16 Gram with one refinement step, and
    BF16 Gram alone.  Reported per form: |f - f_FP64|/f_FP64 and the max-abs
    difference of sampled factor rows against the FP64 oracle after the same
    first iterations from the same x0, ms per ALS-NCG iteration, held-out RMSE,
    and the time to the paper's stopping rule (1/N)||g|| <= gtol."""
    import numpy as np
    import torch

    import synth
    from paper_1508_03110_amd.solver import AlsNcg, DeviceProblem
    ref = load_c3_ref()
    forms = (("fp32", dict(precision="fp")), ("bf16_refined", dict(precision="bf16", refine=True)),
             ("bf16", dict(precision="bf16", refine=False)))
    out = {"gnorm_over_N_tol": gtol, "steps": steps}
    for n_f in C3_NF:
        t0 = time.perf_counter()
        P = synth.c1_ml20m(n_f=n_f)
        Ptr, (hr, hc, hv) = synth.holdout_split(P, HOLDOUT_FRAC, HOLDOUT_SEED)
        r = (ref or {}).get("configs", {}).get(str(n_f))
        if r is not None and r.get("csr_digest") != Ptr.R.digest():
            r = None
        log("C3 n_f=%d: problem %.1f s, oracle reference %s" % (n_f, time.perf_counter() - t0,
                                                               "found" if r else "missing"))
        DP = DeviceProblem(ctx, Ptr.R, Ptr.Rt, n_f, Ptr.lam, torch.float32)
        N = n_f * (Ptr.n_u + Ptr.n_m)
        U0 = P.U0.astype(np.float32)
        M0 = P.M0.astype(np.float32)
        hv64 = hv.astype(np.float64)
        res = {"train_nnz": Ptr.nnz, "held_out": int(hv.size)}
        for name, kw in forms:
            e = {}
            s = AlsNcg(DP, **kw).init(U0, M0)
            K = len(r["als_ncg_f"]) - 1 if r else 3
            fk = []
            for _ in range(K):
                s.step()
                fk.append(DP.loss_and_gnorm(s.x)[0])
            def rmse():
                U = DP.U(s.x)[:, :n_f].cpu().numpy().astype(np.float64)
                M = DP.M(s.x)[:, :n_f].cpu().numpy().astype(np.float64)
                return float(np.sqrt(np.mean((np.einsum("ij,ij->i", U[hr], M[hc]) - hv64) ** 2)))

            e["heldout_rmse_after_%d" % K] = rmse()
            if r:
                e["rel_f_err_vs_fp64"] = [abs(a - b) / b for a, b in zip(fk, r["als_ncg_f"][1:])]
                Us = DP.U(s.x)[torch.as_tensor(r["sample_users"], device=DP.ctx.torch_device), :n_f]
                Ms = DP.M(s.x)[torch.as_tensor(r["sample_items"], device=DP.ctx.torch_device), :n_f]
                e["max_abs_factor_diff_vs_fp64"] = float(max(
                    np.abs(Us.cpu().numpy() - np.array(r["U_sample"])).max(),
                    np.abs(Ms.cpu().numpy() - np.array(r["M_sample"])).max()))
                e["compared_after_iterations"] = K
            s.enable_timing(True)
            torch.cuda.synchronize()
            t = time.perf_counter()
            for _ in range(steps):
                s.step()
            torch.cuda.synchronize()
            e["ms_per_iteration"] = (time.perf_counter() - t) / steps * 1e3
            e["phase_ms"] = {k: round(v, 4) for k, v in s.phase_ms().items()}
            e["heldout_rmse_after_%d" % (K + steps)] = rmse()
            e["f_after"] = {"iterations": K + steps, "f": DP.loss_and_gnorm(s.x)[0]}
            del s
            # time to (1/N)||g|| <= gtol from x0: traced run, then a timed run
            s = AlsNcg(DP, **kw).init(U0, M0)
            kg = None
            for k in range(1, max_iter + 1):
                s.step()
                if s.gnorm() / N <= gtol:
                    kg = k
                    break
            e["iterations_to_g_tol"] = kg
            e["final_gnorm_over_N"] = s.gnorm() / N
            del s
            if kg:
                s = AlsNcg(DP, **kw)
                torch.cuda.synchronize()
                t = time.perf_counter()
                s.init(U0, M0)
                for _ in range(kg):
                    s.step()
                torch.cuda.synchronize()
                e["seconds_to_g_tol"] = time.perf_counter() - t
                del s
            res[name] = e
            log("C3 n_f=%d %s: %s" % (n_f, name, e))
        if r:
            res["fp64_heldout_rmse_after_%d" % (len(r["als_ncg_f"]) - 1)] = r["heldout_rmse"]
        out[str(n_f)] = res
        del DP
    return out


C2_LD = 64  # row stride of the factors at the billion-rating shape (n_f = 50)


def c2_bench(ctx, steps=5, als_steps=3):
    """Billion-rating configuration: 10M users x 1M items, exactly 1e9 ratings
    (power-law user activity on [1, 50000], Zipf 1.1 items), n_f = 50,
    lambda = 0.05, generated on the device.  Plans tuned per orientation; ALS
    sweeps timed eagerly; ALS-NCG timed as replays of the captured one-iteration
    HIP graphs (device-side line-search control)."""
    import numpy as np
    import torch

    from paper_1508_03110_amd import tune
    from paper_1508_03110_amd.solver import Als, AlsNcg, DeviceCsr, DeviceProblem
    from synth import scale
    t0 = time.perf_counter()
    R, U0, M0 = scale.generate(device=ctx.torch_device, log=lambda m: log("C2 gen: " + m))
    n_f, lam = 50, 0.05
    Rd = DeviceCsr(ctx, R.indptr, R.indices, R.values, R.n_m)
    Rtd = DeviceCsr(ctx, R.indptr_t, R.indices_t, R.values_t, R.n_u)
    meta = dict(R.meta)
    del R
    # factor rows padded to 64 floats (256 bytes): every gathered row is two
    # whole 128-byte cache lines instead of straddling three more than half
    # of the time at a 200-byte stride
    DP = DeviceProblem(ctx, Rd, Rtd, n_f, lam, torch.float32, ld=C2_LD)
    x0 = DP.pack(U0, M0)
    del U0, M0
    out = {"workload": "10M x 1M, 1e9 ratings, n_f=50", "n_u": DP.n_u, "n_m": DP.n_m,
           "nnz": DP.R.nnz, "n_f": n_f, "ld": C2_LD, "lambda": lam, "generator": meta,
           "setup_seconds": round(time.perf_counter() - t0, 1)}
    log("C2 problem on device (%.1f s); plans R %s R^T %s" % (time.perf_counter() - t0, DP.R.info(), DP.Rt.info()))
    out["tuning"] = tune.tune(DP, x0, log=log)
    out["plans"] = {"R": DP.R.info(), "Rt": DP.Rt.info()}
    # ALS (Algorithm 1), eager
    als = Als(DP, x0.clone())
    als.sweep()
    torch.cuda.synchronize()
    t = time.perf_counter()
    for _ in range(als_steps):
        als.sweep()
    torch.cuda.synchronize()
    ms_als = (time.perf_counter() - t) / als_steps * 1e3
    out["als"] = {"ms_per_sweep": ms_als, "ratings_per_s": 2.0 * DP.R.nnz / (ms_als * 1e-3)}
    del als
    torch.cuda.empty_cache()
    # ALS-NCG: one eager device-controlled step with phase events, then graphs
    x0_U = x0[: DP.n_u * DP.ld].view(DP.n_u, DP.ld)[:, :n_f]
    x0_M = x0[DP.n_u * DP.ld:].view(DP.n_m, DP.ld)[:, :n_f]
    s = AlsNcg(DP).init(x0_U, x0_M)
    s.enable_timing(True)
    s.step_device()
    phases = s.phase_ms()
    s.enable_timing(False)
    s.capture()
    s.replay()
    torch.cuda.synchronize()
    t = time.perf_counter()
    for _ in range(steps):
        s.replay()
    torch.cuda.synchronize()
    ms_ncg = (time.perf_counter() - t) / steps * 1e3
    s.read_state()
    out["als_ncg"] = {"ms_per_iteration": ms_ncg, "ratings_per_s": 2.0 * DP.R.nnz / (ms_ncg * 1e-3),
                      "graph_replays": steps, "phase_ms_eager_step": {k: round(v, 3) for k, v in phases.items()},
                      "f": s.f, "gnorm_over_N": s.gnorm() / (n_f * (DP.n_u + DP.n_m)),
                      "restarts": s.restarts, "safeguards": s.safeguards, "iterations": s.k}
    counts_u = (DP.R.indptr[1:] - DP.R.indptr[:-1]).cpu().numpy()
    fU = sweep_flops_binned(counts_u, n_f, out["tuning"]["U"]["best"]["dual_max"])
    del counts_u
    out["sweep_U_tflops_eager"] = fU / (phases["sweep_U"] * 1e-3) / 1e12
    out["sweep_U_tflops_eager_eq3_count"] = (sweep_flops(DP.R.nnz, DP.n_u, n_f)
                                             / (phases["sweep_U"] * 1e-3) / 1e12)
    log("C2:", out["als"], out["als_ncg"])
    del s
    out["speedup_vs_gnorm"] = c2_speedup_curve(DP, x0_U, x0_M, ms_als, ms_ncg, log=log)
    del DP, Rd, Rtd, x0, x0_U, x0_M
    torch.cuda.empty_cache()
    return out


def speedup_vs_gnorm(g_ncg, g_als, ms_als, ms_ncg):
    """The speedup curve of Section VI (Fig. 6) from two gradient-norm traces.

    g_ncg[k-1], g_als[j-1]: (1/N)||g|| after ALS-NCG iteration k and ALS
    iteration j.  For each ALS-NCG iteration k >= 2 the level is the mean of
    the norms after iterations k-1 and k (a two-iteration moving average, which
    smooths the non-monotone NCG trace); j is the first ALS iteration whose
    norm is at or below that level, and the speedup is the time of j ALS
    iterations over the time of k ALS-NCG iterations, j ms_als / (k ms_ncg).
    When ALS never gets there within its trace, speedup is None and
    speedup_at_least = len(g_als) ms_als / (k ms_ncg), a lower bound."""
    n_als = len(g_als)
    rows = []
    for k in range(2, len(g_ncg) + 1):
        level = 0.5 * (g_ncg[k - 1] + g_ncg[k - 2])
        j = next((i + 1 for i, g in enumerate(g_als) if g <= level), None)
        rows.append({"ncg_iteration": k, "gnorm_over_N": level, "als_iterations": j,
                     "speedup": (j * ms_als) / (k * ms_ncg) if j else None,
                     "speedup_at_least": None if j else (n_als * ms_als) / (k * ms_ncg)})
    return rows


def c2_speedup_curve(DP, U0, M0, ms_als, ms_ncg, n_ncg=25, n_als=100, log=None):
    """Speedup of ALS-NCG over ALS as a function of the normalised gradient
    norm, by the paper's method (Section VI, Fig. 6): for each ALS-NCG
    iteration k the moving average of (1/N)||g|| over iterations k-1, k is
    taken, the number j of ALS iterations needed to reach an equal or lower
    (1/N)||g|| is looked up, and the times j t_ALS and k t_NCG are compared,
    with the measured average times per iteration."""
    import torch

    from paper_1508_03110_amd.solver import Als, AlsNcg
    N = DP.n_f * (DP.n_u + DP.n_m)
    t0 = time.perf_counter()
    ncg = AlsNcg(DP).init(U0, M0)
    g_ncg = []
    for _ in range(n_ncg):
        ncg.step_device()
        g_ncg.append(ncg.gnorm() / N)
    del ncg
    torch.cuda.empty_cache()
    als = Als(DP, DP.pack(U0, M0))
    g_als = []
    for _ in range(n_als):
        als.sweep()
        g_als.append(DP.loss_and_gnorm(als.x)[1] / N)
    del als
    rows = speedup_vs_gnorm(g_ncg, g_als, ms_als, ms_ncg)
    if log:
        log("C2 speedup curve (%.1f s):" % (time.perf_counter() - t0),
            [(r["ncg_iteration"], "%.2e" % r["gnorm_over_N"], r["als_iterations"],
              round(r["speedup"], 2) if r["speedup"] else ">%.2f" % r["speedup_at_least"])
             for r in rows[::3]])
    return {"method": "paper Section VI: 2-iteration moving average of the ALS-NCG gradient norm, "
                      "ALS iterations to reach it, times from the measured ms per iteration",
            "ms_per_als_iteration": ms_als, "ms_per_ncg_iteration": ms_ncg,
            "als_gnorm_over_N": g_als, "ncg_gnorm_over_N": g_ncg, "curve": rows}


def serve_bench(ctx, M_dev, P, rates=(10_000, 50_000, 200_000), duration=2.0, warm=0.5,
                baseline_cap=20_000, seed=4):
    """Fold-in serving: open-loop Poisson arrivals replayed in real time by the
    native server; latency = result visible on the host - arrival."""
    import numpy as np

    import synth
    from paper_1508_03110_amd.solver import FoldInServer
    t0 = time.perf_counter()
    pool = synth.fold_in_requests(16384, P.n_m, seed=seed, item_perm=P.meta["item_perm"],
                                  M_star=P.meta["M_star"])
    log("request pool: %d requests, %d ratings, mean %.1f (%.1f s)"
        % (pool.n_rows, pool.nnz, pool.nnz / pool.n_rows, time.perf_counter() - t0))
    rng = np.random.default_rng(seed + 1)
    configs = {"continuous_batching": dict(max_inflight=4, max_batch=4096, split=256),
               "one_request_per_launch": dict(max_inflight=1, max_batch=1, split=0)}
    out = {"pool_requests": pool.n_rows, "mean_ratings": pool.nnz / pool.n_rows,
           "duration_s": duration, "warmup_s": warm, "hbm_budget_bytes": 16 << 30}
    for name, cfg in configs.items():
        srv = FoldInServer(ctx, M_dev, P.lam, P.n_f, budget_bytes=16 << 30, **cfg)
        res = {}
        for rate in rates:
            n = int(rate * (duration + warm))
            if name == "one_request_per_launch":
                n = min(n, baseline_cap)
            arrival = np.cumsum(rng.exponential(1e9 / rate, size=n)).astype(np.int64)
            rows = rng.integers(0, pool.n_rows, size=n).astype(np.int32)
            comp, st, _ = srv.replay(arrival, rows, pool)
            keep = arrival >= (warm * 1e9 if n * 1e9 / rate > 2 * warm * 1e9 else 0)
            lat = (comp - arrival)[keep] / 1e6
            span = (comp[keep].max() - arrival[keep].min()) / 1e9
            res[str(rate)] = {"requests": int(keep.sum()), "p50_ms": float(np.percentile(lat, 50)),
                              "p99_ms": float(np.percentile(lat, 99)),
                              "solves_per_s": float(keep.sum() / max(span, 1e-9)),
                              "errors": int((st != 0).sum())}
            log("serve %s @%d req/s: %s" % (name, rate, res[str(rate)]))
        srv.close()
        out[name] = {"config": cfg, "rates": res}
    return out


def _r(x, d=4):
    """Round to d significant digits (None stays None)."""
    if x is None or isinstance(x, (bool, int)):
        return x
    return float("%.*g" % (d, x))


def compact(res, full_path):
    """The one-line result: the headline keys plus a one-number summary of
    every leg (the traces, curves and per-trial lists stay in the full file)."""
    keep = ("metric", "value", "unit", "n_gpus", "steps", "warmup", "ms_per_step",
            "higher_is_better", "scaling", "vs_baseline", "dtype", "data", "config", "roofline",
            "cpu_baseline")
    out = {k: res[k] for k in keep if k in res}
    out["value"] = _r(out["value"], 6)
    out["ms_per_step"] = _r(out["ms_per_step"], 6)
    rl = dict(out["roofline"])
    out["roofline"] = {k: rl[k] for k in ("bound", "achieved", "peak", "unit", "frac", "traffic",
                                          "kernel", "flops_per_launch", "launch_ms",
                                          "algorithmic_bytes", "frac_eq3_count") if k in rl}
    if "cpu_baseline" in out:
        cb = out["cpu_baseline"]
        out["cpu_baseline"] = dict(cb, value=_r(cb["value"]),
                                   half_sweep_ratings_per_s={k: _r(v) for k, v in
                                                             cb["half_sweep_ratings_per_s"].items()})
    out["half_sweep_ratings_per_s"] = {k: _r(v) for k, v in res["half_sweep_ratings_per_s"].items()}
    out["phase_ms"] = {k: _r(v) for k, v in res["phase_ms"].items()}
    out["pass_hbm_gbs"] = {k: _r(v) for k, v in res["pass_hbm_gbs"].items()}
    out["f"] = _r(res["f"], 12)
    if "length_bins" in res:
        out["dual_max"] = {k: v["dual_max"] for k, v in res["length_bins"].items()}
    if "grad_slices" in res:
        out["grad_slices"] = res["grad_slices"]["best"]["slices"]
    if "split_copy" in res:
        out["split_copy"] = res["split_copy"]
    tt = res.get("time_to_tol")
    if tt:
        sm = {"f_gap_tol": tt["f_gap_tol"], "gnorm_over_N_tol": tt["gnorm_over_N_tol"]}
        for name in ("als", "als_ncg", "als_ncg_exact_search"):
            e = tt[name]
            sm[name] = [e["iterations_to_f_tol"], _r(e["seconds_to_f_tol"]),
                        e["iterations_to_g_tol"], _r(e["seconds_to_g_tol"])]
        sm["columns"] = "iterations to f-gap, s, iterations to (1/N)||g||, s"
        for k in ("speedup_f_tol", "speedup_g_tol", "speedup_exact_search_f_tol",
                  "speedup_exact_search_g_tol"):
            sm[k] = _r(tt.get(k))
        ra = tt.get("ranking_accuracy")
        if ra:
            sm["ranking_top20_acceleration"] = {k: _r(v, 3) for k, v in ra["acceleration"].items()}
        out["time_to_tol"] = sm
    rs = res.get("ranking_accuracy_small")
    if rs:
        out["ranking_600x400_acceleration"] = {k: _r(v, 3) for k, v in rs["acceleration"].items()}
    rk = res.get("ranking_kernels")
    if rk:
        out["ranking_kernels_ms"] = {"top_t": rk["top_t_ms"], "accuracy": rk["accuracy_ms"]}
    fi = res.get("fold_in")
    if fi:
        out["fold_in_p99_ms"] = {r: _r(v["p99_ms"], 3)
                                 for r, v in fi["continuous_batching"]["rates"].items()}
        out["fold_in_p50_ms"] = {r: _r(v["p50_ms"], 3)
                                 for r, v in fi["continuous_batching"]["rates"].items()}
        out["fold_in_solves_per_s"] = {r: _r(v["solves_per_s"], 3)
                                       for r, v in fi["continuous_batching"]["rates"].items()}
        out["fold_in_baseline_p99_ms"] = {r: _r(v["p99_ms"], 3) for r, v in
                                          fi["one_request_per_launch"]["rates"].items()}
    c3 = res.get("reduced_precision")
    if c3:
        sm = {}
        for nf in C3_NF:
            d = c3.get(str(nf), {})
            for form in ("fp32", "bf16_refined", "bf16"):
                e = d.get(form)
                if not e:
                    continue
                err = e.get("rel_f_err_vs_fp64")
                sm["%s_nf%d" % (form, nf)] = {
                    "ms_per_it": _r(e["ms_per_iteration"]),
                    "rel_f_err": _r(err[-1], 3) if err else None,
                    "max_abs_dU": _r(e.get("max_abs_factor_diff_vs_fp64"), 3),
                    "rmse": _r(next((v for k, v in e.items() if k.startswith("heldout_rmse_after")
                                     and k != "heldout_rmse_after_%d" % e.get(
                                         "compared_after_iterations", -1)), None)),
                    "s_to_g_tol": _r(e.get("seconds_to_g_tol"))}
        out["reduced_precision"] = sm
    c2 = res.get("scale_1e9")
    if c2:
        out["scale_1e9"] = {"als_ms_per_sweep": _r(c2["als"]["ms_per_sweep"]),
                            "als_ncg_ms_per_iteration": _r(c2["als_ncg"]["ms_per_iteration"]),
                            "als_ncg_ratings_per_s": _r(c2["als_ncg"]["ratings_per_s"]),
                            "sweep_U_tflops": _r(c2["sweep_U_tflops_eager"]),
                            "dual_max": {k: v["best"].get("dual_max") for k, v in
                                         c2.get("tuning", {}).items()},
                            "split_copy": {k: v["best"].get("split_copy") for k, v in
                                           c2.get("tuning", {}).items()},
                            "grad_slices": c2.get("tuning", {}).get("M", {}).get("best", {})
                                             .get("grad_slices"),
                            "phase_ms": {k: _r(v) for k, v in
                                         c2["als_ncg"]["phase_ms_eager_step"].items()}}
        curve = c2.get("speedup_vs_gnorm", {}).get("curve", [])
        if curve:
            out["scale_1e9"]["speedup_vs_gnorm"] = [
                [_r(r["gnorm_over_N"], 3), _r(r["speedup"], 3) if r["speedup"] else
                 ">%s" % _r(r["speedup_at_least"], 3)] for r in curve[::4]]
    out["full_results"] = os.path.relpath(full_path, ROOT) if full_path else None
    return out


def gather_probe(reps=10):
    """How much of each gather-bound phase is the gathers' trip beyond L2:
    the coefficient pass, the M-block gradient and both half-sweeps (length
    bound 78 and the split copy for users) at the 20M-rating shape, timed with the real rating
    ids and with every id folded into [0, 64) (same work and access count,
    every gathered row an L2 hit; the results of the folded runs are not
    used), and the M-block gradient with the real ids over a plan cut at 8
    column slices.  Best of 3 rounds of `reps` launches (HIP events)."""
    import numpy as np
    import torch

    import synth
    from paper_1508_03110_amd.solver import Context, DeviceProblem

    def t_ms(fn):
        fn()
        torch.cuda.synchronize()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        best = float("inf")
        for _ in range(3):
            a.record()
            for _ in range(reps):
                fn()
            b.record()
            torch.cuda.synchronize()
            best = min(best, a.elapsed_time(b) / reps)
        return round(best, 4)

    P = synth.c1_ml20m()
    ctx = Context(0)
    out = {"workload": "20M-rating shape, n_f=100, FP32, user bound 78, user split copy", "reps": reps}
    for mode in ("real_ids", "ids_folded_into_64_rows"):
        R, Rt = P.R, P.Rt
        if mode != "real_ids":
            R = synth.Csr(R.n_rows, R.n_cols, R.indptr, (R.indices % 64).astype(np.int32), R.values)
            Rt = synth.Csr(Rt.n_rows, Rt.n_cols, Rt.indptr, (Rt.indices % 64).astype(np.int32),
                           Rt.values)
        DP = DeviceProblem(ctx, R, Rt, P.n_f, P.lam, torch.float32)
        DP.R.set_dual(78)
        DP.R.set_split_copy(1)
        x = DP.pack(P.U0.astype(np.float32), P.M0.astype(np.float32))
        p = torch.empty_like(x).normal_(0.0, 0.01)
        g = DP.zeros()
        C = torch.zeros(5, dtype=torch.float64, device=x.device)
        X = torch.empty((P.n_u, DP.ld), dtype=torch.float32, device=x.device)
        Mo = torch.empty((P.n_m, DP.ld), dtype=torch.float32, device=x.device)
        out[mode] = {
            "coefficients_ms": t_ms(lambda: DP.coeffs(DP.U(x), DP.M(x), DP.U(p), DP.M(p), C)),
            "gradient_M_ms": t_ms(lambda: DP.gradient(DP.U(x), DP.M(x), None, DP.M(g), None)),
            "sweep_U_ms": t_ms(lambda: DP.sweep("U", DP.M(x), X, X_at=DP.U(x), grad_out=DP.U(g))),
            "sweep_M_ms": t_ms(lambda: DP.sweep("M", DP.U(x), Mo)),
        }
        if mode == "real_ids":  # the gradient over a plan cut at 8 column slices
            DP.Rt.set_grad_slices(8)
            out[mode]["gradient_M_8_slices_ms"] = t_ms(
                lambda: DP.gradient(DP.U(x), DP.M(x), None, DP.M(g), None))
            DP.Rt.set_grad_slices(0)
        log("gather probe", mode, out[mode])
        del DP, x, p, g, X, Mo
        torch.cuda.empty_cache()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-serve", action="store_true", help="skip the fold-in serving measurement")
    ap.add_argument("--no-ttt", action="store_true", help="skip the time-to-f-tolerance measurement")
    ap.add_argument("--no-c3", action="store_true", help="skip the reduced-precision measurement")
    ap.add_argument("--no-c2", action="store_true", help="skip the billion-rating measurement")
    ap.add_argument("--serve-seconds", type=float, default=10.0,
                    help="measured seconds per arrival rate (after --serve-warmup)")
    ap.add_argument("--serve-warmup", type=float, default=1.0)
    ap.add_argument("--full-json", default=os.path.join(ROOT, "gpurun_out", "bench_full.json"),
                    help="where every leg's detailed results are written")
    ap.add_argument("--dual", default=None, metavar="U,M",
                    help="fix the dual-form length bounds of the user and item plans instead of "
                         "timing the candidates (profiling runs)")
    ap.add_argument("--split-copy", default=None, metavar="U,M",
                    help="fix whether the user and item half-sweeps gather a split copy of the "
                         "fixed side (1/0) instead of timing both")
    ap.add_argument("--grad-slices", type=int, default=None, metavar="S",
                    help="fix the column slices of the M-block gradient's plan (0: none) "
                         "instead of timing the candidates")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="run only a plain 1 GiB device copy (reference for HBM traffic counters)")
    ap.add_argument("--gather-probe", action="store_true",
                    help="run only the gather probe: the 20M-rating shape's passes with the real "
                         "rating ids and with the ids folded into 64 rows (every gather an L2 hit)")
    args = ap.parse_args()
    if args.gather_probe:
        print(json.dumps(gather_probe()))
        return
    if args.calibrate_copy:
        import torch
        a = torch.empty(1 << 28, dtype=torch.float32, device="cuda").fill_(1.0)
        b = torch.empty_like(a)
        for _ in range(5):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": a.numel() * 4, "copy_bytes_written": b.numel() * 4,
                          "launches": 5}))
        return
    if args.gpus != 1:
        print("bench.py measures one GPU: there is no multi-GPU path (how the path would shard "
              "is written up with the design notes); run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import synth
    from paper_1508_03110_amd.solver import AlsNcg, Context, DeviceProblem

    t0 = time.perf_counter()
    P = synth.c1_ml20m()
    log("generated %s: %d x %d, nnz=%d in %.1f s" % (P.name, P.n_u, P.n_m, P.nnz, time.perf_counter() - t0))
    ctx = Context(0)
    DP = DeviceProblem(ctx, P.R, P.Rt, P.n_f, P.lam, torch.float32)
    infoR, infoRt = DP.R.info(), DP.Rt.info()
    log("plans: R", infoR, "R^T", infoRt)
    U0 = P.U0.astype(np.float32)
    M0 = P.M0.astype(np.float32)
    # length bins of the half-sweeps: the dual-form bound of each plan, by timing
    from paper_1508_03110_amd import tune
    x_t = DP.pack(U0, M0)
    bins = {}
    fixed = [int(v) for v in args.dual.split(",")] if args.dual else None
    for k, (side, Y, n) in enumerate((("U", DP.M(x_t), P.n_u), ("M", DP.U(x_t), P.n_m))):
        X_t = torch.empty((n, DP.ld), dtype=torch.float32, device=ctx.torch_device)
        cands = (fixed[k],) if fixed else tune.DUAL_CANDIDATES
        smodes = (int(args.split_copy.split(",")[k]),) if args.split_copy is not None else None
        bins[side] = tune.tune_dual(DP, side, Y, X_t, candidates=cands, split_modes=smodes)
        log("length bins and split copy %s: %s" % (side, bins[side]))
        del X_t
    # the M-block gradient's plan: cut at column slices of the user rows or not
    X_t = torch.empty((P.n_m, DP.ld), dtype=torch.float32, device=ctx.torch_device)
    gcands = (args.grad_slices,) if args.grad_slices is not None else tune.GRAD_SLICE_CANDIDATES
    gslices = tune.tune_grad_slices(DP, DP.U(x_t), DP.M(x_t), X_t, candidates=gcands)
    log("gradient column slices: %s" % gslices)
    del X_t
    del x_t
    # Every decision of an iteration (line search, restart, safeguard) is
    # taken on the device, so the iterations are queued back to back with no
    # host read in between; f and the step counters are read once at the end.
    solver = AlsNcg(DP).init(U0, M0)
    for _ in range(args.warmup):
        solver.step_device()
    solver.read_state()
    log("warmup done: f=%.10g alpha=%s trials=%d" % (solver.f, solver.alpha, solver.n_trials))

    solver.enable_timing(True)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for k in range(args.steps):
        solver.step_device()
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    elapsed = t2 - t1
    ms_step = elapsed / args.steps * 1e3
    phases = solver.phase_ms()
    solver.read_state()
    log("timed %d steps: %.3f ms/step, phases %s, f=%.10g" % (args.steps, ms_step, phases, solver.f))

    # the work of the binned half-sweeps as executed (dual-form rows counted
    # with their own, smaller, algorithmic work), and the Eq. (3) count
    fU3 = sweep_flops(P.nnz, P.n_u, P.n_f)
    fU = sweep_flops_binned(P.R.counts(), P.n_f, bins["U"]["best"]["dual_max"])
    fM = sweep_flops_binned(P.Rt.counts(), P.n_f, bins["M"]["best"]["dual_max"])
    tU = phases["sweep_U"] * 1e-3
    tM = phases["sweep_M"] * 1e-3
    achieved = fU / tU / 1e12
    roofline = {"bound": "mfma",
                "kernel": "U half-sweep: sweep_chunks_kernel<float,7> + sweep_dual_kernel bins",
                "achieved": round(achieved, 3), "peak": PEAK_FP32_TFLOPS, "unit": "TFLOP/s",
                "frac": round(achieved / PEAK_FP32_TFLOPS, 4),
                "traffic": profiled_traffic(bins["U"]["best"]["dual_max"], bins["U"]["best"]["split_copy"]),
                "flops_per_launch": fU, "launch_ms": round(phases["sweep_U"], 4),
                "eq3_flops_per_launch": fU3,
                "frac_eq3_count": round(fU3 / tU / 1e12 / PEAK_FP32_TFLOPS, 4),
                # ratings (id + value), row offsets, M read once, U written, X_at read,
                # U block of the gradient written
                "algorithmic_bytes": P.nnz * 8 + (P.n_u + 1) * 8 + P.n_m * P.n_f * 4
                                     + 3 * P.n_u * P.n_f * 4}
    # streaming passes: algorithmic bytes (index+value per rating, factor rows read once, output)
    by_coef = P.nnz * 8 + (P.n_u + P.n_m) * P.n_f * 4 * 2 + (P.n_u + 1 + P.n_m + 1) * 8
    by_grad = P.nnz * 8 + (P.n_u + P.n_m) * P.n_f * 4 + P.n_m * P.n_f * 4 + (P.n_m + 1) * 8
    result = {
        "metric": METRIC,
        "value": 2.0 * P.nnz * args.steps / elapsed,
        "unit": "ratings/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "ALS-NCG iteration, MovieLens-20M-shaped synthetic ratings",
                   "n_u": P.n_u, "n_m": P.n_m, "nnz": P.nnz, "n_f": P.n_f, "lambda": P.lam,
                   "value_def": "2*nnz half-sweep ratings per ALS-NCG iteration / iteration time"},
        "half_sweep_ratings_per_s": {"U": P.nnz / tU, "M": P.nnz / tM},
        "phase_ms": {k: round(v, 4) for k, v in phases.items()},
        "sweep_tflops": {"U": fU / tU / 1e12, "M": fM / tM / 1e12},
        "pass_hbm_gbs": {"linesearch": by_coef / (phases["linesearch"] * 1e-3) / 1e9,
                         "gradient_M": by_grad / (phases["gradient_M"] * 1e-3) / 1e9},
        "roofline": roofline,
        "length_bins": {k: v["best"] for k, v in bins.items()},
        "length_bin_trials": {k: v["trials"] for k, v in bins.items()},
        "grad_slices": gslices,
        "split_copy": {k: v["best"]["split_copy"] for k, v in bins.items()},
        "f": solver.f,
        "restarts": solver.restarts,
        "safeguards": solver.safeguards,
        "gnorm_over_N": solver.gnorm() / (P.n_f * (P.n_u + P.n_m)),
    }
    result["ranking_kernels"] = ranking_kernels(DP, solver.x)
    log("ranking kernels:", result["ranking_kernels"])
    fs = load_fstar()
    if not args.no_ttt and fs is not None and fs.get("problem", {}).get("csr_digest") == P.R.digest():
        ttt = time_to_tol(DP, P, fs["f_star"])
        ttt["f_star_source"] = {"iterations": fs["iterations"], "converged": fs["converged"],
                                "rel_change_last_10": fs["rel_change_last_10"]}
        result["time_to_tol"] = ttt
        log("time to tolerance:", ttt)
    if not args.no_ttt:
        result["ranking_accuracy_small"] = ranking_small(ctx)
        log("ranking accuracy, 600 x 400:", result["ranking_accuracy_small"])
    if not args.no_serve:
        M_dev = DP.M(solver.x)[:, : P.n_f].contiguous()
        result["fold_in"] = serve_bench(ctx, M_dev, P, duration=args.serve_seconds,
                                        warm=args.serve_warmup)
        p99 = {r: v["p99_ms"] for r, v in result["fold_in"]["continuous_batching"]["rates"].items()}
        result["fold_in_p99_ms"] = p99
    if not args.no_c3:
        del solver, DP
        torch.cuda.empty_cache()
        result["reduced_precision"] = c3_bench(ctx)
    if not args.no_c2:
        if args.no_c3:
            del solver, DP
            torch.cuda.empty_cache()
        result["scale_1e9"] = c2_bench(ctx)
    ctx.close()
    if not args.no_cpu_baseline:
        log("cpu baseline ...")
        result["cpu_baseline"] = cpu_baseline(P)
    full = args.full_json
    try:
        os.makedirs(os.path.dirname(os.path.abspath(full)), exist_ok=True)
        with open(full, "w") as fh:
            json.dump(result, fh, indent=1)
        log("full results written to", full)
    except OSError as e:
        log("could not write %s: %s" % (full, e))
        full = None
    line = json.dumps(compact(result, full), separators=(",", ":"))
    print(line, flush=True)


if __name__ == "__main__":
    main()
