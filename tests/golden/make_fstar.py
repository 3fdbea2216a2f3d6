"""Reference minimum f* of Eq. (1) for the MovieLens-20M-shaped synthetic problem.

Writes tests/golden/fstar_ml20m_shape.json from the FP64 oracle only (calls
oracle/ and synth/, nothing else): ALS-NCG (Algorithm 2 with the backtracking
line search of Section V-C) from the shared starting point x0 (the seeded
U0, M0 rounded to FP32, the same point the FP32 GPU runs start from), run
until f changes by less than `--rtol` relative over 10 iterations or
`--max-iter` iterations.  f* is the smallest f seen.  The JSON is rewritten
every 5 iterations with the current estimate and its convergence status;
with --ckpt FILE the state is also saved there every 5 iterations and a run
resumes from it.

Usage: python tests/golden/make_fstar.py [--threads 5] [--max-iter 600] [--ckpt FILE]
"""
import argparse
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import synth  # noqa: E402

OUT = os.path.join(HERE, "fstar_ml20m_shape.json")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--threads", type=int, default=0)
    ap.add_argument("--max-iter", type=int, default=600)
    ap.add_argument("--rtol", type=float, default=1e-13)
    ap.add_argument("--ckpt", default=None,
                    help="checkpoint file (.npz) to write every 5 iterations and resume from; "
                         "none by default")
    args = ap.parse_args()
    threads = oracle.set_threads(args.threads)
    P = synth.c1_ml20m()
    U0 = P.U0.astype(np.float32).astype(np.float64)
    M0 = P.M0.astype(np.float32).astype(np.float64)
    o = oracle.NcgOracle(P.R, P.Rt, P.n_f, P.lam)
    fs = []
    if args.ckpt and os.path.exists(args.ckpt):
        z = np.load(args.ckpt)
        s = oracle.NcgState(x=z["x"], p=z["p"], g=z["g"], gbar=z["gbar"], xbar=z["xbar"],
                            k=int(z["k"]), restarts=int(z["restarts"]), safeguards=int(z["safeguards"]))
        fs = list(z["fs"])
        print("resumed at iteration", s.k, flush=True)
    else:
        s = o.init(U0, M0)
        fs = [o.f(s.x)]
    t0 = time.time()
    converged = False
    while s.k < args.max_iter:
        o.step(s)
        fs.append(s.f if np.isfinite(s.f) else o.f(s.x))
        if len(fs) > 11:
            recent = fs[-11:]
            if (max(recent) - min(recent)) <= args.rtol * abs(min(recent)):
                converged = True
        print("iter %d f=%.15g alpha=%s trials=%d restarts=%d safeguards=%d (%.1fs)"
              % (s.k, fs[-1], s.alpha, s.trials, s.restarts, s.safeguards, time.time() - t0), flush=True)
        if s.k % 5 == 0 or converged or s.k >= args.max_iter:
            if args.ckpt:
                os.makedirs(os.path.dirname(os.path.abspath(args.ckpt)), exist_ok=True)
                np.savez(args.ckpt + ".tmp.npz", x=s.x, p=s.p, g=s.g, gbar=s.gbar, xbar=s.xbar,
                         k=s.k, restarts=s.restarts, safeguards=s.safeguards, fs=np.array(fs))
                os.replace(args.ckpt + ".tmp.npz", args.ckpt)
            last10 = fs[-11:]
            rel = (max(last10) - min(last10)) / abs(min(last10)) if len(last10) > 1 else float("nan")
            with open(OUT + ".tmp", "w") as fh:
                json.dump({
                    "citation": "minimum of the loss of Eq. (1) reached by ALS-NCG (Algorithm 2, "
                                "Section III-B; line search of Section V-C) in FP64",
                    "written_by": "tests/golden/make_fstar.py (FP64 oracle only)",
                    "problem": {"name": P.name, "seed": P.seed, "n_u": P.n_u, "n_m": P.n_m,
                                "nnz": P.nnz, "n_f": P.n_f, "lambda": P.lam,
                                "csr_digest": P.R.digest(), "x0": "seeded U0, M0 rounded to FP32"},
                    "f_star": float(min(fs)),
                    "iterations": int(s.k),
                    "converged": bool(converged),
                    "rel_change_last_10": rel,
                    "restarts": int(s.restarts), "safeguards": int(s.safeguards),
                    "threads": threads,
                    "f_trajectory": [float(v) for v in fs],
                }, fh, indent=1)
            os.replace(OUT + ".tmp", OUT)
        if converged:
            break
    print("done: f* = %.15g after %d iterations (converged=%s)" % (min(fs), s.k, converged))


if __name__ == "__main__":
    main()
